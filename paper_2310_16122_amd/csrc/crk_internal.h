// Internal declarations shared by the forward and backward translation units
// of the CRK library (not part of the public ABI).
#pragma once

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <string>
#include <vector>

#include "crk.h"

namespace crk {

constexpr int kWave = 64;
constexpr double kPi = 3.14159265358979323846;
constexpr double kInvGrid = 2.3283064365386962890625e-10;  // 2^-32
constexpr float kCullMargin = 1.0f + 1.0e-5f;                // list radius^2 factor

// Records a message for crk_last_error and returns `code`.
int fail(int code, const char* fmt, ...);

}  // namespace crk

#define HIP_TRY(expr)                                                                  \
    do {                                                                               \
        hipError_t e_ = (expr);                                                        \
        if (e_ != hipSuccess) return fail(CRK_EHIP, "%s: %s", #expr, hipGetErrorString(e_)); \
    } while (0)

#define LAUNCH_CHECK(name)                                                             \
    do {                                                                               \
        hipError_t e_ = hipGetLastError();                                             \
        if (e_ != hipSuccess) return fail(CRK_EHIP, "launch %s: %s", name, hipGetErrorString(e_)); \
    } while (0)


namespace crk {
namespace {

// ------------------------------------------------------------------ device helpers

template <class R> __device__ __forceinline__ R sep(uint32_t a, uint32_t b) {
    return R(int32_t(a - b)) * R(kInvGrid);
}

template <class R> __device__ __forceinline__ R dsqrt(R x);
template <> __device__ __forceinline__ float dsqrt<float>(float x) { return __builtin_amdgcn_sqrtf(x); }
template <> __device__ __forceinline__ double dsqrt<double>(double x) { return sqrt(x); }

template <class R> __device__ __forceinline__ R drsqrt(R x);
template <> __device__ __forceinline__ float drsqrt<float>(float x) { return __builtin_amdgcn_rsqf(x); }
template <> __device__ __forceinline__ double drsqrt<double>(double x) { return 1.0 / sqrt(x); }

// Wendland C4 shape with support H: W = cW w(q), grad_i W = cF f(q) x_ij,
// cW = 495/(32 pi H^3), cF = -1155/(4 pi H^5), q = r/H; zero for q >= 1.
template <class R> __device__ __forceinline__ void wendland(R q, R& w, R& f) {
    const R t = fmax(R(1) - q, R(0));
    const R t2 = t * t;
    const R t4 = t2 * t2;
    const R t5 = t4 * t;
    const R t6 = t5 * t;
    w = t6 * (R(1) + q * (R(6) + q * R(35.0 / 3.0)));
    f = t5 * (R(1) + R(5) * q);
}

template <class R> __host__ __device__ __forceinline__ R norm_W(R H) {
    return R(495.0 / (32.0 * kPi)) / (H * H * H);
}
template <class R> __host__ __device__ __forceinline__ R norm_F(R H) {
    return R(-1155.0 / (4.0 * kPi)) / (H * H * H * H * H);
}

// compensated accumulation: the sum is s - c
template <class R> __device__ __forceinline__ void kadd(R& s, R& c, R t) {
    const R y = t - c;
    const R u = s + y;
    c = (u - s) - y;
    s = u;
}

__device__ __forceinline__ int lane_id() { return threadIdx.x & (kWave - 1); }

// Work queue: tiles in decreasing-cost order, one per wave or pulled from an
// atomic counter by a persistent grid.
struct Queue {
    const int32_t* order;
    int32_t* counter;
    int32_t n_items;
    int32_t persistent;
};

__device__ __forceinline__ int first_item(const Queue& q, int wave_global) {
    if (!q.persistent) return wave_global;
    int it = 0;
    if (lane_id() == 0) it = atomicAdd(q.counter, 1);
    return __builtin_amdgcn_readfirstlane(it);
}
__device__ __forceinline__ int next_item(const Queue& q, int cur, int n_waves_grid) {
    if (!q.persistent) return q.n_items;  // one tile per wave
    int it = 0;
    if (lane_id() == 0) it = atomicAdd(q.counter, 1);
    return __builtin_amdgcn_readfirstlane(it);
}

__global__ void k_reset(int32_t* c) {
    if (threadIdx.x < 4) c[threadIdx.x] = 0;
}

// ------------------------------------------------------------------ packing (tree order)

__device__ __forceinline__ uint32_t quantize(double x) {
    double t = x - floor(x);
    double v = floor(t * 4294967296.0 + 0.5);
    return v >= 4294967296.0 ? 0u : uint32_t(v);
}

// positions to fixed point (+ support radius bits for the list build)
template <class R>
__global__ void k_pack_quant(int n, const int32_t* perm, const double* x, const double* y,
                             const double* z, const R* h, uint4* quant) {
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= n) return;
    const int i = perm[s];
    uint4 q;
    q.x = quantize(x[i]);
    q.y = quantize(y[i]);
    q.z = quantize(z[i]);
    q.w = h ? __float_as_uint(float(2.0 * double(h[i]))) : 0u;
    quant[s] = q;
}

template <class R> __global__ void k_gather(int n, const int32_t* perm, const R* src, R* dst) {
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s < n) dst[s] = src[perm[s]];
}

// ------------------------------------------------------------------ list access

struct Lists {
    const int32_t* cnt;
    const int64_t* off;
    const int32_t* len;
    const uint32_t* nbr;
};


}  // namespace
}  // namespace crk

// ====================================================================== handle

struct crk_leaves {
    int64_t n = 0;
    int hydro = 0;
    crk_prec prec = CRK_F32;
    double r_fixed = 0.0;
    int64_t n_tiles = 0, n_leaves = 0;
    int n_cu = 1;
    crk_tuning tune{1, 32, 4, 4};
    int32_t* perm = nullptr;
    uint4* quant = nullptr;
    double* Hd = nullptr;
    int32_t* rng_off = nullptr;
    int2* rng = nullptr;
    int32_t* order_cull = nullptr;
    int32_t* order_pair = nullptr;
    int32_t* counter = nullptr;
    int32_t* cnt = nullptr;
    int64_t* ell_off = nullptr;
    int32_t* ell_len = nullptr;
    uint32_t* nbr = nullptr;
    double* partials = nullptr;
    unsigned long long* counts = nullptr;
    void* scratch = nullptr;
    size_t scratch_bytes = 0;
    int64_t stats[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    bool counted = false;
    // kernel timing (events on the launch stream)
    bool timing = false;
    struct Timed {
        int kind;
        hipEvent_t a, b;
    };
    std::vector<Timed> timed;
};


namespace crk {

template <class T> int dalloc(T** p, size_t count) {
    *p = nullptr;
    if (count == 0) count = 1;
    hipError_t e = hipMalloc(reinterpret_cast<void**>(p), count * sizeof(T));
    if (e != hipSuccess) return fail(CRK_ENOMEM, "hipMalloc(%zu bytes): %s", count * sizeof(T), hipGetErrorString(e));
    return CRK_OK;
}

void release(crk_leaves* L);
int ensure_scratch(crk_leaves* L, size_t bytes);
void drop_timed(crk_leaves* L);
Queue make_queue(const crk_leaves* L, const int32_t* order);
int grid_1wave(const crk_leaves* L);
int grid_nwave(const crk_leaves* L);
int check_gas(const crk_leaves* L, const crk_gas* g, bool need_v);
void reset_queue(crk_leaves* L, hipStream_t st);
Lists lists(const crk_leaves* L);

// Brackets one launch with events when timing is enabled.
struct TimeScope {
    crk_leaves* L;
    hipStream_t st;
    int kind;
    hipEvent_t a = nullptr, b = nullptr;
    TimeScope(crk_leaves* l, hipStream_t s, int k) : L(l), st(s), kind(k) {
        if (!L->timing) return;
        if (hipEventCreate(&a) != hipSuccess || hipEventCreate(&b) != hipSuccess) { a = b = nullptr; return; }
        (void)hipEventRecord(a, st);
    }
    ~TimeScope() {
        if (!a) return;
        (void)hipEventRecord(b, st);
        L->timed.push_back({kind, a, b});
    }
};

template <class R>
int pack_positions(crk_leaves* L, const double* x, const double* y, const double* z, const R* h,
                   hipStream_t st) {
    const int n = int(L->n);
    TimeScope ts(L, st, CRK_K_PACK);
    hipLaunchKernelGGL(k_pack_quant<R>, dim3((n + 255) / 256), dim3(256), 0, st, n, L->perm, x, y,
                       z, h, L->quant);
    LAUNCH_CHECK("pack_quant");
    return CRK_OK;
}

}  // namespace crk
