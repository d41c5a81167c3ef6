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
constexpr int kMaxGroups = 16;                                // work-queue chunks (counters)
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

// ------------------------------------------------------------------ device helpers

template <class R> __device__ __forceinline__ R sep(uint32_t a, uint32_t b) {
    return R(int32_t(a - b)) * R(kInvGrid);
}

// the same separation in grid units (2^32 per box length)
template <class R> __device__ __forceinline__ R grid_sep(uint32_t a, uint32_t b) {
    return R(int32_t(a - b));
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

// Work distribution over tiles.  `order` lists the tiles; it is cut into
// `groups` contiguous chunks, and workgroup b works on chunk b % groups first,
// so that with groups = 8 each XCD (workgroups are dispatched round-robin over
// the 8 XCDs) walks its own contiguous stretch of tree order and its L2 holds
// the neighbours those tiles share.  Non-persistent: one tile per wave.
// Persistent: every wave pulls tiles from its chunk's atomic counter and, when
// that chunk is drained, from the next chunks in turn; every wave exits once
// all chunks are drained.
struct Queue {
    const int32_t* order;
    int32_t* counter;  // one counter per group, zeroed before each launch
    int32_t n_items;
    int32_t persistent;
    int32_t groups;
    int32_t per_group;  // ceil(n_items / groups)
};

struct QState {
    int g, tries;
};

__device__ __forceinline__ int queue_next(const Queue& q, QState& st) {
    if (!q.persistent) return -1;
    while (st.tries < q.groups) {
        int it = 0;
        if ((threadIdx.x & 63) == 0) it = atomicAdd(q.counter + st.g, 1);
        it = __builtin_amdgcn_readfirstlane(it);
        const int idx = st.g * q.per_group + it;
        if (it < q.per_group && idx < q.n_items) return __builtin_amdgcn_readfirstlane(q.order[idx]);
        st.g = st.g + 1 == q.groups ? 0 : st.g + 1;
        st.tries += 1;
    }
    return -1;
}

__device__ __forceinline__ int queue_start(const Queue& q, QState& st) {
    const int g = int(blockIdx.x % unsigned(q.groups));
    if (!q.persistent) {
        const int bw = int(blockDim.x >> 6);
        const int slot = int(blockIdx.x / unsigned(q.groups)) * bw + int(threadIdx.x >> 6);
        const int idx = g * q.per_group + slot;
        // the item is wave-uniform: keep it in a scalar register
        return __builtin_amdgcn_readfirstlane((slot < q.per_group && idx < q.n_items) ? q.order[idx] : -1);
    }
    st.g = g;
    st.tries = 0;
    return queue_next(q, st);
}

static __global__ void k_reset(int32_t* c) {
    if (threadIdx.x < kMaxGroups) c[threadIdx.x] = 0;
}

static __global__ void k_zero8(double* t) {
    if (threadIdx.x < 8) t[threadIdx.x] = 0.0;
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

// A tile's neighbour lists: per lane `cnt` entries (the first `cnt` slots),
// per tile `len` slots (the longest lane); slot k of lane l at off + 64 k + l.
// Each slot also names the distinct particles its 64 entries refer to:
// scnt[off / 64 + k] of them, in srec[off + 64 k + e], and lane l's entry is
// the particle at position sidx[off + 64 k + l] of that set.
struct Lists {
    const int32_t* cnt;
    const int64_t* off;
    const int32_t* len;
    const uint32_t* nbr;
    const uint32_t* srec;
    const uint8_t* sidx;
    const int32_t* scnt;
};



// a pointer the caller knows to be wave-uniform, moved to scalar registers
template <class T> __device__ __forceinline__ const T* uniform_ptr(const T* p) {
    const uint64_t a = reinterpret_cast<uint64_t>(p);
    const uint32_t lo = __builtin_amdgcn_readfirstlane(uint32_t(a));
    const uint32_t hi = __builtin_amdgcn_readfirstlane(uint32_t(a >> 32));
    return reinterpret_cast<const T*>((uint64_t(hi) << 32) | lo);
}

// Neighbour-list loop of one lane with software-pipelined loads: the data of
// entry k+kD and the list index of entry k+kD+kI are requested before entry k
// is processed.  A wave's loads complete in issue order, so every wait covers
// all loads issued before the one it needs, among them index rows that miss to
// HBM (the rows stream once per pass and are the bulk of its traffic): both
// lookaheads must be deep for those round trips to hide behind other work.
// The loop is unrolled by eight over rings of registers (no copies between
// iterations); the slot counter stays in scalar registers and the rows are
// read through a buffer descriptor at a scalar offset (no address arithmetic
// per index load).  Every load is unconditional: slots past a lane's count
// hold a valid index (the list build pads them) and slot numbers are clamped
// to the tile's last slot.  row0 is the tile's slot-0 row (lane l of slot k at
// row0[64 k + l]); len is the tile's longest list; load(j) fetches neighbour
// j's data.  body(d, k) runs on every lane for every k < len: a lane past its
// own count must add nothing, by selection rather than a branch, which keeps
// the loop free of divergent control flow.
template <class D, int kD = 6, class Load, class Body>
__device__ __forceinline__ void pipelined_list(const uint32_t* __restrict__ row0, int len, Load load, Body body) {
    constexpr int kI = 8;   // indices requested kI entries ahead of their data
    constexpr int kRD = 8;  // data ring
    constexpr int kU = 8;   // unroll: a whole turn of both rings
    static_assert(kU % kI == 0 && kU % kRD == 0 && kD < kRD, "ring sizes");
    len = __builtin_amdgcn_readfirstlane(len);  // the tile's: a scalar slot loop
    if (len <= 0) return;
    const int last = len - 1;
    const __amdgpu_buffer_rsrc_t rows = __builtin_amdgcn_make_buffer_rsrc(
        const_cast<uint32_t*>(uniform_ptr(row0)), 0, len * kWave * 4, 0x00020000);
    const int vo = lane_id() * 4;
    auto slot = [&](int k) __attribute__((always_inline)) {
        return uint32_t(__builtin_amdgcn_raw_buffer_load_b32(rows, vo, (k < last ? k : last) * (kWave * 4), 0));
    };
    D d[kRD];        // entry e's data in d[e % kRD]
    uint32_t j[kI];  // entry e's index in j[e % kI]
    // The first entries' loads are issued in entry order (the scheduler
    // would otherwise put entry 0's data last, and the loop's waits, which
    // must hold on entry as on the back edge, would shrink to that).
    uint32_t j0[kD];
#pragma unroll
    for (int e = 0; e < kD; ++e) j0[e] = slot(e);
#pragma unroll
    for (int e = 0; e < kD; ++e) {
        d[e] = load(j0[e]);
        __builtin_amdgcn_sched_barrier(0);
    }
#pragma unroll
    for (int e = kD; e < kD + kI; ++e) j[e % kI] = slot(e);
    auto turn = [&](int k) __attribute__((always_inline)) {
#pragma unroll
        for (int u = 0; u < kU; ++u) {
            const int a = u + kD;
            d[a % kRD] = load(j[a % kI]);
            j[a % kI] = slot(k + a + kI);
            if (u == 0 || k + u < len) body(d[u % kRD], k + u);
        }
    };
    // The first turn is peeled: the loop is then entered with as many loads in
    // flight as its back edge carries, and its waits (one static count for
    // both ways in) keep the full depth.
    turn(0);
    for (int k = kU; k < len; k += kU) turn(k);
}

// Neighbour-list loop for large per-particle records (NCH 16-byte chunks),
// staged through LDS.  A per-lane gather of a record touches one cache line
// per lane per 16-byte load, and the L1 resolves about one line per clock, so
// the wave stages the records of a slot cooperatively instead: consecutive
// lanes fetch consecutive chunks of the same record -- whole lines -- with
// direct global-to-LDS loads into a wave-private buffer, and every lane then
// reads its own entry's record from LDS.  Only the slot's distinct particles
// are fetched (the list build orders each tile's lists so that lanes sharing
// a neighbour take it in the same slot): m records in ceil(m NCH / 64)
// loads.  LDS position q (16-byte units) holds chunk (q % NCH) ^ swz(r) of
// set record r = q / NCH; the swizzle (power-of-two NCH only) spreads the
// lanes' reads of one chunk over the banks.  A slot's set (its row of
// particle indices, one direct load into LDS), count and positions are
// fetched one slot ahead, and the slot's records are staged while the
// previous one is processed.
//
// kOff32: the records span at most 4 GiB and each load is a 32-bit offset
// from the scalar base; otherwise 64-bit addresses.  kShared = false stages
// all 64 entries of each slot in lane order instead (fixed LDS addresses per
// lane): the passes with the heaviest arithmetic per pair measure faster so.
template <int NCH> __device__ __forceinline__ int stage_swz(int r) {
    if ((NCH & (NCH - 1)) != 0) return 0;  // odd strides are conflict-free as they are
    return (r ^ (r >> 3)) & (NCH - 1);
}

// index of the calling wave within its workgroup, in a scalar register
__device__ __forceinline__ int wave_in_block() {
    return __builtin_amdgcn_readfirstlane(int(threadIdx.x >> 6));
}

// Byte offset of record j in the 32-bit form: a shift for power-of-two record
// sizes, else one 24-bit multiply (the form is taken only for j < 2^24).
template <class D> __device__ __forceinline__ uint32_t record_offset(uint32_t j) {
    constexpr uint32_t kSize = uint32_t(sizeof(D));
    if constexpr ((kSize & (kSize - 1)) == 0) return j * kSize;
    else return uint32_t(__umul24(j, kSize));
}

template <class D, bool kOff32, bool kShared = true, class Body>
__device__ __forceinline__ void staged_list(const Lists& L, int w, int cnt, int len,
                                            const D* __restrict__ recs, uint4* __restrict__ lds,
                                            Body body) {
    constexpr int NCH = int(sizeof(D) / 16);
    static_assert(sizeof(D) % 16 == 0, "records are whole 16-byte chunks");
    len = __builtin_amdgcn_readfirstlane(len);  // the tile's: slot loop and rows in scalar registers
    if (len <= 0) return;
    const int lane = lane_id();
    const int last = len - 1;
    const int64_t off = L.off[w];
    const uint32_t* row0 = uniform_ptr((kShared ? L.srec : L.nbr) + off);
    const __amdgpu_buffer_rsrc_t sets = __builtin_amdgcn_make_buffer_rsrc(
        const_cast<int32_t*>(uniform_ptr(L.scnt + (off >> 6))), 0, len * 4, 0x00020000);
    // the tile's positions as a buffer: slot k's byte row at a scalar offset
    const __amdgpu_buffer_rsrc_t pos = __builtin_amdgcn_make_buffer_rsrc(
        const_cast<uint8_t*>(uniform_ptr(L.sidx + off)), 0, len * kWave, 0x00020000);
    uint32_t coff[NCH];  // byte offset of the chunk this lane stages, within its record
    uint32_t roff[NCH];  // entry of the slot's set naming that record
#pragma unroll
    for (int t = 0; t < NCH; ++t) {
        const int g = t * kWave + lane;
        coff[t] = uint32_t((g % NCH) ^ stage_swz<NCH>(g / NCH)) * 16u;
        roff[t] = uint32_t(kWave % NCH == 0 ? t * (kWave / NCH) + lane / NCH : g / NCH);
    }
    uint32_t* rowbuf = reinterpret_cast<uint32_t*>(lds + NCH * kWave);
    uint32_t idx[NCH];
    auto load_set = [&](int k) __attribute__((always_inline)) {  // row of slot k into LDS
        const uint32_t* row = row0 + (k < last ? k : last) * kWave;
        __builtin_amdgcn_global_load_lds(row + lane, rowbuf, 4, 0, 0);
    };
    auto load_count = [&](int k) __attribute__((always_inline)) {
        return kShared ? __builtin_amdgcn_raw_buffer_load_b32(sets, 0, (k < last ? k : last) * 4, 0) : kWave;
    };
    auto load_pos = [&](int k) __attribute__((always_inline)) {
        return kShared ? uint32_t(__builtin_amdgcn_raw_buffer_load_b8(pos, lane, (k < last ? k : last) * kWave, 0))
                       : uint32_t(lane);
    };
    auto read_idx = [&](int) __attribute__((always_inline)) {
#pragma unroll
        for (int t = 0; t < NCH; ++t) idx[t] = rowbuf[roff[t]];
    };
    // only the loads that hold chunks of the set are issued (a wave-uniform
    // test); the lanes of the last one past the set fetch the set's first
    // record again (the rows are padded with it): lines already in flight
    auto stage = [&](int m) __attribute__((always_inline)) {
        const char* base = reinterpret_cast<const char*>(recs);
#pragma unroll
        for (int t = 0; t < NCH; ++t) {
            if (t * kWave < m * NCH) {
                const char* src = kOff32 ? base + (record_offset<D>(idx[t]) + coff[t])
                                         : base + size_t(idx[t]) * sizeof(D) + coff[t];
                __builtin_amdgcn_global_load_lds(src, lds + t * kWave, 16, 0, 0);
            }
        }
    };
    const char* lb = reinterpret_cast<const char*>(lds);
    auto read_rec = [&](uint32_t p) __attribute__((always_inline)) {
        D d;
        uint4* dst = reinterpret_cast<uint4*>(&d);
        const uint32_t sw = uint32_t(stage_swz<NCH>(int(p)));
#pragma unroll
        for (int c = 0; c < NCH; ++c)
            dst[c] = *reinterpret_cast<const uint4*>(lb + (p * NCH + (uint32_t(c) ^ sw)) * 16u);
        return d;
    };
    int m_next = __builtin_amdgcn_readfirstlane(load_count(0));
    uint32_t p_cur = load_pos(0);
    load_set(0);
    __builtin_amdgcn_s_waitcnt(0);
    read_idx(m_next);
    __builtin_amdgcn_s_waitcnt(0);
    stage(m_next);
    load_set(1);
    int m_after = load_count(1);
    uint32_t p_next = load_pos(1);
    for (int k = 0; k < len; ++k) {
        __builtin_amdgcn_s_waitcnt(0);  // this slot's records and the next slot's set are in LDS
        const D d = read_rec(p_cur);
        m_next = __builtin_amdgcn_readfirstlane(m_after);
        if (k + 1 < len) read_idx(m_next);
        __builtin_amdgcn_s_waitcnt(0);  // reads done before the buffers are refilled
        if (k + 1 < len) {
            stage(m_next);
            load_set(k + 2);
        }
        p_cur = p_next;
        m_after = load_count(k + 2);
        p_next = load_pos(k + 2);
        if (k < cnt) body(d, k);
    }
}

// True when every record of an array of n records of type D lies within
// 4 GiB of its base, and the index fits the 24-bit multiply where the record
// size is not a power of two (the 32-bit offset form of staged_list).
template <class D> inline bool records_off32(int64_t n) {
    constexpr uint64_t kSize = sizeof(D);
    const bool pow2 = (kSize & (kSize - 1)) == 0;
    return uint64_t(n) * kSize <= (uint64_t(1) << 32) && (pow2 || n <= (int64_t(1) << 24));
}

// Block-cooperative store of one record per thread: the records pass through
// LDS and leave as consecutive 16-byte chunks per lane (a thread storing its
// own 128-byte record would touch one cache line per lane per store).  Every
// thread of the block must call it; `first` is the block's first record and
// `count` the number of valid records from there.  buf holds blockDim.x records.
template <class Rec>
__device__ __forceinline__ void store_records(Rec* __restrict__ out, const Rec& r, bool valid, int first,
                                              int count, uint4* __restrict__ buf) {
    constexpr int NCH = int(sizeof(Rec) / 16);
    const int t = threadIdx.x;
    const uint4* src = reinterpret_cast<const uint4*>(&r);
    __syncthreads();
    if (valid)
#pragma unroll
        for (int c = 0; c < NCH; ++c) buf[t * NCH + c] = src[c];
    __syncthreads();
    uint4* dst = reinterpret_cast<uint4*>(out + first);
    const int total = count * NCH;
    for (int k = t; k < total; k += blockDim.x) dst[k] = buf[k];
}

// Position and volume of a neighbour, the moments pass's per-pair data.
template <class R> struct alignas(16) RecQV;
template <> struct alignas(16) RecQV<float> {
    uint32_t q[3];
    float V;
};
template <> struct alignas(16) RecQV<double> {
    uint32_t q[3];
    uint32_t unused;
    double V;
    double unused2;
};

template <class R> __global__ void k_pack_qv(int n, const int32_t* perm, const uint4* quant, const R* V,
                                             RecQV<R>* out) {
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= n) return;
    RecQV<R> r{};
    const uint4 q = quant[s];
    r.q[0] = q.x; r.q[1] = q.y; r.q[2] = q.z;
    r.V = V[perm[s]];
    out[s] = r;
}

// Whether a list-driven pass stages its neighbour records through LDS: always
// for records larger than 16 bytes; for 16-byte records when kStage16 (else
// they are gathered lane by lane).
template <class D, bool kStage16 = false> __host__ __device__ constexpr bool staged() {
    return sizeof(D) > 16 || kStage16;
}

// LDS of one wave in a list-driven pass, in 16-byte units: the staged records
// of a slot and the slot's row of indices (gathered records need none).
template <class D, bool kStage16 = false> __host__ __device__ constexpr int stage_stride() {
    return staged<D, kStage16>() ? int(sizeof(D) / 16) * kWave + kWave / 4 : 1;
}

// Dynamic LDS of a list-driven launch: one wave's buffers per wave of the
// workgroup.
template <class D, bool kStage16 = false> inline size_t stage_bytes(int block_waves) {
    return size_t(stage_stride<D, kStage16>()) * 16 * size_t(staged<D, kStage16>() ? block_waves : 1);
}

// 16-byte records are gathered lane by lane, with the loads software-pipelined
// (kStage16 = false), or staged through LDS like the larger ones: each slot's
// distinct particles fetched once (about 14 of 64 on the clustered gas), so a
// slot touches that many cache lines instead of one per lane.  The staged form
// calls body(d, k) for k < cnt only, the gathered one on every lane (see
// pipelined_list): a body used with both adds nothing where k >= cnt.
template <class D, bool kOff32, bool kStage16 = false, class Body>
__device__ __forceinline__ void list_loop(const Lists& L, int w, int cnt, int len,
                                          const D* __restrict__ recs, uint4* __restrict__ lds, Body body) {
    if constexpr (!staged<D, kStage16>()) {
        static_assert(sizeof(D) == 16, "gathered records are 16 bytes");
        // the records as a buffer (the 32-bit form spans at most 4 GiB): one
        // shift per load for its offset
        const __amdgpu_buffer_rsrc_t rb = __builtin_amdgcn_make_buffer_rsrc(
            const_cast<D*>(uniform_ptr(recs)), 0, int(0xffffffffu), 0x00020000);
        pipelined_list<D>(
            L.nbr + L.off[w], len,
            [&](uint32_t j) __attribute__((always_inline)) {
                if constexpr (kOff32)
                    return __builtin_bit_cast(D, __builtin_amdgcn_raw_buffer_load_b128(rb, int(j * 16u), 0, 0));
                else
                    return recs[j];
            },
            body);
    } else {
        staged_list<D, kOff32>(L, w, cnt, len, recs, lds, body);
    }
}

// Chunked compensated sums: plain partial sums over `chunk` pairs, folded into
// (s, c) Kahan pairs (FP32); plain sums in FP64.
// A lane adds the pairs of list slots 0, 1, ... in order, so after slot k it
// holds k + 1 pairs: with a power-of-two chunk the fold test depends on the
// wave-uniform slot number only (a scalar branch, no per-lane counter).
template <class R, int N> struct ChunkSums {
    R p[N], s[N], c[N];
    __device__ void zero() {
#pragma unroll
        for (int e = 0; e < N; ++e) { p[e] = R(0); s[e] = R(0); c[e] = R(0); }
    }
    __device__ void add(int e, R t) { p[e] += t; }
    __device__ void fold() {
        if (sizeof(R) != 4) return;
#pragma unroll
        for (int e = 0; e < N; ++e) { kadd(s[e], c[e], p[e]); p[e] = R(0); }
    }
    // after the pair of slot k; chunk is a power of two
    __device__ void next(int k, int chunk) {
        if (sizeof(R) == 4 && ((k + 1) & (chunk - 1)) == 0) fold();
    }
    // value after a final fold
    __device__ R get(int e) const { return sizeof(R) == 4 ? s[e] - c[e] : p[e]; }
};

// The same interface with plain sums (one register per value), for small
// secondary terms where the compensation's registers would cost occupancy.
template <class R, int N> struct PlainSums {
    R p[N];
    __device__ void zero() {
#pragma unroll
        for (int e = 0; e < N; ++e) p[e] = R(0);
    }
    __device__ void add(int e, R t) { p[e] += t; }
    __device__ void fold() {}
    __device__ void next(int, int) {}
    __device__ R get(int e) const { return p[e]; }
};

// ------------------------------------------------------------------ moments

// The correction moments of the lane's particle, as 29 independent FP64 sums
// S, and the number of neighbours inside the support.  The 40 moments (storage
// order: m0, m1[3], m2[6] (xx xy xz yy yz zz), g0[3], g1[9] (g1[a][c],
// a-major), g2[18] (g2[ab][c], ab in the m2 order)) follow from S
// (moments_from_sums).  Per pair (w = cW w(q) V_j, f = cF f(q) V_j, x = x_ij):
//   m0 += w, m1^a += x^a w, m2^ab += x^a x^b w, g0^c += f x^c,
//   t1^ac += f x^a x^c (symmetric: 6), t3^abc += f x^a x^b x^c (fully symmetric: 10);
// j = i is added analytically to m0; then g1^ac = delta^ac m0 + t1^ac and
// g2^abc = delta^ac m1^b + delta^bc m1^a + t3^abc.  FP32: plain sums over
// `chunk` pairs folded into compensated sums.  Every lane of the wave must call
// this (the loop runs over the tile's longest list).
template <class R, bool kOff32, bool kStage16 = false>
__device__ inline void moment_sums(int w, int s, bool valid, const Lists& L, const RecQV<R>* __restrict__ qv,
                                   uint4* __restrict__ lds, R H, int chunk, double S[29], int& nnb) {
    constexpr bool kComp = sizeof(R) == 4;
    constexpr int kN = 29;
    const int lane = lane_id();
    const RecQV<R> self = qv[valid ? s : 0];
    const uint4 qi = make_uint4(self.q[0], self.q[1], self.q[2], 0u);
    // separations in grid units (2^32 per box length): the sums of pairs with
    // g powers of x are 2^(32 g) times the physical ones (exact power-of-two
    // factors, removed in FP64 at the end)
    const R invHg = (R(1) / H) * R(kInvGrid);
    const R cW = norm_W(H), cF = norm_F(H);
    const int cnt = valid ? L.cnt[s] : 0;
    const int len = L.len[w];
    R p[kN], sm[kN], cm[kN];
#pragma unroll
    for (int e = 0; e < kN; ++e) { p[e] = R(0); sm[e] = R(0); cm[e] = R(0); }
    nnb = 0;
    list_loop<RecQV<R>, kOff32, kStage16>(
        L, w, cnt, len, qv, lds,
        [&](const RecQV<R>& d, int k) __attribute__((always_inline)) {
            const bool act = k < cnt;  // past the count: the pair adds zeros
            const R Vj = d.V;
            const R x[3] = {grid_sep<R>(qi.x, d.q[0]), grid_sep<R>(qi.y, d.q[1]), grid_sep<R>(qi.z, d.q[2])};
            const R r = dsqrt(x[0] * x[0] + x[1] * x[1] + x[2] * x[2]);
            const R q = r * invHg;
            R wq, fq;
            wendland(q, wq, fq);
            nnb += (act && q < R(1)) ? 1 : 0;
            const R wv = act ? cW * wq * Vj : R(0);
            const R fv = act ? cF * fq * Vj : R(0);
            R xx[6], x3[10];
            xx[0] = x[0] * x[0]; xx[1] = x[0] * x[1]; xx[2] = x[0] * x[2];
            xx[3] = x[1] * x[1]; xx[4] = x[1] * x[2]; xx[5] = x[2] * x[2];
            x3[0] = xx[0] * x[0]; x3[1] = xx[0] * x[1]; x3[2] = xx[0] * x[2];
            x3[3] = xx[1] * x[1]; x3[4] = xx[1] * x[2]; x3[5] = xx[2] * x[2];
            x3[6] = xx[3] * x[1]; x3[7] = xx[3] * x[2]; x3[8] = xx[4] * x[2]; x3[9] = xx[5] * x[2];
            p[0] += wv;
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                p[1 + a] += x[a] * wv;
                p[10 + a] += x[a] * fv;
            }
#pragma unroll
            for (int e = 0; e < 6; ++e) {
                p[4 + e] += xx[e] * wv;
                p[13 + e] += xx[e] * fv;
            }
#pragma unroll
            for (int e = 0; e < 10; ++e) p[19 + e] += x3[e] * fv;
            if (kComp && ((k + 1) & (chunk - 1)) == 0) {  // see ChunkSums
#pragma unroll
                for (int e = 0; e < kN; ++e) { kadd(sm[e], cm[e], p[e]); p[e] = R(0); }
            }
        });
#pragma unroll
    for (int e = 0; e < kN; ++e) {
        // power of x in sum e: m0 0, m1 1, m2 2, g0 1, t1 2, t3 3
        const int g = e == 0 ? 0 : e < 4 ? 1 : e < 10 ? 2 : e < 13 ? 1 : e < 19 ? 2 : 3;
        const double unit = g == 0 ? 1.0 : g == 1 ? kInvGrid : g == 2 ? kInvGrid * kInvGrid
                                                                   : kInvGrid * kInvGrid * kInvGrid;
        if (kComp) {
            kadd(sm[e], cm[e], p[e]);
            S[e] = (double(sm[e]) - double(cm[e])) * unit;
        } else {
            S[e] = double(p[e]) * unit;
        }
    }
    if (valid) S[0] += double(cW) * double(self.V);  // j = i
}

// The 40 moments from the 29 independent sums (self term included).
__device__ inline void moments_from_sums(const double S[29], double M[40]) {
    const int sym[3][3] = {{0, 1, 2}, {1, 3, 4}, {2, 4, 5}};
    const int cub[3][3][3] = {{{0, 1, 2}, {1, 3, 4}, {2, 4, 5}},
                              {{1, 3, 4}, {3, 6, 7}, {4, 7, 8}},
                              {{2, 4, 5}, {4, 7, 8}, {5, 8, 9}}};
    for (int e = 0; e < 13; ++e) M[e] = S[e];  // m0, m1, m2, g0
    for (int a = 0; a < 3; ++a)
        for (int c = 0; c < 3; ++c) M[13 + 3 * a + c] = (a == c ? S[0] : 0.0) + S[13 + sym[a][c]];
    for (int a = 0; a < 3; ++a)
        for (int b = a; b < 3; ++b)
            for (int c = 0; c < 3; ++c) {
                double t = S[19 + cub[a][b][c]];
                if (a == c) t += S[1 + b];
                if (b == c) t += S[1 + a];
                M[22 + 3 * sym[a][b] + c] = t;
            }
}

// FP64 per-particle solve of the reproducing conditions from the 40 moments
// (m0, m1[3], m2[6] (xx xy xz yy yz zz), g0[3], g1[9] (a-major), g2[18]
// ((ab) in m2 order, c fastest)).  Returns 1 for the zeroth-order fallback.
__device__ inline int solve_moments(const double* M, int nnb, double& A, double B[3], double dA[3],
                             double dB[9]) {
    const double m0 = M[0];
    const double* m1 = M + 1;
    const double* s = M + 4;
    const double* g0 = M + 10;
    const double* g1 = M + 13;
    const double* g2 = M + 22;
    // symmetric m2 and its adjugate
    const double a11 = s[0], a12 = s[1], a13 = s[2], a22 = s[3], a23 = s[4], a33 = s[5];
    const double i11 = a22 * a33 - a23 * a23;
    const double i12 = a13 * a23 - a12 * a33;
    const double i13 = a12 * a23 - a13 * a22;
    const double i22 = a11 * a33 - a13 * a13;
    const double i23 = a12 * a13 - a11 * a23;
    const double i33 = a11 * a22 - a12 * a12;
    const double det = a11 * i11 + a12 * i12 + a13 * i13;
    const double tr = (a11 + a22 + a33) / 3.0;
    if (nnb < 4 || !(det > 1e-12 * tr * tr * tr)) {
        A = 1.0 / m0;
        for (int c = 0; c < 3; ++c) {
            B[c] = 0.0;
            dA[c] = -g0[c] / (m0 * m0);
        }
        for (int k = 0; k < 9; ++k) dB[k] = 0.0;
        return 1;
    }
    const double rd = 1.0 / det;
    const double inv[3][3] = {{i11 * rd, i12 * rd, i13 * rd},
                              {i12 * rd, i22 * rd, i23 * rd},
                              {i13 * rd, i23 * rd, i33 * rd}};
    for (int a = 0; a < 3; ++a)
        B[a] = -(inv[a][0] * m1[0] + inv[a][1] * m1[1] + inv[a][2] * m1[2]);
    A = 1.0 / (m0 + B[0] * m1[0] + B[1] * m1[1] + B[2] * m1[2]);
    const int sym[3][3] = {{0, 1, 2}, {1, 3, 4}, {2, 4, 5}};
    for (int c = 0; c < 3; ++c) {
        double rhs[3];
        for (int a = 0; a < 3; ++a) {
            double t = g1[3 * a + c];
            for (int b = 0; b < 3; ++b) t += g2[3 * sym[a][b] + c] * B[b];
            rhs[a] = t;
        }
        double gA = g0[c];
        for (int a = 0; a < 3; ++a) {
            const double d = -(inv[a][0] * rhs[0] + inv[a][1] * rhs[1] + inv[a][2] * rhs[2]);
            dB[3 * a + c] = d;
            gA += B[a] * g1[3 * a + c] + m1[a] * d;
        }
        dA[c] = -A * A * gA;
    }
    return 0;
}


}  // namespace crk

// ====================================================================== handle

struct crk_leaves {
    int64_t n = 0;
    int hydro = 0;
    crk_prec prec = CRK_F32;
    double r_fixed = 0.0;
    double skin = 0.0;  // hydro lists: every support widened by this much (list reuse while particles move)
    bool dev_tree = false;  // built by crk_build_leaf_pairs_device (its scratch also holds the build's temporaries)
    double hmax = 0.0;      // device build: the largest support radius 2h
    int64_t n_tiles = 0, n_leaves = 0;
    int n_cu = 1;
    crk_tuning tune{0, 16, 4, 4, 8, 0, 0, 0, 0};  // measured best on the C2 workload
    int32_t* perm = nullptr;
    uint4* quant = nullptr;
    double* Hd = nullptr;
    int32_t* rng_off = nullptr;
    int2* rng = nullptr;
    int32_t* order_cull = nullptr;
    int32_t* order_pair = nullptr;
    int32_t* order_tree = nullptr;
    int32_t* counter = nullptr;
    int32_t* cnt = nullptr;
    int32_t* cnt_gather = nullptr;  // entries with r < H_i (the front of each lane's list)
    int64_t* ell_off = nullptr;
    int32_t* ell_len = nullptr;
    int32_t* ell_len_gather = nullptr;  // per tile: longest gather part
    int32_t* build_err = nullptr;       // lanes whose count and fill passes disagreed
    uint32_t* nbr = nullptr;
    uint32_t* srec = nullptr;  // per slot: its distinct particles (Lists)
    uint8_t* sidx = nullptr;   // per entry: its particle's position in the slot's set
    int32_t* scnt = nullptr;   // per slot: size of the set
    double* partials = nullptr;
    unsigned long long* counts = nullptr;
    // the caller's workspace: every device array above points into it, and
    // the per-pass scratch (records, adjoint partials) is its last part
    char* ws = nullptr;
    size_t ws_bytes = 0;
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

// Lays arrays out in the caller's workspace, each on a 256-byte boundary.
// With a null base it only measures (the pointers it returns are null).
struct Carver {
    char* base;
    size_t off = 0;
    explicit Carver(char* b) : base(b) {}
    template <class T> T* take(size_t count) {
        off = (off + 255) / 256 * 256;
        T* p = base ? reinterpret_cast<T*>(base + off) : nullptr;
        off += (count == 0 ? 1 : count) * sizeof(T);
        return p;
    }
    size_t used() const { return (off + 255) / 256 * 256; }
};

// Per-pass scratch of a handle (carved from its workspace at build time and
// sized for both precisions): CRK_ENOSPC if a pass would need more.
int pass_scratch(crk_leaves* L, size_t bytes, void** out);
// Scratch the backward pass needs for n particles in precision prec.
size_t backward_scratch_bytes(int64_t n, bool f64);
void drop_timed(crk_leaves* L);
Queue make_queue(const crk_leaves* L, const int32_t* order);
int grid_1wave(const crk_leaves* L);
int grid_nwave(const crk_leaves* L);
int check_gas(const crk_leaves* L, const crk_gas* g, bool need_v);
void reset_queue(crk_leaves* L, hipStream_t st);
Lists lists(const crk_leaves* L);         // pairs r < max(H_i, H_j)
Lists lists_gather(const crk_leaves* L);  // their front parts: r < H_i

// Device leaf build (Morton octree), in the handle's per-pass scratch:
// bytes it needs there; tree order (perm, quant, Hd) and leaves, with the
// inputs validated (CRK_EINVAL); tile candidate ranges (rng == nullptr: counts
// them into rng_off, *total and the host tile_cand; else fills rng); every
// leaf ordered by decreasing list length (cnt); list lengths per tile
// (ell_len, ell_off) with the total slots and entries on the host.
size_t devtree_scratch_bytes(int64_t n, int64_t nt);
int devtree_leaves(crk_leaves* L, const double* x, const double* y, const double* z, const void* h,
                   int leaf_max, hipStream_t st);
int devtree_ranges(crk_leaves* L, int2* rng, int64_t* total, std::vector<int64_t>* tile_cand, hipStream_t st);
int devtree_sort_leaves(crk_leaves* L, hipStream_t st);
int devtree_list_layout(crk_leaves* L, int64_t* slots, int64_t* entries, std::vector<int32_t>* len,
                        hipStream_t st);
constexpr int kDevLeafMax = 1024;  // largest leaf of the device build (one workgroup sorts it in LDS)

// Whether a pass over n records of type D takes the 32-bit offset form.
template <class D> inline bool off32(const crk_leaves* L) {
    return !L->tune.addr64 && records_off32<D>(L->n);
}

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
