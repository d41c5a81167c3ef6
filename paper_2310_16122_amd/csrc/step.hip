// Time step and kick-drift update for MI355X (gfx950).
//
// The paper's code advances particles with a global time step taken as the
// minimum of a per-particle limit over all particles, reduced on the device
// with a floating-point atomic minimum (its SYCL port relies on atomic
// fetch_min of floats, Sec. 5.1).  Here the per-particle limit is the
// Courant condition and an acceleration condition,
//   dt_i = min( C_cfl 2h_i / (c_i + |v_i|),  C_acc sqrt(2h_i / |a_i|) ),
//   c_i = sqrt(gamma (gamma - 1) u_i),
// and the global minimum is reduced per workgroup in LDS and then across
// workgroups with one atomic minimum each on the bits of the (positive) value:
// positive IEEE numbers order like their bit patterns, and a minimum does not
// depend on the order of the updates, so the result is deterministic.  The
// step stays on the device: the kick-drift reads it from there.

#include "crk_internal.h"

using namespace crk;

namespace {

template <class R> struct Bits;
template <> struct Bits<float> {
    using U = unsigned int;
    static __device__ U of(float v) { return __float_as_uint(v); }
};
template <> struct Bits<double> {
    using U = unsigned long long;
    static __device__ U of(double v) { return static_cast<U>(__double_as_longlong(v)); }
};

template <class R> __global__ void k_dt_init(R* dt) {
    if (threadIdx.x == 0) dt[0] = R(INFINITY);
}

template <class R>
__global__ __launch_bounds__(256) void k_dt_min(int n, const R* __restrict__ h, const R* __restrict__ u,
                                                const R* __restrict__ vx, const R* __restrict__ vy,
                                                const R* __restrict__ vz, const R* __restrict__ a, R g1,
                                                R c_cfl, R c_acc, R* __restrict__ dt) {
    using U = typename Bits<R>::U;
    __shared__ R red[256];
    R best = R(INFINITY);
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        const R H = R(2) * h[i];
        const R cs = sqrt(g1 * u[i]);
        const R v = sqrt(vx[i] * vx[i] + vy[i] * vy[i] + vz[i] * vz[i]);
        R t = c_cfl * H / (cs + v);
        const R am = sqrt(a[3 * i] * a[3 * i] + a[3 * i + 1] * a[3 * i + 1] + a[3 * i + 2] * a[3 * i + 2]);
        if (am > R(0)) t = fmin(t, c_acc * sqrt(H / am));
        best = fmin(best, t);
    }
    red[threadIdx.x] = best;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if (int(threadIdx.x) < s) red[threadIdx.x] = fmin(red[threadIdx.x], red[threadIdx.x + s]);
        __syncthreads();
    }
    if (threadIdx.x == 0) atomicMin(reinterpret_cast<U*>(dt), Bits<R>::of(red[0]));
}

// v <- v + a dt, u <- u + du/dt dt, then x <- x + v dt wrapped into [0, 1);
// with disp, the step's largest drift |v dt| goes to disp[1] (atomic maximum
// on the bits of the positive value)
template <class R>
__global__ __launch_bounds__(256) void k_kick_drift(int n, double* __restrict__ x, double* __restrict__ y,
                                                    double* __restrict__ z, R* __restrict__ vx,
                                                    R* __restrict__ vy, R* __restrict__ vz, R* __restrict__ u,
                                                    const R* __restrict__ a, const R* __restrict__ dudt,
                                                    const R* __restrict__ dtp, double* __restrict__ disp) {
    __shared__ double red[256];
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    double moved = 0.0;
    if (i < n) {
        const R dt = dtp[0];
        const R v[3] = {vx[i] + a[3 * i] * dt, vy[i] + a[3 * i + 1] * dt, vz[i] + a[3 * i + 2] * dt};
        vx[i] = v[0];
        vy[i] = v[1];
        vz[i] = v[2];
        u[i] = u[i] + dudt[i] * dt;
        double* p[3] = {x, y, z};
        double d2 = 0.0;
        for (int c = 0; c < 3; ++c) {
            const double dx = double(v[c]) * double(dt);
            const double q = p[c][i] + dx;
            p[c][i] = q - floor(q);
            d2 += dx * dx;
        }
        moved = sqrt(d2);
    }
    if (!disp) return;  // uniform over the launch
    red[threadIdx.x] = moved;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if (int(threadIdx.x) < s) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + s]);
        __syncthreads();
    }
    if (threadIdx.x == 0)
        atomicMax(reinterpret_cast<unsigned long long*>(disp + 1),
                  static_cast<unsigned long long>(__double_as_longlong(red[0])));
}

// disp[0] += disp[1] (the step's largest drift), disp[1] = 0
__global__ void k_disp_add(double* disp) {
    if (threadIdx.x == 0) {
        disp[0] += disp[1];
        disp[1] = 0.0;
    }
}

template <class R>
int timestep_impl(int64_t n, const R* h, const R* u, const R* vx, const R* vy, const R* vz, const R* a,
                  double gamma, double c_cfl, double c_acc, R* dt, hipStream_t st) {
    hipLaunchKernelGGL(k_dt_init<R>, dim3(1), dim3(64), 0, st, dt);
    LAUNCH_CHECK("dt init");
    if (n == 0) return CRK_OK;
    const int blocks = int(std::min<int64_t>((n + 255) / 256, 4096));
    hipLaunchKernelGGL(k_dt_min<R>, dim3(blocks), dim3(256), 0, st, int(n), h, u, vx, vy, vz, a,
                       R(gamma * (gamma - 1.0)), R(c_cfl), R(c_acc), dt);
    LAUNCH_CHECK("dt min");
    return CRK_OK;
}

}  // namespace

extern "C" {

int crk_timestep(int64_t n, const void* h, const void* u, const void* vx, const void* vy, const void* vz,
                 const void* a, double gamma, double c_cfl, double c_acc, crk_prec prec, void* dt,
                 hipStream_t st) {
    if (n < 0 || n >= (int64_t(1) << 31)) return fail(CRK_EINVAL, "n out of range");
    if (!dt) return fail(CRK_EINVAL, "dt is required");
    if (n > 0 && (!h || !u || !vx || !vy || !vz || !a)) return fail(CRK_EINVAL, "h, u, v and a are required");
    if (!(gamma > 1.0) || !(c_cfl > 0.0) || !(c_acc > 0.0))
        return fail(CRK_EINVAL, "gamma > 1, c_cfl > 0 and c_acc > 0 are required");
    if (prec == CRK_F32)
        return timestep_impl<float>(n, (const float*)h, (const float*)u, (const float*)vx, (const float*)vy,
                                    (const float*)vz, (const float*)a, gamma, c_cfl, c_acc, (float*)dt, st);
    if (prec == CRK_F64)
        return timestep_impl<double>(n, (const double*)h, (const double*)u, (const double*)vx, (const double*)vy,
                                     (const double*)vz, (const double*)a, gamma, c_cfl, c_acc, (double*)dt, st);
    return fail(CRK_EINVAL, "unknown precision");
}

int crk_kick_drift(int64_t n, double* x, double* y, double* z, void* vx, void* vy, void* vz, void* u,
                   const void* a, const void* dudt, const void* dt, double* disp, crk_prec prec,
                   hipStream_t st) {
    if (n < 0 || n >= (int64_t(1) << 31)) return fail(CRK_EINVAL, "n out of range");
    if (n == 0) return CRK_OK;
    if (!x || !y || !z || !vx || !vy || !vz || !u || !a || !dudt || !dt)
        return fail(CRK_EINVAL, "positions, velocities, u, a, dudt and dt are required");
    if (prec != CRK_F32 && prec != CRK_F64) return fail(CRK_EINVAL, "unknown precision");
    const dim3 grid(unsigned((n + 255) / 256)), block(256);
    if (prec == CRK_F32)
        hipLaunchKernelGGL(k_kick_drift<float>, grid, block, 0, st, int(n), x, y, z, (float*)vx, (float*)vy,
                           (float*)vz, (float*)u, (const float*)a, (const float*)dudt, (const float*)dt, disp);
    else
        hipLaunchKernelGGL(k_kick_drift<double>, grid, block, 0, st, int(n), x, y, z, (double*)vx, (double*)vy,
                           (double*)vz, (double*)u, (const double*)a, (const double*)dudt, (const double*)dt,
                           disp);
    LAUNCH_CHECK("kick drift");
    if (disp) {
        hipLaunchKernelGGL(k_disp_add, dim3(1), dim3(64), 0, st, disp);
        LAUNCH_CHECK("displacement");
    }
    return CRK_OK;
}

}  // extern "C"
