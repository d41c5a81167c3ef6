// Extras pass for MI355X (gfx950): the CRK density and the reproducing-kernel
// gradients of velocity and internal energy (the paper's kernel sequence runs
// Geometry, Corrections, Extras, then Acceleration and Energy, Sec. 5; Extras
// evaluates the density and the state gradients the viscosity needs).
//
// Per particle i over its gather support (j with |x_ij| < H_i = 2h_i), with
// the corrected kernel W^R_ij = A_i (1 + B_i.x_ij) W_ij and its x_i-gradient
// G_ij (the same corrected gradient the force pass uses):
//   rhoR_i     = sum_j m_j W^R_ij                  (j = i included: m_i A_i W(0, h_i))
//   dv_i[a][c] = sum_{j != i} V_j (v_j^a - v_i^a) G_ij^c
//   du_i[c]    = sum_{j != i} V_j (u_j - u_i) G_ij^c
// Both gradients are exact for linear fields (the reproducing conditions).
// The pass walks the front (gather) part of each lane's neighbour list, with
// the neighbours' records staged through LDS.

#include "crk_internal.h"

using namespace crk;

namespace {

// What a neighbour contributes: position, volume, mass, velocity, energy.
template <class R> struct alignas(16) RecEx;
template <> struct alignas(16) RecEx<float> {
    uint32_t q[3];
    float V, m, vx, vy, vz, u;
    float pad[3];
};
template <> struct alignas(16) RecEx<double> {
    uint32_t q[3];
    uint32_t pad;
    double V, m, vx, vy, vz, u;
};
static_assert(sizeof(RecEx<float>) == 48 && sizeof(RecEx<double>) == 64, "whole 16-byte chunks");

template <class R>
__global__ void k_pack_ex(int n, const int32_t* __restrict__ perm, const uint4* __restrict__ quant,
                          const R* __restrict__ V, const R* __restrict__ m, const R* __restrict__ vx,
                          const R* __restrict__ vy, const R* __restrict__ vz, const R* __restrict__ u,
                          RecEx<R>* __restrict__ out) {
    __shared__ uint4 buf[256 * (sizeof(RecEx<R>) / 16)];
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    const bool valid = s < n;
    const int i = valid ? perm[s] : 0;
    RecEx<R> r{};
    const uint4 q = quant[valid ? s : 0];
    r.q[0] = q.x; r.q[1] = q.y; r.q[2] = q.z;
    r.V = V[i]; r.m = m[i];
    r.vx = vx[i]; r.vy = vy[i]; r.vz = vz[i];
    r.u = u[i];
    const int first = blockIdx.x * blockDim.x;
    store_records(out, r, valid, first, min(int(blockDim.x), n - first), buf);
}

template <class R, bool kOff32>
__global__ __launch_bounds__(256) void k_extras(Queue qu, int n, Lists L, const int32_t* __restrict__ perm,
                                                const RecEx<R>* __restrict__ rec, const R* __restrict__ h,
                                                const R* __restrict__ A, const R* __restrict__ B,
                                                const R* __restrict__ dA, const R* __restrict__ dB, int chunk,
                                                R* __restrict__ rhoR_out, R* __restrict__ dv_out,
                                                R* __restrict__ du_out) {
    constexpr int kStage = stage_stride<RecEx<R>>();
    extern __shared__ uint4 stage_buf[];  // kStage per wave (stage_bytes)
    const int lane = lane_id();
    QState qs;
    for (int w = queue_start(qu, qs); w >= 0; w = queue_next(qu, qs)) {
        const int s = w * kWave + lane;
        const bool valid = s < n;
        const int i = valid ? perm[s] : 0;
        const RecEx<R> ri = rec[valid ? s : 0];
        const R H = valid ? R(2) * h[i] : R(1);
        const R invH = R(1) / H;
        const R cW = norm_W(H), cF = norm_F(H);
        const R Ai = A[i];
        R Bi[3], dAi[3], dBi[9];
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            Bi[a] = B[3 * i + a];
            dAi[a] = dA[3 * i + a];
        }
#pragma unroll
        for (int k = 0; k < 9; ++k) dBi[k] = dB[9 * i + k];
        const int cnt = valid ? L.cnt[s] : 0;
        const int len = L.len[w];
        // sums: rhoR, dv[a][c] (a-major), du[c]
        ChunkSums<R, 13> S;
        S.zero();
        S.add(0, ri.m * Ai * cW);  // j = i: W(0, h_i) = cW
        staged_list<RecEx<R>, kOff32>(
            L, w, cnt, len, rec, stage_buf + wave_in_block() * kStage,
            [&](const RecEx<R>& rj, int k) __attribute__((always_inline)) {
                const R x[3] = {sep<R>(ri.q[0], rj.q[0]), sep<R>(ri.q[1], rj.q[1]), sep<R>(ri.q[2], rj.q[2])};
                const R r = dsqrt(x[0] * x[0] + x[1] * x[1] + x[2] * x[2]);
                R wq, fq;
                wendland(r * invH, wq, fq);
                const R W = cW * wq, F = cF * fq;
                const R lin = R(1) + Bi[0] * x[0] + Bi[1] * x[1] + Bi[2] * x[2];
                const R AW = Ai * W;
                S.add(0, rj.m * (AW * lin));
                const R dW = lin * W, AlF = Ai * lin * F;
                const R fv[3] = {rj.V * (rj.vx - ri.vx), rj.V * (rj.vy - ri.vy), rj.V * (rj.vz - ri.vz)};
                const R fu = rj.V * (rj.u - ri.u);
#pragma unroll
                for (int c = 0; c < 3; ++c) {
                    const R dBx = dBi[c] * x[0] + dBi[3 + c] * x[1] + dBi[6 + c] * x[2];
                    const R G = dAi[c] * dW + AW * (dBx + Bi[c]) + AlF * x[c];
#pragma unroll
                    for (int a = 0; a < 3; ++a) S.add(1 + 3 * a + c, fv[a] * G);
                    S.add(10 + c, fu * G);
                }
                S.next(k, chunk);
            });
        S.fold();
        if (valid) {
            rhoR_out[i] = S.get(0);
#pragma unroll
            for (int k = 0; k < 9; ++k) dv_out[9 * i + k] = S.get(1 + k);
#pragma unroll
            for (int c = 0; c < 3; ++c) du_out[3 * i + c] = S.get(10 + c);
        }
    }
}

template <class R>
int extras_impl(crk_leaves* L, const crk_gas* g, const R* V, const crk_corr* C, R* rhoR, R* dv, R* du,
                hipStream_t st) {
    const int n = int(L->n);
    int rc = pack_positions<R>(L, g->x, g->y, g->z, static_cast<const R*>(g->h), st);
    if (rc) return rc;
    void* sp = nullptr;
    if ((rc = pass_scratch(L, sizeof(RecEx<R>) * size_t(n), &sp))) return rc;
    RecEx<R>* rec = static_cast<RecEx<R>*>(sp);
    {
        TimeScope tp(L, st, CRK_K_PACK);
        hipLaunchKernelGGL(k_pack_ex<R>, dim3((n + 255) / 256), dim3(256), 0, st, n, L->perm, L->quant, V,
                           static_cast<const R*>(g->m), static_cast<const R*>(g->vx),
                           static_cast<const R*>(g->vy), static_cast<const R*>(g->vz),
                           static_cast<const R*>(g->u), rec);
    }
    LAUNCH_CHECK("pack extras");
    reset_queue(L, st);
    TimeScope ts(L, st, CRK_K_EXTRAS);
    auto kern = off32<RecEx<R>>(L) ? k_extras<R, true> : k_extras<R, false>;
    const int bw = L->tune.block_waves;
    hipLaunchKernelGGL(kern, dim3(grid_nwave(L)), dim3(kWave * bw), stage_bytes<RecEx<R>>(bw), st,
                       make_queue(L, L->order_pair), n, lists_gather(L), L->perm, rec,
                       static_cast<const R*>(g->h), static_cast<const R*>(C->A), static_cast<const R*>(C->B),
                       static_cast<const R*>(C->dA), static_cast<const R*>(C->dB), L->tune.kahan_chunk, rhoR,
                       dv, du);
    LAUNCH_CHECK("extras");
    return CRK_OK;
}

}  // namespace

extern "C" int crk_extras(crk_leaves* L, const crk_gas* g, const void* V, const crk_corr* C, crk_prec prec,
                          void* rhoR, void* dv, void* du, hipStream_t st) {
    int rc = check_gas(L, g, true);
    if (rc) return rc;
    if (L->n == 0) return CRK_OK;
    if (!V || !C || !C->A || !C->B || !C->dA || !C->dB || !rhoR || !dv || !du)
        return fail(CRK_EINVAL, "V, the corrections, rhoR, dv and du are required");
    if (prec == CRK_F32)
        return extras_impl<float>(L, g, (const float*)V, C, (float*)rhoR, (float*)dv, (float*)du, st);
    if (prec == CRK_F64)
        return extras_impl<double>(L, g, (const double*)V, C, (double*)rhoR, (double*)dv, (double*)du, st);
    return fail(CRK_EINVAL, "unknown precision");
}
