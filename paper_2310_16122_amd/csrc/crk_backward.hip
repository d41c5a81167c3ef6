// Adjoint of the acceleration/energy pass and of the corrections and volume
// passes it depends on (reverse mode, gather form, per-tile recomputation).
//
// Given the upstream adjoints abar_i = dL/da_i and dubar_i = dL/d(du_i/dt),
// the gradients of L with respect to positions, velocities and internal
// energies are produced by four list-driven pair passes and two per-particle
// steps, with no pair quantity stored:
//
//  1. force adjoint (pairs): recompute F_ij, then with
//       Fbar_ij = abar_i/m_i - abar_j/m_j - (dubar_i/2m_i + dubar_j/2m_j)(v_i - v_j)
//     accumulate, for the lane's own particle only, vbar, Vbar, Pbar, the
//     adjoint of its corrections (A, B, dA, dB) through G_ij and xbar through
//     both G_ij and G_ji;
//  2. corrections adjoint (per particle, FP64): recompute the 40 moments with
//     the forward's arithmetic, then reverse the 3x3 solve -> Mbar;
//  3. moments adjoint (pairs): M_k = sum_j V_j phi(x_kj, h_k) gives xbar and
//     Vbar from the lane's own moments and from every neighbour whose moments
//     contain the lane's particle; then per particle Sbar = -Vbar V^2 + m rhobar
//     with rhobar = (gamma-1) u Pbar, and ubar = (gamma-1) rho Pbar;
//  4. volume adjoint (pairs): S_k = sum_j W(r_kj, h_k) gives xbar.
//
// Each lane accumulates only its own particle's adjoints, so no atomics are
// used and the result is bitwise reproducible.  FP32 path: pair arithmetic in
// FP32 with compensated sums; the solve adjoint in FP64.

#include <cstdio>

#include "crk_internal.h"

using namespace crk;

namespace {

// Per-particle record of the backward passes (unnormalised corrections;
// cW, cF, cF2 are the kernel, gradient and Hessian normalisations of h_i).
template <class R> struct alignas(128) RecBwd {
    uint32_t q[3];
    R invH;
    R V, P, A, dubar;  // dubar = (dL/d du_i) / (2 m_i)
    R cW, cF, cF2;
    R B[3], dA[3], dB[9], v[3];
    R abar[3];  // (dL/d a_i) / m_i
};
static_assert(sizeof(RecBwd<float>) == 128, "f32 backward record is one line");
static_assert(sizeof(RecBwd<double>) == 256, "f64 backward record is two lines");

// The backward record with what the artificial viscosity needs (box units):
// the velocity gradient dv[3a + c] = d_c v^a, h, the density and the sound speed.
template <class R> struct alignas(16) RecBwdV {
    uint32_t q[3];
    R invH;
    R V, P, A, dubar;
    R cW, cF, cF2;
    R B[3], dA[3], dB[9], v[3];
    R abar[3];
    R dv[9];
    R h, rho, cs;
};
static_assert(sizeof(RecBwdV<float>) % 16 == 0 && sizeof(RecBwdV<double>) % 16 == 0, "whole 16-byte chunks");

// Record of the extras adjoint: a particle's corrections, volume, velocity and
// the adjoint of its velocity gradient dvb[3a + c] = dL/d(d_c v^a).
template <class R> struct alignas(16) RecExA {
    uint32_t q[3];
    R invH;
    R V, A, cW, cF, cF2;
    R B[3], dA[3], dB[9], v[3];
    R dvb[9];
};
static_assert(sizeof(RecExA<float>) % 16 == 0 && sizeof(RecExA<double>) % 16 == 0, "whole 16-byte chunks");
static_assert(sizeof(RecExA<float>) <= sizeof(RecBwdV<float>) && sizeof(RecExA<double>) <= sizeof(RecBwdV<double>),
              "the extras adjoint's records reuse the force adjoint's");

// viscosity constants of a backward launch
template <class R> struct ViscB {
    R Cl, Cq, eps_q, g1;  // g1 = gamma (gamma - 1) / 2: d c / d u = g1 / c
};

// Wendland C4 shapes and the Hessian factor: W = cW w, grad W = cF f x,
// grad (cF f) = cF2 f2 x.
template <class R> __device__ __forceinline__ void shapes(R q, R& w, R& f, R& f2) {
    const R t = fmax(R(1) - q, R(0));
    const R t2 = t * t;
    f2 = t2 * t2;
    const R t5 = f2 * t;
    w = t5 * t * (R(1) + q * (R(6) + q * R(35.0 / 3.0)));
    f = t5 * (R(1) + R(5) * q);
}

// One side of a pair: the corrected kernel gradient of a particle (record r)
// at separation y from it, G^c = dA^c lin W + A t^c W + A lin F y^c, with
// lin = 1 + B.y and t^c = sum_a dB[a][c] y^a + B^c, and the pieces its adjoints
// share.  Written factored (the compiler does not reassociate): per side the
// gradient takes 3 FMA per component after lin and t.
template <class R> struct Side {
    R lin, t[3];
};

template <class R, class Rec> __device__ __forceinline__ Side<R> side_terms(const Rec& r, const R y[3]) {
    Side<R> s;
    s.lin = R(1) + r.B[0] * y[0] + r.B[1] * y[1] + r.B[2] * y[2];
#pragma unroll
    for (int c = 0; c < 3; ++c) s.t[c] = r.dB[c] * y[0] + r.dB[3 + c] * y[1] + r.dB[6 + c] * y[2] + r.B[c];
    return s;
}

template <class R, class Rec>
__device__ __forceinline__ void corr_grad(const Rec& r, const Side<R>& s, R W, R F, const R y[3], R G[3]) {
    const R LW = s.lin * W, AW = r.A * W, K = r.A * s.lin * F;
#pragma unroll
    for (int c = 0; c < 3; ++c) G[c] = LW * r.dA[c] + AW * s.t[c] + K * y[c];
}

// Contractions of the upstream adjoint g = Gbar with one side:
// al = g.dA, be = g.t, ga = g.y.
template <class R> struct Dots {
    R al, be, ga;
};

template <class R, class Rec>
__device__ __forceinline__ Dots<R> side_dots(const Rec& r, const Side<R>& s, const R y[3], const R g[3]) {
    return Dots<R>{g[0] * r.dA[0] + g[1] * r.dA[1] + g[2] * r.dA[2],
                   g[0] * s.t[0] + g[1] * s.t[1] + g[2] * s.t[2],
                   g[0] * y[0] + g[1] * y[1] + g[2] * y[2]};
}

// out += (dG/dy)^T g, i.e. per component e
//   W (al B^e + A (dB g)^e) + y^e (F (al lin + A be) + A lin F2 ga) + A F (ga B^e + lin g^e)
// (F2: the gradient factor of F, grad F = F2 y).
template <class R, class Rec>
__device__ __forceinline__ void corr_grad_dy(const Rec& r, const Side<R>& s, const Dots<R>& d, R W, R F,
                                             R F2, const R y[3], const R g[3], R out[3]) {
    const R AW = r.A * W, AF = r.A * F;
    const R KB = d.al * W + AF * d.ga;                                    // coefficient of B^e
    const R KY = F * (d.al * s.lin + r.A * d.be) + r.A * F2 * s.lin * d.ga;  // of y^e
    const R KG = AF * s.lin;                                              // of g^e
#pragma unroll
    for (int e = 0; e < 3; ++e) {
        const R dBg = r.dB[3 * e] * g[0] + r.dB[3 * e + 1] * g[1] + r.dB[3 * e + 2] * g[2];
        out[e] += KB * r.B[e] + AW * dBg + KY * y[e] + KG * g[e];
    }
}

// adjoint of G with respect to (A, B, dA, dB), given g = Gbar:
//   A: be W + lin F ga,  B^e: y^e (al W + A F ga) + A W g^e,
//   dA^d: lin W g^d,  dB[a][d]: A W y^a g^d
template <class R, class Rec, class Acc>
__device__ __forceinline__ void corr_grad_dC(const Rec& r, const Side<R>& s, const Dots<R>& d, R W, R F,
                                             const R y[3], const R g[3], Acc& acc) {
    const R AW = r.A * W, LW = s.lin * W;
    const R KB = d.al * W + r.A * F * d.ga;
    acc.add(0, d.be * W + s.lin * F * d.ga);  // A
#pragma unroll
    for (int e = 0; e < 3; ++e) acc.add(1 + e, KB * y[e] + AW * g[e]);  // B
#pragma unroll
    for (int c = 0; c < 3; ++c) acc.add(4 + c, LW * g[c]);  // dA
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const R AWy = AW * y[a];
#pragma unroll
        for (int c = 0; c < 3; ++c) acc.add(7 + 3 * a + c, AWy * g[c]);  // dB[a][c]
    }
}

// Record of particle i (tree position s).  Viscous records (RecBwdV) also get
// dv, h, rho and the sound speed c = sqrt(gamma (gamma - 1) u).
template <class R, class Rec>
__global__ void k_pack_bwd(int n, const int32_t* perm, const uint4* quant, const R* h, const R* u,
                           const R* vx, const R* vy, const R* vz, const R* m, const R* V,
                           const R* rho, const R* A, const R* B, const R* dA, const R* dB,
                           const R* ga, const R* gdu, R gm1, const R* dv, Rec* rec, R* aux) {
    __shared__ uint4 buf[256 * (sizeof(Rec) / 16)];
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    const bool valid = s < n;
    const int i = valid ? perm[s] : 0;
    Rec r;
    const uint4 q = quant[valid ? s : 0];
    r.q[0] = q.x; r.q[1] = q.y; r.q[2] = q.z;
    const R H = R(2) * h[i];
    const R invH = R(1) / H;
    r.invH = invH;
    r.V = V[i];
    r.P = gm1 * rho[i] * u[i];
    r.A = A[i];
    const R mi = m[i];
    r.dubar = gdu[i] / (R(2) * mi);
    r.cW = norm_W(H);
    r.cF = norm_F(H);
    const R i2 = invH * invH;
    r.cF2 = R(17325.0 / (2.0 * kPi)) * i2 * i2 * i2 * invH;
    for (int a = 0; a < 3; ++a) {
        r.B[a] = B[3 * i + a];
        r.dA[a] = dA[3 * i + a];
        r.abar[a] = ga[3 * i + a] / mi;
    }
    for (int k = 0; k < 9; ++k) r.dB[k] = dB[9 * i + k];
    r.v[0] = vx[i]; r.v[1] = vy[i]; r.v[2] = vz[i];
    if constexpr (sizeof(Rec) != sizeof(RecBwd<R>)) {
        for (int k = 0; k < 9; ++k) r.dv[k] = dv[9 * i + k];
        r.h = h[i];
        r.rho = rho[i];
        r.cs = sqrt((gm1 + R(1)) * gm1 * u[i]);
    }
    const int first = blockIdx.x * blockDim.x;
    store_records(rec, r, valid, first, min(int(blockDim.x), n - first), buf);
    if (valid) {
        aux[2 * s] = invH;
        aux[2 * s + 1] = r.V;
    }
}

// Artificial viscosity of a pair (box units, x = x_i - x_j) and the pieces its
// adjoint reuses: D_k = dv_k x, s_k = x.D_k, the van Leer limiter Phi, the
// reconstructed velocity difference w and mu_k = min(0, h_k (w.x) / den_k),
// den_k = r^2 + eps_q h_k^2; Q = sum_k rho_k (-C_l c_k mu_k + C_q mu_k^2).
template <class R> struct ViscPair {
    R Di[3], Dj[3], si, sj, phi, w[3], wx, deni, denj, mi, mj, Q;
};

template <class R, class Rec>
__device__ __forceinline__ ViscPair<R> visc_pair(const Rec& ri, const Rec& rj, const R x[3], R r2,
                                                 const ViscB<R>& vq) {
    ViscPair<R> p;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        p.Di[a] = ri.dv[3 * a] * x[0] + ri.dv[3 * a + 1] * x[1] + ri.dv[3 * a + 2] * x[2];
        p.Dj[a] = rj.dv[3 * a] * x[0] + rj.dv[3 * a + 1] * x[1] + rj.dv[3 * a + 2] * x[2];
    }
    p.si = x[0] * p.Di[0] + x[1] * p.Di[1] + x[2] * p.Di[2];
    p.sj = x[0] * p.Dj[0] + x[1] * p.Dj[1] + x[2] * p.Dj[2];
    const R sp = p.si * p.sj, ss = p.si + p.sj;
    p.phi = sp > R(0) ? R(4) * sp / (ss * ss) : R(0);
    p.wx = R(0);
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        p.w[a] = (ri.v[a] - rj.v[a]) - R(0.5) * p.phi * (p.Di[a] + p.Dj[a]);
        p.wx += p.w[a] * x[a];
    }
    p.deni = r2 + vq.eps_q * ri.h * ri.h;
    p.denj = r2 + vq.eps_q * rj.h * rj.h;
    p.mi = fmin(R(0), ri.h * p.wx / p.deni);
    p.mj = fmin(R(0), rj.h * p.wx / p.denj);
    p.Q = ri.rho * p.mi * (vq.Cq * p.mi - vq.Cl * ri.cs) + rj.rho * p.mj * (vq.Cq * p.mj - vq.Cl * rj.cs);
    return p;
}

// Reverse of visc_pair for the lane's own inputs, given Qb = dL/dQ: adds to
// xb (dL/dx_i), vb (dL/dv_i), dvb (dL/d dv_i), and returns dL/drho_i, dL/du_i.
template <class R, class Rec>
__device__ __forceinline__ void visc_pair_adj(const Rec& ri, const Rec& rj, const R x[3], const ViscPair<R>& p,
                                              const ViscB<R>& vq, R Qb, R xb[3], R vb[3], R dvb[9], R& rhob,
                                              R& ub) {
    const R mbi = p.mi < R(0) ? Qb * ri.rho * (R(2) * vq.Cq * p.mi - vq.Cl * ri.cs) : R(0);
    const R mbj = p.mj < R(0) ? Qb * rj.rho * (R(2) * vq.Cq * p.mj - vq.Cl * rj.cs) : R(0);
    rhob = Qb * p.mi * (vq.Cq * p.mi - vq.Cl * ri.cs);
    ub = ri.cs > R(0) ? -Qb * ri.rho * vq.Cl * p.mi * vq.g1 / ri.cs : R(0);
    const R wxb = mbi * ri.h / p.deni + mbj * rj.h / p.denj;
    const R r2b = -(mbi * p.mi / p.deni + mbj * p.mj / p.denj);
    R phib = R(0);
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const R wb = wxb * x[a];
        vb[a] += wb;
        xb[a] += wxb * p.w[a] + R(2) * r2b * x[a];
        phib -= R(0.5) * wb * (p.Di[a] + p.Dj[a]);
    }
    const R sp = p.si * p.sj, ss = p.si + p.sj;
    R sbi = R(0), sbj = R(0);
    if (sp > R(0)) {
        const R k = R(4) * phib / (ss * ss * ss);
        sbi = k * p.sj * (p.sj - p.si);
        sbj = k * p.si * (p.si - p.sj);
    }
    R Dbi[3], Dbj[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const R Db = -R(0.5) * p.phi * wxb * x[a];
        Dbi[a] = Db + sbi * x[a];
        Dbj[a] = Db + sbj * x[a];
        xb[a] += sbi * p.Di[a] + sbj * p.Dj[a];
    }
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        xb[c] += Dbi[0] * ri.dv[c] + Dbi[1] * ri.dv[3 + c] + Dbi[2] * ri.dv[6 + c] + Dbj[0] * rj.dv[c] +
                 Dbj[1] * rj.dv[3 + c] + Dbj[2] * rj.dv[6 + c];
#pragma unroll
        for (int a = 0; a < 3; ++a) dvb[3 * a + c] += Dbi[a] * x[c];
    }
}

// 1. force adjoint (kVisc: with the artificial viscosity, whose Q joins
// P_i + P_j; its adjoint also gives dL/d dv_i (dvbar) and dL/drho_i, dL/du_i
// through Q (qbar), all in tree order)
template <class R, bool kOff32, bool kVisc = false, class Rec = RecBwd<R>>
__device__ __forceinline__ void accel_adj_body(Queue qu, int n, Lists L, const int32_t* __restrict__ perm,
                                               const Rec* __restrict__ rec, int chunk, R* __restrict__ cbar,
                                               R* __restrict__ vpbar, R* __restrict__ xbar, R* __restrict__ gv,
                                               ViscB<R> vq, R* __restrict__ dvbar, R* __restrict__ qbar) {
    constexpr int kStage = stage_stride<Rec>();
    extern __shared__ uint4 stage_buf[];  // kStage per wave (stage_bytes)
    const int lane = lane_id();
    QState qs;
    for (int w = queue_start(qu, qs); w >= 0; w = queue_next(qu, qs)) {
        const int s = w * kWave + lane;
        const bool valid = s < n;
        const Rec ri = rec[valid ? s : 0];
        const int cnt = valid ? L.cnt[s] : 0;
        const int len = L.len[w];
        ChunkSums<R, 16> cb;  // A, B[3], dA[3], dB[9]
        ChunkSums<R, 8> ob;   // Vbar, Pbar, xbar[3], vbar[3]
        // dvbar[9], rhobar, ubar (through Q): the viscosity's own adjoints, summed
        // plainly in FP32 (their compensation's registers would halve the occupancy)
        PlainSums<R, kVisc ? 11 : 1> qb;
        cb.zero();
        ob.zero();
        qb.zero();
        staged_list<Rec, kOff32, false>(  // measured faster with fixed LDS addresses
            L, w, cnt, len, rec, stage_buf + wave_in_block() * kStage,
            [&](const Rec& rj, int k) __attribute__((always_inline)) {
                const R x[3] = {sep<R>(ri.q[0], rj.q[0]), sep<R>(ri.q[1], rj.q[1]), sep<R>(ri.q[2], rj.q[2])};
                const R y[3] = {-x[0], -x[1], -x[2]};
                const R r = dsqrt(x[0] * x[0] + x[1] * x[1] + x[2] * x[2]);
                R wi, fi, f2i, wj, fj, f2j;
                shapes(r * ri.invH, wi, fi, f2i);
                shapes(r * rj.invH, wj, fj, f2j);
                const R Wi = ri.cW * wi, Fi = ri.cF * fi, F2i = ri.cF2 * f2i;
                const R Wj = rj.cW * wj, Fj = rj.cF * fj, F2j = rj.cF2 * f2j;
                const Side<R> si = side_terms(ri, x), sj = side_terms(rj, y);
                R Gi[3], Gj[3];
                corr_grad(ri, si, Wi, Fi, x, Gi);
                corr_grad(rj, sj, Wj, Fj, y, Gj);
                const R D[3] = {Gi[0] - Gj[0], Gi[1] - Gj[1], Gi[2] - Gj[2]};
                const R VV = ri.V * rj.V;
                ViscPair<R> vp{};
                if constexpr (kVisc) vp = visc_pair(ri, rj, x, x[0] * x[0] + x[1] * x[1] + x[2] * x[2], vq);
                const R PP = kVisc ? (ri.P + rj.P) + vp.Q : ri.P + rj.P;
                const R coef = R(-0.5) * (VV * PP);
                const R kap = ri.dubar + rj.dubar;
                R Fb[3], s_ = R(0);
#pragma unroll
                for (int c = 0; c < 3; ++c) {
                    const R vij = ri.v[c] - rj.v[c];
                    Fb[c] = ri.abar[c] - rj.abar[c] - kap * vij;
                    s_ += Fb[c] * D[c];
                    ob.add(5 + c, -kap * coef * D[c]);  // vbar_i
                }
                ob.add(0, R(-0.5) * rj.V * PP * s_);  // Vbar_i
                ob.add(1, R(-0.5) * VV * s_);         // Pbar_i
                const R g[3] = {coef * Fb[0], coef * Fb[1], coef * Fb[2]};
                const Dots<R> di = side_dots(ri, si, x, g), dj = side_dots(rj, sj, y, g);
                corr_grad_dC(ri, si, di, Wi, Fi, x, g, cb);
                R xb[3] = {R(0), R(0), R(0)};
                if constexpr (kVisc) {
                    // Q enters like P_i + P_j: dL/dQ = dL/dP_i of this pair
                    R vb[3] = {R(0), R(0), R(0)}, dvb[9], rhob, ub;
#pragma unroll
                    for (int e = 0; e < 9; ++e) dvb[e] = R(0);
                    visc_pair_adj(ri, rj, x, vp, vq, R(-0.5) * VV * s_, xb, vb, dvb, rhob, ub);
#pragma unroll
                    for (int c = 0; c < 3; ++c) ob.add(5 + c, vb[c]);
#pragma unroll
                    for (int e = 0; e < 9; ++e) qb.add(e, dvb[e]);
                    qb.add(9, rhob);
                    qb.add(10, ub);
                    qb.next(k, chunk);
                }
                corr_grad_dy(ri, si, di, Wi, Fi, F2i, x, g, xb);
                corr_grad_dy(rj, sj, dj, Wj, Fj, F2j, y, g, xb);
#pragma unroll
                for (int c = 0; c < 3; ++c) ob.add(2 + c, xb[c]);
                cb.next(k, chunk);
                ob.next(k, chunk);
            });
        cb.fold();
        ob.fold();
        qb.fold();
        if (valid) {
            const int i = perm[s];
            if constexpr (kVisc) {
#pragma unroll
                for (int e = 0; e < 9; ++e) dvbar[9 * s + e] = qb.get(e);
                qbar[2 * s] = qb.get(9);
                qbar[2 * s + 1] = qb.get(10);
            }
#pragma unroll
            for (int e = 0; e < 16; ++e) cbar[16 * s + e] = cb.get(e);
            vpbar[2 * s] = ob.get(0);
            vpbar[2 * s + 1] = ob.get(1);
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                xbar[4 * s + c] = ob.get(2 + c);
                gv[3 * i + c] = ob.get(5 + c);
            }
        }
    }
}

template <class R, bool kOff32>
__global__ __launch_bounds__(256) void k_accel_adj(Queue qu, int n, Lists L, const int32_t* __restrict__ perm,
                                                   const RecBwd<R>* __restrict__ rec, int chunk,
                                                   R* __restrict__ cbar, R* __restrict__ vpbar,
                                                   R* __restrict__ xbar, R* __restrict__ gv) {
    accel_adj_body<R, kOff32>(qu, n, L, perm, rec, chunk, cbar, vpbar, xbar, gv, ViscB<R>{}, nullptr, nullptr);
}

// the viscous form, held to two waves per SIMD (FP32: a few registers spill)
template <class R, bool kOff32>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(sizeof(R) == 4 ? 2 : 1)))
void k_accel_adj_visc(Queue qu, int n, Lists L, const int32_t* __restrict__ perm,
                      const RecBwdV<R>* __restrict__ rec, int chunk, R* __restrict__ cbar, R* __restrict__ vpbar,
                      R* __restrict__ xbar, R* __restrict__ gv, ViscB<R> vq, R* __restrict__ dvbar,
                      R* __restrict__ qbar) {
    accel_adj_body<R, kOff32, true, RecBwdV<R>>(qu, n, L, perm, rec, chunk, cbar, vpbar, xbar, gv, vq, dvbar, qbar);
}

// Reverse of the FP64 solve (solve_moments) for one particle: corrections
// adjoint Cb (A, B[3], dA[3], dB[9]) -> moments adjoint Mb[40] (storage order).
__device__ inline void solve_moments_adjoint(const double* M, int nnb, const double* Cb, double* Mb) {
    for (int e = 0; e < 40; ++e) Mb[e] = 0.0;
    const double m0 = M[0];
    const double* m1 = M + 1;
    const double* sm = M + 4;
    const double* g0 = M + 10;
    const double* g1 = M + 13;
    const double* g2 = M + 22;
    const double a11 = sm[0], a12 = sm[1], a13 = sm[2], a22 = sm[3], a23 = sm[4], a33 = sm[5];
    const double i11 = a22 * a33 - a23 * a23;
    const double i12 = a13 * a23 - a12 * a33;
    const double i13 = a12 * a23 - a13 * a22;
    const double i22 = a11 * a33 - a13 * a13;
    const double i23 = a12 * a13 - a11 * a23;
    const double i33 = a11 * a22 - a12 * a12;
    const double det = a11 * i11 + a12 * i12 + a13 * i13;
    const double tr = (a11 + a22 + a33) / 3.0;
    if (nnb < 4 || !(det > 1e-12 * tr * tr * tr)) {
        // A = 1/m0, dA = -g0/m0^2
        double mb = -Cb[0] / (m0 * m0);
        for (int c = 0; c < 3; ++c) {
            mb += Cb[4 + c] * 2.0 * g0[c] / (m0 * m0 * m0);
            Mb[10 + c] = -Cb[4 + c] / (m0 * m0);
        }
        Mb[0] = mb;
        return;
    }
    const double rd = 1.0 / det;
    const double inv[3][3] = {{i11 * rd, i12 * rd, i13 * rd},
                              {i12 * rd, i22 * rd, i23 * rd},
                              {i13 * rd, i23 * rd, i33 * rd}};
    const int sym[3][3] = {{0, 1, 2}, {1, 3, 4}, {2, 4, 5}};
    double B[3];
    for (int a = 0; a < 3; ++a) B[a] = -(inv[a][0] * m1[0] + inv[a][1] * m1[1] + inv[a][2] * m1[2]);
    const double A = 1.0 / (m0 + B[0] * m1[0] + B[1] * m1[1] + B[2] * m1[2]);
    double Ab = Cb[0];
    double Bb[3] = {Cb[1], Cb[2], Cb[3]};
    double m0b = 0.0, m1b[3] = {0, 0, 0}, g0b[3] = {0, 0, 0};
    double g1b[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}};
    double g2b[3][3][3];
    double invb[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}};
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b)
            for (int c = 0; c < 3; ++c) g2b[a][b][c] = 0.0;
    for (int c = 0; c < 3; ++c) {
        double rhs[3], dB[3];
        for (int a = 0; a < 3; ++a) {
            double t = g1[3 * a + c];
            for (int b = 0; b < 3; ++b) t += g2[3 * sym[a][b] + c] * B[b];
            rhs[a] = t;
        }
        double tc = g0[c];
        for (int a = 0; a < 3; ++a) {
            dB[a] = -(inv[a][0] * rhs[0] + inv[a][1] * rhs[1] + inv[a][2] * rhs[2]);
            tc += B[a] * g1[3 * a + c] + m1[a] * dB[a];
        }
        // dA_c = -A^2 tc
        const double dAb = Cb[4 + c];
        const double tb = -A * A * dAb;
        Ab += -2.0 * A * tc * dAb;
        g0b[c] += tb;
        double dBb[3];
        for (int a = 0; a < 3; ++a) {
            Bb[a] += tb * g1[3 * a + c];
            g1b[a][c] += tb * B[a];
            m1b[a] += tb * dB[a];
            dBb[a] = Cb[7 + 3 * a + c] + tb * m1[a];
        }
        // dB[.,c] = -inv rhs
        double rb[3];
        for (int b = 0; b < 3; ++b) rb[b] = -(inv[0][b] * dBb[0] + inv[1][b] * dBb[1] + inv[2][b] * dBb[2]);
        for (int a = 0; a < 3; ++a)
            for (int b = 0; b < 3; ++b) invb[a][b] += -dBb[a] * rhs[b];
        // rhs = g1[.,c] + g2[.,.,c] B
        for (int a = 0; a < 3; ++a) {
            g1b[a][c] += rb[a];
            for (int b = 0; b < 3; ++b) {
                g2b[a][b][c] += rb[a] * B[b];
                Bb[b] += g2[3 * sym[a][b] + c] * rb[a];
            }
        }
    }
    // A = 1/den, den = m0 + B.m1
    const double denb = -A * A * Ab;
    m0b += denb;
    for (int a = 0; a < 3; ++a) {
        Bb[a] += denb * m1[a];
        m1b[a] += denb * B[a];
    }
    // B = -inv m1
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) invb[a][b] += -Bb[a] * m1[b];
    for (int b = 0; b < 3; ++b) m1b[b] += -(inv[0][b] * Bb[0] + inv[1][b] * Bb[1] + inv[2][b] * Bb[2]);
    // inv = m2^-1: m2b = -inv invb inv
    double t[3][3], m2b[3][3];
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) t[a][b] = invb[a][0] * inv[0][b] + invb[a][1] * inv[1][b] + invb[a][2] * inv[2][b];
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) m2b[a][b] = -(inv[a][0] * t[0][b] + inv[a][1] * t[1][b] + inv[a][2] * t[2][b]);
    Mb[0] = m0b;
    for (int a = 0; a < 3; ++a) {
        Mb[1 + a] = m1b[a];
        Mb[10 + a] = g0b[a];
        for (int c = 0; c < 3; ++c) Mb[13 + 3 * a + c] = g1b[a][c];
    }
    for (int a = 0; a < 3; ++a)
        for (int b = a; b < 3; ++b) {
            const int p = sym[a][b];
            Mb[4 + p] = a == b ? m2b[a][a] : m2b[a][b] + m2b[b][a];
            for (int c = 0; c < 3; ++c)
                Mb[22 + 3 * p + c] = a == b ? g2b[a][a][c] : g2b[a][b][c] + g2b[b][a][c];
        }
}

// Record of the moments adjoint: Mbar . phi(y) for the 40 moment kernels phi
// of a particle (support radius 1/invH) is
//   Phi(y) = W(r) P(y) + F(r) Q(y),   grad W = F y,  grad F = F2 y,
// with P = P0 + P1.y + y.P2.y and Q = Q1.y + y.Q2.y + Q3(y, y, y).  The 40
// adjoints collapse to 29 coefficients: c[0] P0, c[1..3] P1, c[4..9] P2,
// c[10..12] Q1, c[13..18] Q2 (monomials xx xy xz yy yz zz), c[19..28] Q3
// (monomials xxx xxy xxz xyy xyz xzz yyy yyz yzz zzz).
template <class R> struct alignas(16) RecMom {
    uint32_t q[3];
    R invH;
    R V;
    R c[29];
};

// 40 moment adjoints (storage order) -> 29 polynomial coefficients
__device__ inline void moment_poly(const double* Mb, double* c) {
    const int pa[6] = {0, 0, 0, 1, 1, 2}, pb[6] = {0, 1, 2, 1, 2, 2};
    const double* mu1 = Mb + 1;
    const double* mu2 = Mb + 4;
    const double* g0 = Mb + 10;
    const double* g1 = Mb + 13;
    const double* g2 = Mb + 22;
    for (int e = 0; e < 29; ++e) c[e] = 0.0;
    c[0] = Mb[0] + g1[0] + g1[4] + g1[8];
    for (int e = 0; e < 3; ++e) {
        c[1 + e] = mu1[e];
        c[10 + e] = g0[e];
    }
    // cubic monomial index of sorted (a <= b <= c)
    auto cub = [](int a, int b, int cc) {
        int t;
        if (a > b) { t = a; a = b; b = t; }
        if (b > cc) { t = b; b = cc; cc = t; }
        if (a > b) { t = a; a = b; b = t; }
        const int base[3] = {0, 6, 9};  // monomials starting with x, y, z
        const int off2[3][3] = {{0, 1, 2}, {0, 3, 4}, {0, 0, 5}};  // (b, c) within x-block
        if (a == 0) return off2[b][cc];
        if (a == 1) return base[1] + (b == 1 ? (cc == 1 ? 0 : cc == 2 ? 1 : 0) : 2);
        return base[2];
    };
    for (int p = 0; p < 6; ++p) {
        c[4 + p] = mu2[p];
        // delta terms of g2: delta^ac x^b W + delta^bc x^a W
        c[1 + pb[p]] += g2[3 * p + pa[p]];
        c[1 + pa[p]] += g2[3 * p + pb[p]];
        for (int cc = 0; cc < 3; ++cc) c[19 + cub(pa[p], pb[p], cc)] += g2[3 * p + cc];
    }
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) {
            const int lo = a < b ? a : b, hi = a < b ? b : a;
            const int p = lo == 0 ? hi : (lo == 1 ? 2 + hi : 5);
            c[13 + p] += g1[3 * a + b];
        }
}

// Gradient-ready coefficients.  The records hold the 29 coefficients with the
// multiplicities of the derivatives folded in (scale_coefficients): for the
// quadratic forms (monomials xx xy xz yy yz zz) the diagonal ones doubled, for
// the cubic form (xxx xxy xxz xyy xyz xzz yyy yyz yzz zzz) the pure cubes
// tripled and xyz halved.  With Y2 = (y0^2, 2 y0 y1, 2 y0 y2, y1^2, 2 y1 y2,
// y2^2) every gradient component is then a plain dot product.
__device__ inline void scale_coefficients(double* c) {
    for (int o : {4, 13}) {
        c[o + 0] *= 2.0;
        c[o + 3] *= 2.0;
        c[o + 5] *= 2.0;
    }
    c[19 + 0] *= 3.0;
    c[19 + 4] *= 0.5;
    c[19 + 6] *= 3.0;
    c[19 + 9] *= 3.0;
}

// grad of the symmetric quadratic form with monomial coefficients k[6] (value = y.grad / 2)
template <class R> __device__ __forceinline__ void quad_grad(const R* k, const R y[3], R g[3]) {
    g[0] = R(2) * k[0] * y[0] + k[1] * y[1] + k[2] * y[2];
    g[1] = k[1] * y[0] + R(2) * k[3] * y[1] + k[4] * y[2];
    g[2] = k[2] * y[0] + k[4] * y[1] + R(2) * k[5] * y[2];
}

// grad of the symmetric cubic form with monomial coefficients k[10] (value = y.grad / 3)
template <class R> __device__ __forceinline__ void cubic_grad(const R* k, const R Y2[6], R g[3]) {
    g[0] = R(3) * k[0] * Y2[0] + R(2) * k[1] * Y2[1] + R(2) * k[2] * Y2[2] + k[3] * Y2[3] + k[4] * Y2[4] +
           k[5] * Y2[5];
    g[1] = k[1] * Y2[0] + R(2) * k[3] * Y2[1] + k[4] * Y2[2] + R(3) * k[6] * Y2[3] + R(2) * k[7] * Y2[4] +
           k[8] * Y2[5];
    g[2] = k[2] * Y2[0] + k[4] * Y2[1] + R(2) * k[5] * Y2[2] + k[7] * Y2[3] + R(2) * k[8] * Y2[4] +
           R(3) * k[9] * Y2[5];
}

// Phi(y) and grad Phi(y) from the 29 coefficients of a particle, stored
// pre-multiplied by its kernel normalisations (c[0..9] by cW, c[10..28] by
// cF), so that with the bare shapes w, f, f2 at q = |y|/H and s2 = 1/H^2:
//   Phi = w P + f Q,  grad = w dP + f dQ + s2 (a f P + b f2 Q) y,
// a = (cF / cW) H^2 = -56/3 and b = (cF2 / cF) H^2 = -30 for the Wendland C4.
template <class R>
__device__ __forceinline__ void moment_phi(const R* c, R W, R F, R F2, R s2, const R y[3], R& Phi,
                                           R grad[3]) {
    R Y2[6];
    Y2[0] = y[0] * y[0]; Y2[1] = y[0] * y[1]; Y2[2] = y[0] * y[2];
    Y2[3] = y[1] * y[1]; Y2[4] = y[1] * y[2]; Y2[5] = y[2] * y[2];
    R gP2[3], gQ2[3], gQ3[3];
    quad_grad(c + 4, y, gP2);
    quad_grad(c + 13, y, gQ2);
    cubic_grad(c + 19, Y2, gQ3);
    const R yP2 = y[0] * gP2[0] + y[1] * gP2[1] + y[2] * gP2[2];
    const R yQ2 = y[0] * gQ2[0] + y[1] * gQ2[1] + y[2] * gQ2[2];
    const R yQ3 = y[0] * gQ3[0] + y[1] * gQ3[1] + y[2] * gQ3[2];
    const R P = c[0] + c[1] * y[0] + c[2] * y[1] + c[3] * y[2] + R(0.5) * yP2;
    const R Q = c[10] * y[0] + c[11] * y[1] + c[12] * y[2] + R(0.5) * yQ2 + yQ3 * R(1.0 / 3.0);
    Phi = W * P + F * Q;
    const R radial = s2 * (R(-56.0 / 3.0) * F * P + R(-30.0) * F2 * Q);
#pragma unroll
    for (int e = 0; e < 3; ++e)
        grad[e] = W * (c[1 + e] + gP2[e]) + F * (c[10 + e] + gQ2[e] + gQ3[e]) + radial * y[e];
}

// Record of the volume adjoint: position, 1/H and Sbar of a neighbour.
template <class R> struct alignas(16) RecVA {
    uint32_t q[3];
    R invH;
    R Sbar;
};

// Per particle (tree position s): the adjoint of the FP64 solve from the 40
// moments and the correction adjoints, compressed to the 29 polynomial
// coefficients of the moments adjoint, written with the position, 1/H and V.
template <class R>
__device__ inline void moments_adjoint_record(int s, const double M[40], int nnb, const uint4* __restrict__ quant,
                                              const R* __restrict__ aux, const R* __restrict__ cbar,
                                              RecMom<R>* __restrict__ mrec) {
    double Cb[16], Mb[40], c[29];
    for (int e = 0; e < 16; ++e) Cb[e] = double(cbar[16 * s + e]);
    solve_moments_adjoint(M, nnb, Cb, Mb);
    moment_poly(Mb, c);
    RecMom<R> r;
    const uint4 q = quant[s];
    r.q[0] = q.x; r.q[1] = q.y; r.q[2] = q.z;
    r.invH = aux[2 * s];
    r.V = aux[2 * s + 1];
    // pre-multiplied by the kernel normalisations of h_s (see moment_phi)
    const double ih = double(r.invH);
    const double cW = 495.0 / (32.0 * kPi) * ih * ih * ih;
    const double cF = -1155.0 / (4.0 * kPi) * ih * ih * ih * ih * ih;
    for (int e = 0; e < 29; ++e) r.c[e] = R(c[e] * (e < 10 ? cW : cF));
    mrec[s] = r;
}

// 2. moments recomputed with the forward's arithmetic, then the solve adjoint
// (three waves per SIMD: the few spilled values live outside the neighbour loop)
template <class R, bool kOff32>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(3))) void k_moments_bwd(
    Queue qu, int n, Lists L, const int32_t* __restrict__ perm, const uint4* __restrict__ quant,
    const R* __restrict__ aux, const RecQV<R>* __restrict__ qv, const R* __restrict__ h, int chunk,
    const R* __restrict__ cbar, RecMom<R>* __restrict__ mrec) {
    constexpr int kStage = stage_stride<RecQV<R>>();
    extern __shared__ uint4 stage_buf[];  // kStage per wave (stage_bytes)
    const int lane = lane_id();
    QState qs;
    for (int w = queue_start(qu, qs); w >= 0; w = queue_next(qu, qs)) {
        const int s = w * kWave + lane;
        const bool valid = s < n;
        const int i = valid ? perm[s] : 0;
        const R H = valid ? R(2) * h[i] : R(1);
        double S[29], M[40];
        int nnb = 0;
        moment_sums<R, kOff32>(w, s, valid, L, qv, stage_buf + wave_in_block() * kStage, H, chunk, S, nnb);
        moments_from_sums(S, M);
        if (valid) moments_adjoint_record(s, M, nnb, quant, aux, cbar, mrec);
    }
}

// 2'. the same from the forward's stored moment sums (one thread per particle)
template <class R>
__global__ __launch_bounds__(256) void k_moments_bwd_stored(int n, const int32_t* __restrict__ perm,
                                                            const uint4* __restrict__ quant,
                                                            const R* __restrict__ aux,
                                                            const double* __restrict__ sums,
                                                            const R* __restrict__ cbar,
                                                            RecMom<R>* __restrict__ mrec) {
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= n) return;
    const int i = perm[s];
    double S[29], M[40];
    for (int e = 0; e < 29; ++e) S[e] = sums[int64_t(e) * n + i];
    const int nnb = int(sums[int64_t(29) * n + i]);
    moments_from_sums(S, M);
    moments_adjoint_record(s, M, nnb, quant, aux, cbar, mrec);
}

// 3. moments adjoint, then the per-particle volume/pressure adjoints
template <class R, bool kOff32>
__global__ __launch_bounds__(256) void k_moments_adj(Queue qu, int n, Lists L, const int32_t* __restrict__ perm,
                                                     const RecMom<R>* __restrict__ mrec,
                                                     const R* __restrict__ vpbar, const R* __restrict__ m,
                                                     const R* __restrict__ u, const R* __restrict__ rho, R gm1,
                                                     int chunk, R* __restrict__ xbar, RecVA<R>* __restrict__ varec,
                                                     R* __restrict__ gu, const R* __restrict__ qbar = nullptr) {
    constexpr int kStage = stage_stride<RecMom<R>>();
    extern __shared__ uint4 stage_buf[];  // kStage per wave (stage_bytes)
    const int lane = lane_id();
    QState qs;
    for (int w = queue_start(qu, qs); w >= 0; w = queue_next(qu, qs)) {
        const int s = w * kWave + lane;
        const bool valid = s < n;
        const RecMom<R> ri = mrec[valid ? s : 0];
        const R invHi = ri.invH, Vi = ri.V;
        const R i2 = invHi * invHi;

        const int cnt = valid ? L.cnt[s] : 0;
        const int len = L.len[w];
        ChunkSums<R, 4> acc;  // Vbar, xbar[3]
        acc.zero();
        staged_list<RecMom<R>, kOff32, false>(  // measured faster with fixed LDS addresses
            L, w, cnt, len, mrec, stage_buf + wave_in_block() * kStage,
            [&](const RecMom<R>& rj, int k) __attribute__((always_inline)) {
                const R x[3] = {sep<R>(ri.q[0], rj.q[0]), sep<R>(ri.q[1], rj.q[1]), sep<R>(ri.q[2], rj.q[2])};
                const R y[3] = {-x[0], -x[1], -x[2]};
                const R r = dsqrt(x[0] * x[0] + x[1] * x[1] + x[2] * x[2]);
                R w_, f_, f2_;
                // own moments: M_i contains V_j phi(x_ij, h_i)
                shapes(r * invHi, w_, f_, f2_);
                R Phi, g[3];
                moment_phi(ri.c, w_, f_, f2_, i2, x, Phi, g);
                const R xb[3] = {rj.V * g[0], rj.V * g[1], rj.V * g[2]};
                // the neighbour's moments contain V_i phi(x_ji, h_j)
                const R invHj = rj.invH;
                const R j2 = invHj * invHj;
                shapes(r * invHj, w_, f_, f2_);
                moment_phi(rj.c, w_, f_, f2_, j2, y, Phi, g);
                acc.add(0, Phi);
#pragma unroll
                for (int c = 0; c < 3; ++c) acc.add(1 + c, xb[c] - Vi * g[c]);
                acc.next(k, chunk);
            });
        acc.fold();
        if (valid) {
            const int i = perm[s];
            // j = i term of the own moments: V_i phi(0) = V_i W(0) P0
            const double Vbar = double(acc.get(0)) + double(ri.c[0]) + double(vpbar[2 * s]);
            const double Pbar = double(vpbar[2 * s + 1]);
            // qbar: dL/drho and dL/du through the viscosity (tree order)
            const double rhobar = double(gm1) * double(u[i]) * Pbar + (qbar ? double(qbar[2 * s]) : 0.0);
            const double Sbar = -Vbar * double(Vi) * double(Vi) + double(m[i]) * rhobar;
            RecVA<R> va{};
            va.q[0] = ri.q[0]; va.q[1] = ri.q[1]; va.q[2] = ri.q[2];
            va.invH = invHi;
            va.Sbar = R(Sbar);
            varec[s] = va;
            gu[i] = R(double(gm1) * double(rho[i]) * Pbar + (qbar ? double(qbar[2 * s + 1]) : 0.0));
#pragma unroll
            for (int c = 0; c < 3; ++c) xbar[4 * s + c] += acc.get(1 + c);
        }
    }
}

// Extras adjoint (viscous chain).  The velocity gradients
//   dv_k[a][c] = sum_{j != k, r < H_k} V_j (v_j^a - v_k^a) G_kj^c
// (G_kj the corrected kernel gradient of particle k at x_kj) enter the force
// pass; given their adjoints dvb, each lane gathers the adjoints of its own
// particle's inputs from its own sum (through G_ij: corrections and x_i; and
// -v_i) and from every neighbour's sum that contains it (V_i, v_i, and x_i
// through G_ji).  Beyond a support W, F and F2 vanish, so every pair of the
// force list is taken whole.  Adds to cbar, vpbar (Vbar), xbar (tree order)
// and gv (caller order).
template <class R>
__global__ void k_pack_exa(int n, const int32_t* perm, const uint4* quant, const R* h, const R* vx, const R* vy,
                           const R* vz, const R* V, const R* A, const R* B, const R* dA, const R* dB,
                           const R* dvbar, RecExA<R>* rec) {
    __shared__ uint4 buf[256 * (sizeof(RecExA<R>) / 16)];
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    const bool valid = s < n;
    const int i = valid ? perm[s] : 0;
    const int sv = valid ? s : 0;
    RecExA<R> r;
    const uint4 q = quant[sv];
    r.q[0] = q.x; r.q[1] = q.y; r.q[2] = q.z;
    const R H = R(2) * h[i];
    const R invH = R(1) / H;
    r.invH = invH;
    r.V = V[i];
    r.A = A[i];
    r.cW = norm_W(H);
    r.cF = norm_F(H);
    const R i2 = invH * invH;
    r.cF2 = R(17325.0 / (2.0 * kPi)) * i2 * i2 * i2 * invH;
    for (int a = 0; a < 3; ++a) {
        r.B[a] = B[3 * i + a];
        r.dA[a] = dA[3 * i + a];
    }
    for (int k = 0; k < 9; ++k) {
        r.dB[k] = dB[9 * i + k];
        r.dvb[k] = dvbar[9 * sv + k];
    }
    r.v[0] = vx[i]; r.v[1] = vy[i]; r.v[2] = vz[i];
    const int first = blockIdx.x * blockDim.x;
    store_records(rec, r, valid, first, min(int(blockDim.x), n - first), buf);
}

template <class R, bool kOff32>
__global__ __launch_bounds__(256) void k_extras_adj(Queue qu, int n, Lists L, const int32_t* __restrict__ perm,
                                                    const RecExA<R>* __restrict__ rec, int chunk,
                                                    R* __restrict__ cbar, R* __restrict__ vpbar,
                                                    R* __restrict__ xbar, R* __restrict__ gv) {
    constexpr int kStage = stage_stride<RecExA<R>>();
    extern __shared__ uint4 stage_buf[];  // kStage per wave (stage_bytes)
    const int lane = lane_id();
    QState qs;
    for (int w = queue_start(qu, qs); w >= 0; w = queue_next(qu, qs)) {
        const int s = w * kWave + lane;
        const bool valid = s < n;
        const RecExA<R> ri = rec[valid ? s : 0];
        const int cnt = valid ? L.cnt[s] : 0;
        const int len = L.len[w];
        ChunkSums<R, 16> cb;  // A, B[3], dA[3], dB[9]
        ChunkSums<R, 7> ob;   // Vbar, xbar[3], vbar[3]
        cb.zero();
        ob.zero();
        staged_list<RecExA<R>, kOff32, false>(
            L, w, cnt, len, rec, stage_buf + wave_in_block() * kStage,
            [&](const RecExA<R>& rj, int k) __attribute__((always_inline)) {
                const R x[3] = {sep<R>(ri.q[0], rj.q[0]), sep<R>(ri.q[1], rj.q[1]), sep<R>(ri.q[2], rj.q[2])};
                const R y[3] = {-x[0], -x[1], -x[2]};
                const R r = dsqrt(x[0] * x[0] + x[1] * x[1] + x[2] * x[2]);
                R wi, fi, f2i, wj, fj, f2j;
                shapes(r * ri.invH, wi, fi, f2i);
                shapes(r * rj.invH, wj, fj, f2j);
                const R Wi = ri.cW * wi, Fi = ri.cF * fi, F2i = ri.cF2 * f2i;
                const R Wj = rj.cW * wj, Fj = rj.cF * fj, F2j = rj.cF2 * f2j;
                const Side<R> si = side_terms(ri, x), sj = side_terms(rj, y);
                R Gi[3], Gj[3];
                corr_grad(ri, si, Wi, Fi, x, Gi);
                corr_grad(rj, sj, Wj, Fj, y, Gj);
                // own sum: V_j (v_j - v_i) (x) G_ij
                R g[3], gp[3], e[3], Vb = R(0);
#pragma unroll
                for (int a = 0; a < 3; ++a) e[a] = ri.v[a] - rj.v[a];
#pragma unroll
                for (int c = 0; c < 3; ++c) {
                    g[c] = -rj.V * (ri.dvb[c] * e[0] + ri.dvb[3 + c] * e[1] + ri.dvb[6 + c] * e[2]);
                    // the neighbour's sum: V_i (v_i - v_j) (x) G_ji, through x_ji = -x
                    gp[c] = -ri.V * (rj.dvb[c] * e[0] + rj.dvb[3 + c] * e[1] + rj.dvb[6 + c] * e[2]);
                }
#pragma unroll
                for (int a = 0; a < 3; ++a) {
                    const R ti = ri.dvb[3 * a] * Gi[0] + ri.dvb[3 * a + 1] * Gi[1] + ri.dvb[3 * a + 2] * Gi[2];
                    const R tj = rj.dvb[3 * a] * Gj[0] + rj.dvb[3 * a + 1] * Gj[1] + rj.dvb[3 * a + 2] * Gj[2];
                    ob.add(4 + a, ri.V * tj - rj.V * ti);  // vbar_i
                    Vb += e[a] * tj;
                }
                ob.add(0, Vb);
                const Dots<R> di = side_dots(ri, si, x, g), dj = side_dots(rj, sj, y, gp);
                corr_grad_dC(ri, si, di, Wi, Fi, x, g, cb);
                R xb[3] = {R(0), R(0), R(0)};
                corr_grad_dy(ri, si, di, Wi, Fi, F2i, x, g, xb);
                corr_grad_dy(rj, sj, dj, Wj, Fj, F2j, y, gp, xb);
#pragma unroll
                for (int c = 0; c < 3; ++c) ob.add(1 + c, xb[c]);
                cb.next(k, chunk);
                ob.next(k, chunk);
            });
        cb.fold();
        ob.fold();
        if (valid) {
            const int i = perm[s];
#pragma unroll
            for (int e = 0; e < 16; ++e) cbar[16 * s + e] += cb.get(e);
            vpbar[2 * s] += ob.get(0);
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                xbar[4 * s + c] += ob.get(1 + c);
                gv[3 * i + c] += ob.get(4 + c);
            }
        }
    }
}

// 4. volume adjoint; writes the position gradient in caller order
template <class R, bool kOff32>
__global__ __launch_bounds__(256) void k_volume_adj(Queue qu, int n, Lists L, const int32_t* __restrict__ perm,
                                                    const RecVA<R>* __restrict__ varec,
                                                    const R* __restrict__ xbar, int chunk,
                                                    R* __restrict__ gx) {
    constexpr int kStage = stage_stride<RecVA<R>>();
    extern __shared__ uint4 stage_buf[];  // kStage per wave (stage_bytes)
    const int lane = lane_id();
    QState qs;
    for (int w = queue_start(qu, qs); w >= 0; w = queue_next(qu, qs)) {
        const int s = w * kWave + lane;
        const bool valid = s < n;
        const RecVA<R> ri = varec[valid ? s : 0];
        const R invHi = ri.invH;
        const R i2 = invHi * invHi;
        const R cFi = R(-1155.0 / (4.0 * kPi)) * i2 * i2 * invHi;
        const R Sbi = ri.Sbar;
        const int cnt = valid ? L.cnt[s] : 0;
        const int len = L.len[w];
        ChunkSums<R, 3> acc;
        acc.zero();
        list_loop<RecVA<R>, kOff32>(
            L, w, cnt, len, varec, stage_buf + wave_in_block() * kStage,
            [&](const RecVA<R>& d, int k) __attribute__((always_inline)) {
                const R invHj = d.invH;
                const R x[3] = {sep<R>(ri.q[0], d.q[0]), sep<R>(ri.q[1], d.q[1]), sep<R>(ri.q[2], d.q[2])};
                const R r = dsqrt(x[0] * x[0] + x[1] * x[1] + x[2] * x[2]);
                R w_, fi, fj, f2_;
                shapes(r * invHi, w_, fi, f2_);
                shapes(r * invHj, w_, fj, f2_);
                const R j2 = invHj * invHj;
                const R cFj = R(-1155.0 / (4.0 * kPi)) * j2 * j2 * invHj;
                const R coef = Sbi * cFi * fi + d.Sbar * cFj * fj;
#pragma unroll
                for (int c = 0; c < 3; ++c) acc.add(c, coef * x[c]);
                acc.next(k, chunk);
            });
        acc.fold();
        if (valid) {
            const int i = perm[s];
#pragma unroll
            for (int c = 0; c < 3; ++c) gx[3 * i + c] = xbar[4 * s + c] + acc.get(c);
        }
    }
}

template <class T> T* carve(char*& p, size_t count) {
    T* r = reinterpret_cast<T*>(p);
    p += (count * sizeof(T) + 255) / 256 * 256;  // keep every array 256-byte aligned
    return r;
}

// scratch of one backward call: records and per-particle partial adjoints
// (visc: the larger force-adjoint records, reused by the extras adjoint, and
// the adjoints of the velocity gradients, rho and u through the viscosity)
template <class R> size_t scratch_bytes(int64_t n, bool visc) {
    const size_t per = (visc ? sizeof(RecBwdV<R>) : sizeof(RecBwd<R>)) + sizeof(RecMom<R>) + sizeof(RecQV<R>) +
                       sizeof(RecVA<R>) + sizeof(R) * (16 + 2 + 4 + 2 + (visc ? 9 + 2 : 0));
    return per * size_t(n) + 10 * 256;  // ten arrays, each on a 256-byte boundary
}

// dv, q: the viscous chain (velocity gradients from the Extras pass and the
// viscosity constants), else nullptr
template <class R>
int backward_impl(crk_leaves* L, const crk_gas* g, const R* V, const R* rho, const crk_corr* C,
                  double gamma, const R* ga, const R* gdu, R* gx, R* gv, R* gu, hipStream_t st,
                  const R* dv = nullptr, const crk_visc* q_visc = nullptr) {
    const int n = int(L->n);
    const bool visc = dv != nullptr;
    int rc = pack_positions<R>(L, g->x, g->y, g->z, static_cast<const R*>(g->h), st);
    if (rc) return rc;
    void* sp = nullptr;
    if ((rc = pass_scratch(L, scratch_bytes<R>(n, visc), &sp))) return rc;
    char* p = static_cast<char*>(sp);
    // the force adjoint's records; the extras adjoint's (viscous chain) reuse them
    void* rec_any = visc ? static_cast<void*>(carve<RecBwdV<R>>(p, n)) : static_cast<void*>(carve<RecBwd<R>>(p, n));
    RecBwd<R>* rec = static_cast<RecBwd<R>*>(rec_any);
    RecBwdV<R>* recv = static_cast<RecBwdV<R>*>(rec_any);
    R* dvbar = visc ? carve<R>(p, 9 * size_t(n)) : nullptr;
    R* qbar = visc ? carve<R>(p, 2 * size_t(n)) : nullptr;
    R* aux = carve<R>(p, 2 * size_t(n));
    RecQV<R>* qv = carve<RecQV<R>>(p, n);
    R* cbar = carve<R>(p, 16 * size_t(n));
    R* vpbar = carve<R>(p, 2 * size_t(n));
    R* xbar = carve<R>(p, 4 * size_t(n));
    RecMom<R>* mrec = carve<RecMom<R>>(p, n);
    RecVA<R>* varec = carve<RecVA<R>>(p, n);
    const R gm1 = R(gamma - 1.0);
    {
        TimeScope tp(L, st, CRK_K_PACK);
        const R *h = static_cast<const R*>(g->h), *u = static_cast<const R*>(g->u);
        const R *vx = static_cast<const R*>(g->vx), *vy = static_cast<const R*>(g->vy),
                *vz = static_cast<const R*>(g->vz), *m = static_cast<const R*>(g->m);
        const R *A = static_cast<const R*>(C->A), *B = static_cast<const R*>(C->B),
                *dA = static_cast<const R*>(C->dA), *dB = static_cast<const R*>(C->dB);
        if (visc)
            hipLaunchKernelGGL((k_pack_bwd<R, RecBwdV<R>>), dim3((n + 255) / 256), dim3(256), 0, st, n, L->perm,
                               L->quant, h, u, vx, vy, vz, m, V, rho, A, B, dA, dB, ga, gdu, gm1, dv, recv, aux);
        else
            hipLaunchKernelGGL((k_pack_bwd<R, RecBwd<R>>), dim3((n + 255) / 256), dim3(256), 0, st, n, L->perm,
                               L->quant, h, u, vx, vy, vz, m, V, rho, A, B, dA, dB, ga, gdu, gm1,
                               static_cast<const R*>(nullptr), rec, aux);
        hipLaunchKernelGGL(k_pack_qv<R>, dim3((n + 255) / 256), dim3(256), 0, st, n, L->perm, L->quant, V, qv);
    }
    LAUNCH_CHECK("pack backward");
    const int bw = L->tune.block_waves;
    const dim3 grid(grid_nwave(L)), block(kWave * bw);
    const Queue q = make_queue(L, L->order_pair);
    reset_queue(L, st);
    if (!visc) {
        TimeScope ts(L, st, CRK_K_ACCEL_ADJ);
        auto kern = off32<RecBwd<R>>(L) ? k_accel_adj<R, true> : k_accel_adj<R, false>;
        hipLaunchKernelGGL(kern, grid, block, stage_bytes<RecBwd<R>>(bw), st, q, n, lists(L),
                           L->perm, rec, L->tune.kahan_chunk, cbar, vpbar, xbar, gv);
    } else {
        TimeScope ts(L, st, CRK_K_ACCEL_ADJ);
        const ViscB<R> vq{R(q_visc->Cl), R(q_visc->Cq), R(q_visc->eps_q), R(0.5 * gamma * (gamma - 1.0))};
        auto kern = off32<RecBwdV<R>>(L) ? k_accel_adj_visc<R, true> : k_accel_adj_visc<R, false>;
        hipLaunchKernelGGL(kern, grid, block, stage_bytes<RecBwdV<R>>(bw), st, q, n, lists(L), L->perm, recv,
                           L->tune.kahan_chunk, cbar, vpbar, xbar, gv, vq, dvbar, qbar);
    }
    LAUNCH_CHECK("accel adjoint");
    if (visc) {
        // the Extras pass's velocity gradients: their adjoints, to the inputs
        RecExA<R>* erec = reinterpret_cast<RecExA<R>*>(rec_any);
        {
            TimeScope tp(L, st, CRK_K_PACK);
            hipLaunchKernelGGL(k_pack_exa<R>, dim3((n + 255) / 256), dim3(256), 0, st, n, L->perm, L->quant,
                               static_cast<const R*>(g->h), static_cast<const R*>(g->vx),
                               static_cast<const R*>(g->vy), static_cast<const R*>(g->vz), V,
                               static_cast<const R*>(C->A), static_cast<const R*>(C->B),
                               static_cast<const R*>(C->dA), static_cast<const R*>(C->dB), dvbar, erec);
        }
        LAUNCH_CHECK("pack extras adjoint");
        reset_queue(L, st);
        TimeScope ts(L, st, CRK_K_EXTRAS_ADJ);
        auto kern = off32<RecExA<R>>(L) ? k_extras_adj<R, true> : k_extras_adj<R, false>;
        hipLaunchKernelGGL(kern, grid, block, stage_bytes<RecExA<R>>(bw), st, q, n, lists(L), L->perm, erec,
                           L->tune.kahan_chunk, cbar, vpbar, xbar, gv);
        LAUNCH_CHECK("extras adjoint");
    }
    if (C->M) {
        TimeScope ts(L, st, CRK_K_SOLVE_ADJ);  // the forward's moment sums, stored
        hipLaunchKernelGGL(k_moments_bwd_stored<R>, dim3((n + 255) / 256), dim3(256), 0, st, n, L->perm,
                           L->quant, aux, C->M, cbar, mrec);
    } else {
        reset_queue(L, st);
        TimeScope ts(L, st, CRK_K_MOMENTS);  // the forward moments, recomputed
        auto kern = off32<RecQV<R>>(L) ? k_moments_bwd<R, true> : k_moments_bwd<R, false>;
        hipLaunchKernelGGL(kern, grid, block, stage_bytes<RecQV<R>>(bw), st, q, n,
                           lists_gather(L), L->perm, L->quant, aux, qv, static_cast<const R*>(g->h),
                           L->tune.kahan_chunk, cbar, mrec);
    }
    LAUNCH_CHECK("moments + solve adjoint");
    reset_queue(L, st);
    {
        TimeScope ts(L, st, CRK_K_MOMENTS_ADJ);
        auto kern = off32<RecMom<R>>(L) ? k_moments_adj<R, true> : k_moments_adj<R, false>;
        hipLaunchKernelGGL(kern, grid, block, stage_bytes<RecMom<R>>(bw), st, q, n, lists(L),
                           L->perm, mrec, vpbar, static_cast<const R*>(g->m), static_cast<const R*>(g->u),
                           rho, gm1, L->tune.kahan_chunk, xbar, varec, gu, static_cast<const R*>(qbar));
    }
    LAUNCH_CHECK("moments adjoint");
    reset_queue(L, st);
    {
        TimeScope ts(L, st, CRK_K_VOLUME_ADJ);
        auto kern = off32<RecVA<R>>(L) ? k_volume_adj<R, true> : k_volume_adj<R, false>;
        hipLaunchKernelGGL(kern, grid, block, stage_bytes<RecVA<R>>(bw), st, q, n, lists(L),
                           L->perm, varec, xbar, L->tune.kahan_chunk, gx);
    }
    LAUNCH_CHECK("volume adjoint");
    return CRK_OK;
}

}  // namespace

size_t crk::backward_scratch_bytes(int64_t n, bool f64) {
    return f64 ? scratch_bytes<double>(n, true) : scratch_bytes<float>(n, true);
}

extern "C" int crk_accel_energy_backward(crk_leaves* L, const crk_gas* g, const void* V,
                                         const void* rho, const crk_corr* C, double gamma,
                                         const void* ga, const void* gdudt, crk_prec prec, void* gx,
                                         void* gv, void* gu, hipStream_t st) {
    int rc = check_gas(L, g, true);
    if (rc) return rc;
    if (L->n == 0) return CRK_OK;
    if (!V || !rho || !C || !C->A || !C->B || !C->dA || !C->dB || !ga || !gdudt || !gx || !gv || !gu)
        return fail(CRK_EINVAL, "V, rho, corrections, upstream adjoints and all gradients are required");
    if (prec == CRK_F32)
        return backward_impl<float>(L, g, (const float*)V, (const float*)rho, C, gamma, (const float*)ga,
                                    (const float*)gdudt, (float*)gx, (float*)gv, (float*)gu, st);
    if (prec == CRK_F64)
        return backward_impl<double>(L, g, (const double*)V, (const double*)rho, C, gamma,
                                     (const double*)ga, (const double*)gdudt, (double*)gx, (double*)gv,
                                     (double*)gu, st);
    return fail(CRK_EINVAL, "unknown precision");
}

extern "C" int crk_accel_energy_visc_backward(crk_leaves* L, const crk_gas* g, const void* V, const void* rho,
                                              const crk_corr* C, const void* dv, const crk_visc* q, double gamma,
                                              const void* ga, const void* gdudt, crk_prec prec, void* gx, void* gv,
                                              void* gu, hipStream_t st) {
    int rc = check_gas(L, g, true);
    if (rc) return rc;
    if (!q) return fail(CRK_EINVAL, "viscosity parameters are required");
    if (!(q->Cl >= 0.0) || !(q->Cq >= 0.0) || !(q->eps_q > 0.0))
        return fail(CRK_EINVAL, "viscosity needs Cl >= 0, Cq >= 0 and eps_q > 0");
    if (!(gamma > 1.0)) return fail(CRK_EINVAL, "gamma must exceed 1 (the sound speed)");
    if (L->n == 0) return CRK_OK;
    if (!V || !rho || !C || !C->A || !C->B || !C->dA || !C->dB || !dv || !ga || !gdudt || !gx || !gv || !gu)
        return fail(CRK_EINVAL, "V, rho, corrections, dv, upstream adjoints and all gradients are required");
    if (prec == CRK_F32)
        return backward_impl<float>(L, g, (const float*)V, (const float*)rho, C, gamma, (const float*)ga,
                                    (const float*)gdudt, (float*)gx, (float*)gv, (float*)gu, st, (const float*)dv, q);
    if (prec == CRK_F64)
        return backward_impl<double>(L, g, (const double*)V, (const double*)rho, C, gamma, (const double*)ga,
                                     (const double*)gdudt, (double*)gx, (double*)gv, (double*)gu, st,
                                     (const double*)dv, q);
    return fail(CRK_EINVAL, "unknown precision");
}
