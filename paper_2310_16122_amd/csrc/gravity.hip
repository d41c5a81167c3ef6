// Short-range particle-particle gravity for MI355X (gfx950): the pair pass,
// its adjoint, and the polynomial fit of the particle-mesh force it subtracts.
//
// The paper splits the gravitational force into a long-range part solved on a
// particle mesh (FFT) and a short-range part evaluated by direct summation
// over particle pairs within a cutoff, with the grid force represented in the
// short-range kernel by a fifth-order polynomial (Sec. 3.1; the build option
// HACC_CUDA_POLY_ORDER=5 in the appendix).  Here the pair kernel is
//   a_i = -G sum_{j != i, r_ij < r_c} m_j x_ij [(r^2 + eps^2)^(-3/2) - P(r^2)],
// P(s) = sum_k p_k s^k, over every species, on tiles of 64 particles in tree
// order that stream the leaves within r_c of their box.

#include <cstring>
#include <type_traits>
#include <vector>

#include "crk_internal.h"

using namespace crk;

namespace {

struct GravParams {
    double G, eps2, rc2;
    double poly[6];
    int use_poly;
};

// Staged candidates: position relative to the tile origin and mass (forward);
// the adjoint also carries the candidate's upstream adjoint dL/da_j.
template <class R> struct alignas(4 * sizeof(R)) GravRec {
    R x, y, z, m;
};
template <class R> struct alignas(8 * sizeof(R)) GravAdjRec {
    R x, y, z, m;
    R gx, gy, gz, pad;
};

// The softened kernel and its s = r^2 derivative: phi = (s + eps^2)^(-3/2) - P(s),
// dphi = -3/2 (s + eps^2)^(-5/2) - P'(s).
template <class R, bool kPoly, bool kDeriv>
__device__ __forceinline__ void grav_phi(R r2, R eps2, const R pc[6], R& phi, R& dphi) {
    const R ir = drsqrt(r2 + eps2);
    const R ir2 = ir * ir;
    phi = ir2 * ir;
    if (kDeriv) dphi = R(-1.5) * phi * ir2;
    if (kPoly) {
        R pv = pc[5];
#pragma unroll
        for (int k = 4; k >= 0; --k) pv = pv * r2 + pc[k];
        phi -= pv;
        if (kDeriv) {
            R dv = R(5) * pc[5];
#pragma unroll
            for (int k = 4; k >= 1; --k) dv = dv * r2 + R(k) * pc[k];
            dphi -= dv;
        }
    }
}

// How the kept candidates of a block reach the lanes that evaluate them -- the
// exchange variants the paper compares for its pair kernels (local memory,
// broadcasts, cross-lane shuffles; Sec. 5.3), here on gfx950:
//   kExLds:    compacted into LDS, every lane reads the same entry (an LDS broadcast);
//   kExSgpr:   left in the lanes that loaded them; the wave walks the kept
//              lanes with a scalar loop and v_readlane moves each candidate into
//              scalar registers, which every lane's arithmetic reads directly;
//   kExPermute: the same walk, each candidate fetched by every lane with
//              ds_bpermute (the select-from-group form).
// The same candidates are evaluated in the same order with the compensated
// fold after every kChunk of them (counted over the whole stream), so the
// three give the same sums bit for bit.
constexpr int kExLds = 0, kExSgpr = 1, kExPermute = 2;

template <int kEx, class T> __device__ __forceinline__ T lane_value(T v, int k) {
    static_assert(sizeof(T) == 4 || sizeof(T) == 8, "32- or 64-bit values");
    if constexpr (sizeof(T) == 4) {
        int b;
        __builtin_memcpy(&b, &v, 4);
        b = kEx == kExSgpr ? __builtin_amdgcn_readlane(b, k) : __builtin_amdgcn_ds_bpermute(k << 2, b);
        T r;
        __builtin_memcpy(&r, &b, 4);
        return r;
    } else {
        int b[2];
        __builtin_memcpy(b, &v, 8);
        for (int h = 0; h < 2; ++h)
            b[h] = kEx == kExSgpr ? __builtin_amdgcn_readlane(b[h], k) : __builtin_amdgcn_ds_bpermute(k << 2, b[h]);
        T r;
        __builtin_memcpy(&r, b, 8);
        return r;
    }
}

// A whole record (or position) from lane k, field by field.
template <int kEx, class Rec> __device__ __forceinline__ Rec lane_record(const Rec& v, int k) {
    static_assert(sizeof(Rec) % 4 == 0, "whole dwords");
    constexpr int kWords = int(sizeof(Rec) / 4);
    int w[kWords];
    __builtin_memcpy(w, &v, sizeof(Rec));
#pragma unroll
    for (int h = 0; h < kWords; ++h) w[h] = lane_value<kEx>(w[h], k);
    Rec r;
    __builtin_memcpy(&r, w, sizeof(Rec));
    return r;
}

// One wave per tile: streams the tile's candidate blocks of 64 (the next
// block's loads are issued before the current one is evaluated), keeps the
// candidates that can interact with some lane, and evaluates them against
// every lane.  Positions are taken relative to the tile's first particle as
// reals, so a pair's separation is three subtractions: for a compact tile
// (every lane within 1/4 of that origin, r_c < 1/4) the relative coordinates
// of every pair within r_c are exact minimum images and every pair beyond r_c
// stays beyond it; other tiles use the exact fixed-point separation.  In a
// compact tile a candidate farther than r_c from the tile's bounding box
// cannot interact with any lane and is dropped before it reaches LDS; the
// survivors are appended (ballot + mbcnt) to an LDS queue of up to 2 x 64
// entries that carries over from block to block, whole chunks of kChunk are
// evaluated in straight-line code with fold() after each once 64 are queued
// (the remainder moves to the front), and the last partial chunk is padded
// with `pad` records (far away, massless).  The chunks are thus the kept
// candidates in stream order, eight at a time, whatever the block sizes.
//   load(j): the candidate's record with its non-positional fields set;
//   eval(rec, dx, dy, dz): one pair, x_ij = (dx, dy, dz).
template <class R, class Rec, int kChunk, int kEx, class Load, class Eval, class Fold>
__device__ __forceinline__ void gravity_tile(int w, int n, const uint4* __restrict__ quant,
                                             const int32_t* __restrict__ rng_off,
                                             const int2* __restrict__ rng, R rc2, Rec* srec, uint4* sq,
                                             const Rec& pad, Load load, Eval eval, Fold fold) {
    const int lane = lane_id();
    const int s = w * kWave + lane;
    const bool valid = s < n;
    // the box test keeps a margin over the pair test so rounding never drops
    // a candidate that some lane would count
    const R keep2 = rc2 * R(1.001);
    const uint4 qo = quant[w * kWave];  // tile origin (wave-uniform)
    const uint4 qi = valid ? quant[s] : qo;
    const R xi = sep<R>(qi.x, qo.x), yi = sep<R>(qi.y, qo.y), zi = sep<R>(qi.z, qo.z);
    const bool far = fmax(fabs(xi), fmax(fabs(yi), fabs(zi))) >= R(0.25);
    const bool compact = __ballot(far) == 0 && rc2 < R(0.0625);
    R lo[3] = {xi, yi, zi}, hi[3] = {xi, yi, zi};
#pragma unroll
    for (int o = 32; o > 0; o >>= 1)
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            lo[c] = fmin(lo[c], R(__shfl_xor(lo[c], o)));
            hi[c] = fmax(hi[c], R(__shfl_xor(hi[c], o)));
        }
    // candidate blocks: range r, block [b, min(b + 64, e))
    auto uni = [](int v) __attribute__((always_inline)) { return __builtin_amdgcn_readfirstlane(v); };
    const int r1 = uni(rng_off[w + 1]);
    int r = uni(rng_off[w]), b = 0, e = 0;
    if (r < r1) { const int2 g = rng[r]; b = uni(g.x); e = uni(g.y); }
    uint4 nq = qo;
    Rec nrec = pad;
    if (r < r1 && lane < e - b) { nq = quant[b + lane]; nrec = load(b + lane); }
    int done = 0;  // walk forms: candidates evaluated since the last fold
    int have = 0;  // LDS form: candidates queued
    // evaluates the first `count` queued entries (a multiple of kChunk)
    auto eval_queued = [&](int count) __attribute__((always_inline)) {
        if (compact) {
            for (int j0 = 0; j0 < count; j0 += kChunk) {
#pragma unroll
                for (int u = 0; u < kChunk; ++u) {
                    const Rec c = srec[j0 + u];
                    eval(c, xi - c.x, yi - c.y, zi - c.z);
                }
                fold();
            }
        } else {
            for (int j0 = 0; j0 < count; j0 += kChunk) {
#pragma unroll
                for (int u = 0; u < kChunk; ++u) {
                    const uint4 c = sq[j0 + u];
                    eval(srec[j0 + u], sep<R>(qi.x, c.x), sep<R>(qi.y, c.y), sep<R>(qi.z, c.z));
                }
                fold();
            }
        }
    };
    while (r < r1) {
        const int mcnt = min(kWave, e - b);
        const uint4 qj = nq;
        Rec g = nrec;
        // advance and prefetch the next block
        int nb = b + kWave, ne = e, nr = r;
        if (nb >= ne) {
            ++nr;
            if (nr < r1) { const int2 gg = rng[nr]; nb = uni(gg.x); ne = uni(gg.y); }
        }
        if (nr < r1 && lane < ne - nb) { nq = quant[nb + lane]; nrec = load(nb + lane); }
        r = nr; b = nb; e = ne;

        g.x = sep<R>(qj.x, qo.x);
        g.y = sep<R>(qj.y, qo.y);
        g.z = sep<R>(qj.z, qo.z);
        bool keep = lane < mcnt;
        if (compact && keep) {
            const R d0 = fmax(fmax(lo[0] - g.x, g.x - hi[0]), R(0));
            const R d1 = fmax(fmax(lo[1] - g.y, g.y - hi[1]), R(0));
            const R d2 = fmax(fmax(lo[2] - g.z, g.z - hi[2]), R(0));
            keep = d0 * d0 + d1 * d1 + d2 * d2 < keep2;
        }
        const uint64_t mask = __ballot(keep);
        if (mask == 0) continue;
        if constexpr (kEx != kExLds) {
            // walk the kept lanes in lane order (the LDS form's compacted order)
            uint64_t left = mask;
            while (left) {
                const int k = __builtin_amdgcn_readfirstlane(int(__builtin_ctzll(left)));
                left &= left - 1;
                const Rec c = lane_record<kEx>(g, k);
                if (compact) {
                    eval(c, xi - c.x, yi - c.y, zi - c.z);
                } else {
                    const uint4 qc = lane_record<kEx>(qj, k);
                    eval(c, sep<R>(qi.x, qc.x), sep<R>(qi.y, qc.y), sep<R>(qi.z, qc.z));
                }
                if (++done == kChunk) {
                    fold();
                    done = 0;
                }
            }
            continue;
        }
        const int cnt = __popcll(mask);
        const int pos = __builtin_amdgcn_mbcnt_hi(uint32_t(mask >> 32),
                                                  __builtin_amdgcn_mbcnt_lo(uint32_t(mask), 0u));
        __syncthreads();  // queued entries moved by the previous step are in place
        if (keep) { srec[have + pos] = g; sq[have + pos] = qj; }
        have += cnt;  // < 2 x 64: fewer than 64 were queued before
        __syncthreads();
        if (have >= kWave) {
            const int whole = have / kChunk * kChunk;
            eval_queued(whole);
            // the remainder (fewer than kChunk) to the front
            const int rest = have - whole;
            Rec tr = pad;
            uint4 tq = qo;
            if (lane < rest) { tr = srec[whole + lane]; tq = sq[whole + lane]; }
            __syncthreads();
            if (lane < rest) { srec[lane] = tr; sq[lane] = tq; }
            have = rest;
        }
    }
    if constexpr (kEx != kExLds) {
        if (done) fold();  // the LDS form pads the last chunk with zeros, then folds
    } else if (have > 0) {
        const int padded = (have + kChunk - 1) / kChunk * kChunk;
        __syncthreads();
        if (lane >= have && lane < padded) {
            srec[lane] = pad;
            sq[lane] = qo;
        }
        __syncthreads();
        eval_queued(padded);
    }
}

// Forward pass: a_i.
template <class R, bool kPoly, bool kSoft, int kEx>
__global__ __launch_bounds__(64) void k_gravity(Queue qu, int n, const int32_t* __restrict__ perm,
                                                const uint4* __restrict__ quant, const R* __restrict__ ms,
                                                const int32_t* __restrict__ rng_off,
                                                const int2* __restrict__ rng, GravParams gp,
                                                R* __restrict__ a_out) {
    constexpr bool kComp = sizeof(R) == 4;
    __shared__ GravRec<R> srec[2 * kWave];
    __shared__ uint4 sq[2 * kWave];
    const int lane = lane_id();
    const R rc2 = R(gp.rc2), eps2 = R(gp.eps2);
    R pc[6];
    for (int k = 0; k < 6; ++k) pc[k] = R(gp.poly[k]);
    QState qs;
    for (int wq = queue_start(qu, qs); wq >= 0; wq = queue_next(qu, qs)) {
        const int w = __builtin_amdgcn_readfirstlane(wq);
        R acc[3] = {R(0), R(0), R(0)}, cmp[3] = {R(0), R(0), R(0)}, part[3] = {R(0), R(0), R(0)};
        gravity_tile<R, GravRec<R>, 8, kEx>(
            w, n, quant, rng_off, rng, rc2, srec, sq, GravRec<R>{R(2), R(2), R(2), R(0)},
            [&](int j) __attribute__((always_inline)) { return GravRec<R>{R(0), R(0), R(0), ms[j]}; },
            [&](const GravRec<R>& c, R dx, R dy, R dz) __attribute__((always_inline)) {
                const R r2 = dx * dx + dy * dy + dz * dz;
                // with softening a coincident pair (the self pair included) has a
                // finite f and a zero separation, so it adds exactly zero
                const bool in = kSoft ? r2 < rc2 : (r2 < rc2 && r2 > R(0));
                R f, df;
                grav_phi<R, kPoly, false>(r2, eps2, pc, f, df);
                f = in ? c.m * f : R(0);
                part[0] += f * dx;
                part[1] += f * dy;
                part[2] += f * dz;
            },
            [&]() __attribute__((always_inline)) {
                if (kComp)
                    for (int c = 0; c < 3; ++c) { kadd(acc[c], cmp[c], part[c]); part[c] = R(0); }
            });
        const int s = w * kWave + lane;
        if (s < n) {
            const int i = perm[s];
            for (int c = 0; c < 3; ++c) {
                const R tot = kComp ? (acc[c] - cmp[c]) : part[c];
                a_out[3 * i + c] = R(-gp.G) * tot;
            }
        }
    }
}

// Adjoint: with abar = dL/da, per pair (x = x_ij, s = r^2, d = m_j abar_i - m_i abar_j)
//   dL/dx_i = -G sum_j [phi d + 2 phi'(s) (x . d) x],
// the derivative of both a_i (through x_ij) and a_j (through x_ji = -x_ij).
// Each lane accumulates its own particle's adjoint from its neighbours'
// masses and upstream adjoints: no atomics.
template <class R, bool kPoly, bool kSoft, int kEx>
__global__ __launch_bounds__(64) void k_gravity_adj(Queue qu, int n, const int32_t* __restrict__ perm,
                                                    const uint4* __restrict__ quant,
                                                    const R* __restrict__ mg,  // [4n]: m, abar (tree order)
                                                    const int32_t* __restrict__ rng_off,
                                                    const int2* __restrict__ rng, GravParams gp,
                                                    R* __restrict__ gx_out) {
    constexpr bool kComp = sizeof(R) == 4;
    __shared__ GravAdjRec<R> srec[2 * kWave];
    __shared__ uint4 sq[2 * kWave];
    const int lane = lane_id();
    const R rc2 = R(gp.rc2), eps2 = R(gp.eps2);
    R pc[6];
    for (int k = 0; k < 6; ++k) pc[k] = R(gp.poly[k]);
    QState qs;
    for (int wq = queue_start(qu, qs); wq >= 0; wq = queue_next(qu, qs)) {
        const int w = __builtin_amdgcn_readfirstlane(wq);
        const int s = w * kWave + lane;
        const bool valid = s < n;
        const R mi = valid ? mg[s] : R(0);
        const R ai[3] = {valid ? mg[n + s] : R(0), valid ? mg[2 * n + s] : R(0), valid ? mg[3 * n + s] : R(0)};
        R acc[3] = {R(0), R(0), R(0)}, cmp[3] = {R(0), R(0), R(0)}, part[3] = {R(0), R(0), R(0)};
        gravity_tile<R, GravAdjRec<R>, 8, kEx>(
            w, n, quant, rng_off, rng, rc2, srec, sq,
            GravAdjRec<R>{R(2), R(2), R(2), R(0), R(0), R(0), R(0), R(0)},
            [&](int j) __attribute__((always_inline)) {
                return GravAdjRec<R>{R(0), R(0), R(0), mg[j], mg[n + j], mg[2 * n + j], mg[3 * n + j], R(0)};
            },
            [&](const GravAdjRec<R>& c, R dx, R dy, R dz) __attribute__((always_inline)) {
                const R r2 = dx * dx + dy * dy + dz * dz;
                const bool in = kSoft ? r2 < rc2 : (r2 < rc2 && r2 > R(0));
                R phi, dphi;
                grav_phi<R, kPoly, true>(r2, eps2, pc, phi, dphi);
                // selected before use: phi is infinite for an excluded coincident pair
                phi = in ? phi : R(0);
                dphi = in ? dphi : R(0);
                R d[3];
                {
                    // each product rounded on its own: the self pair gives d = 0 exactly
#pragma clang fp contract(off)
                    d[0] = c.m * ai[0] - mi * c.gx;
                    d[1] = c.m * ai[1] - mi * c.gy;
                    d[2] = c.m * ai[2] - mi * c.gz;
                }
                const R t = R(2) * dphi * (dx * d[0] + dy * d[1] + dz * d[2]);
                part[0] += phi * d[0] + t * dx;
                part[1] += phi * d[1] + t * dy;
                part[2] += phi * d[2] + t * dz;
            },
            [&]() __attribute__((always_inline)) {
                if (kComp)
                    for (int c = 0; c < 3; ++c) { kadd(acc[c], cmp[c], part[c]); part[c] = R(0); }
            });
        if (valid) {
            const int i = perm[s];
            for (int c = 0; c < 3; ++c) {
                const R tot = kComp ? (acc[c] - cmp[c]) : part[c];
                gx_out[3 * i + c] = R(-gp.G) * tot;
            }
        }
    }
}

// masses and upstream adjoints into tree order, [4n]: m, abar_x, abar_y, abar_z
template <class R>
__global__ void k_pack_grav_adj(int n, const int32_t* __restrict__ perm, const R* __restrict__ m,
                                const R* __restrict__ ga, R* __restrict__ out) {
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= n) return;
    const int i = perm[s];
    out[s] = m[i];
    out[n + s] = ga[3 * i + 0];
    out[2 * n + s] = ga[3 * i + 1];
    out[3 * n + s] = ga[3 * i + 2];
}

// softening large enough that a coincident pair's f = m eps^-3 is no larger
// than a real close pair's (eps^-3 <= 2^120 in FP32)
template <class R> bool softened(const GravParams& gp) { return R(gp.eps2) >= R(0x1p-80); }

// The instantiation for a launch: polynomial term or not, softened or not,
// exchange variant.  make(poly, soft, ex) receives std::integral_constant tags.
template <class R, class Make> auto pick(const GravParams& gp, int exchange, Make make) {
    using T = std::true_type;
    using F = std::false_type;
    auto by_ex = [&](auto poly, auto soft) {
        return exchange == kExSgpr      ? make(poly, soft, std::integral_constant<int, kExSgpr>{})
               : exchange == kExPermute ? make(poly, soft, std::integral_constant<int, kExPermute>{})
                                        : make(poly, soft, std::integral_constant<int, kExLds>{});
    };
    const bool soft = softened<R>(gp);
    return gp.use_poly ? (soft ? by_ex(T{}, T{}) : by_ex(T{}, F{})) : (soft ? by_ex(F{}, T{}) : by_ex(F{}, F{}));
}

template <class R>
int gravity_impl(crk_leaves* L, const double* x, const double* y, const double* z, const R* m,
                 const GravParams& gp, R* a, hipStream_t st) {
    const int n = int(L->n);
    int rc = pack_positions<R>(L, x, y, z, nullptr, st);
    if (rc) return rc;
    void* sp = nullptr;
    if ((rc = pass_scratch(L, sizeof(R) * size_t(n), &sp))) return rc;
    R* ms = static_cast<R*>(sp);
    {
        TimeScope tp(L, st, CRK_K_PACK);
        hipLaunchKernelGGL(k_gather<R>, dim3((n + 255) / 256), dim3(256), 0, st, n, L->perm, m, ms);
    }
    LAUNCH_CHECK("gather m");
    reset_queue(L, st);
    TimeScope ts(L, st, CRK_K_GRAVITY);
    auto kern = pick<R>(gp, L->tune.exchange, [](auto poly, auto soft, auto ex) {
        return k_gravity<R, decltype(poly)::value, decltype(soft)::value, decltype(ex)::value>;
    });
    hipLaunchKernelGGL(kern, dim3(grid_1wave(L)), dim3(kWave), 0, st,
                       make_queue(L, L->order_cull), n, L->perm, L->quant, ms, L->rng_off, L->rng,
                       gp, a);
    LAUNCH_CHECK("gravity");
    return CRK_OK;
}

template <class R>
int gravity_backward_impl(crk_leaves* L, const double* x, const double* y, const double* z, const R* m,
                          const GravParams& gp, const R* ga, R* gx, hipStream_t st) {
    const int n = int(L->n);
    int rc = pack_positions<R>(L, x, y, z, nullptr, st);
    if (rc) return rc;
    void* sp = nullptr;
    if ((rc = pass_scratch(L, 4 * sizeof(R) * size_t(n), &sp))) return rc;
    R* mg = static_cast<R*>(sp);
    {
        TimeScope tp(L, st, CRK_K_PACK);
        hipLaunchKernelGGL(k_pack_grav_adj<R>, dim3((n + 255) / 256), dim3(256), 0, st, n, L->perm, m, ga, mg);
    }
    LAUNCH_CHECK("pack gravity adjoint");
    reset_queue(L, st);
    TimeScope ts(L, st, CRK_K_GRAVITY_ADJ);
    auto kern = pick<R>(gp, L->tune.exchange, [](auto poly, auto soft, auto ex) {
        return k_gravity_adj<R, decltype(poly)::value, decltype(soft)::value, decltype(ex)::value>;
    });
    hipLaunchKernelGGL(kern, dim3(grid_1wave(L)), dim3(kWave), 0, st,
                       make_queue(L, L->order_cull), n, L->perm, L->quant, mg, L->rng_off, L->rng,
                       gp, gx);
    LAUNCH_CHECK("gravity adjoint");
    return CRK_OK;
}

int gravity_args(crk_leaves* L, int64_t n, const double* x, const double* y, const double* z, const void* m,
                 double G, double eps, double r_cut, const double* poly, GravParams& gp) {
    if (!L) return fail(CRK_EINVAL, "null handle");
    if (n != L->n) return fail(CRK_EINVAL, "n does not match the handle");
    if (L->hydro) return fail(CRK_ESTATE, "gravity needs a handle built in fixed-radius mode");
    if (!(r_cut > 0.0) || r_cut > L->r_fixed)
        return fail(CRK_EINVAL, "r_cut must be in (0, r_fixed of the handle]");
    if (!(eps >= 0.0)) return fail(CRK_EINVAL, "eps must be >= 0");
    if (n > 0 && (!x || !y || !z || !m)) return fail(CRK_EINVAL, "x, y, z and m are required");
    gp.G = G;
    gp.eps2 = eps * eps;
    gp.rc2 = r_cut * r_cut;
    gp.use_poly = poly != nullptr;
    for (int k = 0; k < 6; ++k) gp.poly[k] = poly ? poly[k] : 0.0;
    return CRK_OK;
}

// ---------------------------------------------------------------- the particle-mesh force fit
// Long-range force per unit mass of a mesh potential filtered by exp(-k^2 r_s^2)
// (the potential of a Gaussian cloud of variance 2 r_s^2 per axis), over r:
//   g = f_L(r) / r,  f_L = [erf(x) - (2x/sqrt(pi)) exp(-x^2)] / r^2,  x = r / (2 r_s).
// The bracket equals (4/sqrt(pi)) int_0^x t^2 exp(-t^2) dt; its power series is
// used below x = 1/2, where the closed form loses digits to cancellation.
double long_range_over_r(double r, double r_s) {
    const double x = r / (2.0 * r_s);
    double F;
    if (x < 0.5) {
        // (4/sqrt(pi)) sum_k (-1)^k x^(2k+3) / (k! (2k+3))
        double term = x * x * x, sum = 0.0;
        for (int k = 0; k < 40; ++k) {
            const double t = term / double(2 * k + 3);
            sum += t;
            if (std::fabs(t) <= 1e-17 * std::fabs(sum)) break;
            term *= -x * x / double(k + 1);
        }
        F = 4.0 / std::sqrt(kPi) * sum;
    } else {
        F = std::erf(x) - 2.0 * x / std::sqrt(kPi) * std::exp(-x * x);
    }
    return F / (r * r * r);
}

// Weighted least squares by Householder QR: minimise sum_k [w_k (y_k - sum_m c_m t_k^m)]^2
// over 6 coefficients (K >= 6 rows).  Returns false if the system is rank deficient.
bool lsq6(int K, const double* t, const double* y, const double* w, double c[6]) {
    std::vector<double> A(size_t(K) * 6), b(K);
    for (int k = 0; k < K; ++k) {
        double p = w[k];
        for (int m = 0; m < 6; ++m) { A[size_t(k) * 6 + m] = p; p *= t[k]; }
        b[k] = w[k] * y[k];
    }
    double diag[6];
    for (int col = 0; col < 6; ++col) {
        double nrm = 0.0;
        for (int k = col; k < K; ++k) nrm += A[size_t(k) * 6 + col] * A[size_t(k) * 6 + col];
        nrm = std::sqrt(nrm);
        if (!(nrm > 0.0)) return false;
        const double a0 = A[size_t(col) * 6 + col];
        const double alpha = a0 > 0 ? -nrm : nrm;
        // v = column - alpha e_col, stored in place; H = I - 2 v v^T / (v^T v)
        A[size_t(col) * 6 + col] = a0 - alpha;
        double vv = 0.0;
        for (int k = col; k < K; ++k) vv += A[size_t(k) * 6 + col] * A[size_t(k) * 6 + col];
        for (int j = col + 1; j < 6; ++j) {
            double dot = 0.0;
            for (int k = col; k < K; ++k) dot += A[size_t(k) * 6 + col] * A[size_t(k) * 6 + j];
            const double f = 2.0 * dot / vv;
            for (int k = col; k < K; ++k) A[size_t(k) * 6 + j] -= f * A[size_t(k) * 6 + col];
        }
        double dot = 0.0;
        for (int k = col; k < K; ++k) dot += A[size_t(k) * 6 + col] * b[k];
        const double f = 2.0 * dot / vv;
        for (int k = col; k < K; ++k) b[k] -= f * A[size_t(k) * 6 + col];
        diag[col] = alpha;
    }
    for (int col = 5; col >= 0; --col) {
        double s = b[col];
        for (int j = col + 1; j < 6; ++j) s -= A[size_t(col) * 6 + j] * c[j];
        c[col] = s / diag[col];
    }
    return true;
}

}  // namespace

extern "C" {

int sr_gravity(crk_leaves* L, int64_t n, const double* x, const double* y, const double* z,
               const void* m, double G, double eps, double r_cut, const double* poly, crk_prec prec,
               void* a, hipStream_t st) {
    GravParams gp;
    int rc = gravity_args(L, n, x, y, z, m, G, eps, r_cut, poly, gp);
    if (rc) return rc;
    if (n == 0) return CRK_OK;
    if (!a) return fail(CRK_EINVAL, "a is required");
    if (prec == CRK_F32) return gravity_impl<float>(L, x, y, z, (const float*)m, gp, (float*)a, st);
    if (prec == CRK_F64) return gravity_impl<double>(L, x, y, z, (const double*)m, gp, (double*)a, st);
    return fail(CRK_EINVAL, "unknown precision");
}

int sr_gravity_backward(crk_leaves* L, int64_t n, const double* x, const double* y, const double* z,
                        const void* m, double G, double eps, double r_cut, const double* poly,
                        const void* ga, crk_prec prec, void* gx, hipStream_t st) {
    GravParams gp;
    int rc = gravity_args(L, n, x, y, z, m, G, eps, r_cut, poly, gp);
    if (rc) return rc;
    if (n == 0) return CRK_OK;
    if (!ga || !gx) return fail(CRK_EINVAL, "ga and gx are required");
    if (prec == CRK_F32)
        return gravity_backward_impl<float>(L, x, y, z, (const float*)m, gp, (const float*)ga, (float*)gx, st);
    if (prec == CRK_F64)
        return gravity_backward_impl<double>(L, x, y, z, (const double*)m, gp, (const double*)ga, (double*)gx,
                                             st);
    return fail(CRK_EINVAL, "unknown precision");
}

int sr_gravity_fit_poly(double r_s, double r_cut, int samples, double* poly) {
    if (!poly) return fail(CRK_EINVAL, "poly is NULL");
    if (!(r_s > 0.0) || !(r_cut > 0.0) || !std::isfinite(r_s) || !std::isfinite(r_cut))
        return fail(CRK_EINVAL, "r_s and r_cut must be positive and finite");
    if (samples < 6 || samples > (1 << 20)) return fail(CRK_EINVAL, "samples must be in [6, 2^20]");
    std::vector<double> t(samples), y(samples), w(samples);
    for (int k = 0; k < samples; ++k) {
        t[k] = (double(k) + 0.5) / double(samples);  // s / r_cut^2
        const double r = r_cut * std::sqrt(t[k]);
        y[k] = long_range_over_r(r, r_s);
        w[k] = r * r * r;  // error of the pair force relative to the Newtonian one
    }
    double c[6];
    if (!lsq6(samples, t.data(), y.data(), w.data(), c)) return fail(CRK_EINVAL, "rank-deficient fit");
    double sc = 1.0;
    for (int k = 0; k < 6; ++k) {
        poly[k] = c[k] / sc;
        sc *= r_cut * r_cut;
    }
    return CRK_OK;
}

}  // extern "C"
