// CRK-SPH pair passes and short-range gravity for MI355X (gfx950): forward
// kernels, tree and list build, and the C ABI.
//
// Layout.  Particles are reordered along the RCB tree (tree.cpp).  Tree order
// is cut into tiles of 64 consecutive particles; a tile is the unit of work of
// one wavefront, one particle per lane.  Positions are 32-bit fixed point in
// the unit periodic box, so a separation is an exact signed 32-bit difference
// that wraps to the minimum image by itself.
//
// Interaction lists.  For the CRK passes every tile owns a wave-interleaved
// neighbour list: entry k of lane l lives at off[tile] + 64 k + l, so the 64
// lanes of a wave read their k-th neighbours with one coalesced load.  The
// list is built once per tree by streaming the tile's candidate leaves through
// LDS and testing every pair (count pass, host prefix sum, fill pass); all
// three forward passes reuse it.  Short-range gravity has no list: each tile
// streams its candidate leaves through LDS and evaluates every candidate pair
// branch-free with a cutoff mask.
//
// Work distribution.  Tiles are issued in decreasing-cost order (longest
// processing time first) either one per wave or through a persistent grid in
// which every wave pulls the next tile from an atomic counter.
//
// Precision.  Each pass is a template on the real type R.  R = float: pair
// arithmetic in FP32 with compensated (Kahan) FP32 sums; the 3x3 correction
// solve and the momentum/energy totals in FP64.  R = double: the same kernels
// in FP64 with plain sums.

#include <chrono>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <numeric>

#include "crk_internal.h"
#include "tree.h"

namespace crk {

thread_local std::string g_err;

int fail(int code, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return code;
}

}  // namespace crk

using namespace crk;

namespace {

// Per-particle record for the force pass: everything a neighbour contributes,
// with the kernel normalisations, the linear correction and the fixed-point
// scale s = 2^-32 folded in.  For y the separation in grid units (x = s y) and
// q = |y| invHs, the gradient of the particle's corrected kernel is
//   G[c] = w(q) (T0[c] + sum_a Qs[a][c] y[a]) + f(q) (P4s + PBs . y) y[c]
// with T0 = cW (A B + dA), Q[a][c] = cW (A dB[a][c] + dA[c] B[a]), P4 = cF A,
// PB = P4 B and Qs = s Q, P4s = s P4, PBs = s^2 PB, invHs = s / H (exact
// power-of-two scalings): the product rule on A (1 + B . x) W, expanded.
// The record fills whole 128-byte lines (one in FP32, two in FP64): a record
// that straddled a line boundary would cost an extra line lookup when staged.
template <class R> struct alignas(16) RecAcc {
    uint32_t q[3];
    R invHs;
    R V, P, P4s;
    R PBs[3], T0[3], v[3];
    R Qs[9];
    R u;  // specific internal energy (the compatible energy partition)
    R pad[sizeof(R) == 4 ? 5 : 7];
};
static_assert(sizeof(RecAcc<float>) == 128, "f32 record is one 128-byte line");
static_assert(sizeof(RecAcc<double>) == 256, "f64 record is two 128-byte lines");

// The force record with what the artificial viscosity needs of a particle:
// its velocity gradient in grid units dvs = s dv (dvs[3a + c] = s d_c v^a),
// hs = h / s, rcl = rho C_l c_s and rcq = rho C_q (c_s the sound speed).
template <class R> struct alignas(16) RecAccV {
    uint32_t q[3];
    R invHs;
    R V, P, P4s;
    R PBs[3], T0[3], v[3];
    R Qs[9];
    R dvs[9];
    R hs, rcl, rcq;
    R u;
    R pad[sizeof(R) == 4 ? 2 : 3];
};
static_assert(sizeof(RecAccV<float>) == 160 && sizeof(RecAccV<double>) == 320, "whole 16-byte chunks");

// The inviscid part of a force record (shared by both record types).
template <class R, class Rec>
__device__ __forceinline__ void fill_acc(Rec& r, int i, const uint4& q, const R* h, const R* u, const R* vx,
                                         const R* vy, const R* vz, const R* V, const R* rho, const R* A,
                                         const R* B, const R* dA, const R* dB, R gm1) {
    r.q[0] = q.x; r.q[1] = q.y; r.q[2] = q.z;
    // the folded coefficients in FP64, rounded once
    const double sc = kInvGrid;
    const double H = 2.0 * double(h[i]);
    const double cW = norm_W(H), cF = norm_F(H);
    const double Ai = A[i];
    const double P4 = cF * Ai;
    double Bd[3], dAd[3];
    for (int a = 0; a < 3; ++a) {
        Bd[a] = B[3 * i + a];
        dAd[a] = dA[3 * i + a];
    }
    r.invHs = R(sc / H);
    r.V = V[i];
    r.P = gm1 * rho[i] * u[i];
    r.P4s = R(sc * P4);
    for (int a = 0; a < 3; ++a) {
        r.PBs[a] = R(sc * sc * P4 * Bd[a]);
        r.T0[a] = R(cW * (Ai * Bd[a] + dAd[a]));
        for (int c = 0; c < 3; ++c)
            r.Qs[3 * a + c] = R(sc * cW * (Ai * double(dB[9 * i + 3 * a + c]) + dAd[c] * Bd[a]));
    }
    r.v[0] = vx[i]; r.v[1] = vy[i]; r.v[2] = vz[i];
    r.u = u[i];
}

template <class R>
__global__ void k_pack_acc(int n, const int32_t* perm, const uint4* quant, const R* h, const R* u,
                           const R* vx, const R* vy, const R* vz, const R* V, const R* rho,
                           const R* A, const R* B, const R* dA, const R* dB, R gm1,
                           RecAcc<R>* rec) {
    __shared__ uint4 buf[256 * (sizeof(RecAcc<R>) / 16)];
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    const bool valid = s < n;
    const int i = valid ? perm[s] : 0;
    RecAcc<R> r{};
    fill_acc<R>(r, i, quant[valid ? s : 0], h, u, vx, vy, vz, V, rho, A, B, dA, dB, gm1);
    const int first = blockIdx.x * blockDim.x;
    store_records(rec, r, valid, first, min(int(blockDim.x), n - first), buf);
}

// viscosity constants of a launch
struct ViscParams {
    double Cl, Cq, eps_q, gamma;
};

template <class R>
__global__ void k_pack_acc_visc(int n, const int32_t* perm, const uint4* quant, const R* h, const R* u,
                                const R* vx, const R* vy, const R* vz, const R* V, const R* rho,
                                const R* A, const R* B, const R* dA, const R* dB, const R* dv, R gm1,
                                ViscParams vp, RecAccV<R>* rec) {
    __shared__ uint4 buf[256 * (sizeof(RecAccV<R>) / 16)];
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    const bool valid = s < n;
    const int i = valid ? perm[s] : 0;
    RecAccV<R> r{};
    fill_acc<R>(r, i, quant[valid ? s : 0], h, u, vx, vy, vz, V, rho, A, B, dA, dB, gm1);
    for (int k = 0; k < 9; ++k) r.dvs[k] = R(kInvGrid * double(dv[9 * i + k]));
    r.hs = R(double(h[i]) / kInvGrid);
    const double cs = sqrt(vp.gamma * (vp.gamma - 1.0) * double(u[i]));
    r.rcl = R(double(rho[i]) * vp.Cl * cs);
    r.rcq = R(double(rho[i]) * vp.Cq);
    const int first = blockIdx.x * blockDim.x;
    store_records(rec, r, valid, first, min(int(blockDim.x), n - first), buf);
}

// ------------------------------------------------------------------ list build

// One wave per tile: candidate particles are staged 64 at a time in LDS and
// every (lane, candidate) pair is tested against max(H_i, H_j)^2 (with a tiny
// margin so that no pair inside either support is missed in FP32).  The fill
// pass puts the pairs inside the lane's own support (r < H_i, same margin)
// at the front of its list and the others at the back, so the passes that
// gather over r < H_i only stop at the gather count.
// Squared separation for the list membership test.  The count and fill
// passes are separate kernels: with contraction off and a fixed order both
// evaluate it bit for bit alike, so a pair on the boundary is either in both
// or in neither (and lanes i and j agree, the separations being exact
// negatives).
__device__ __forceinline__ float cull_r2(const uint4& qi, const uint4& qj) {
#pragma clang fp contract(off)
    const float dx = sep<float>(qi.x, qj.x);
    const float dy = sep<float>(qi.y, qj.y);
    const float dz = sep<float>(qi.z, qj.z);
    return (dx * dx + dy * dy) + dz * dz;
}

__device__ __forceinline__ float cull_scale(float a2, float b2) {
#pragma clang fp contract(off)
    return fmaxf(a2, b2) * kCullMargin;
}

template <bool FILL>
__global__ __launch_bounds__(64) void k_cull(Queue qu, int n, const uint4* __restrict__ quant,
                                             const int32_t* __restrict__ rng_off,
                                             const int2* __restrict__ rng, int32_t* cnt_out,
                                             const int64_t* __restrict__ ell_off,
                                             const int32_t* __restrict__ ell_len,
                                             uint32_t* __restrict__ nbr, int32_t* __restrict__ cntg_out,
                                             int32_t* __restrict__ leng_out, int32_t* __restrict__ err,
                                             float skin) {
    __shared__ uint4 sj[kWave];
    const int lane = lane_id();
    QState qs;
    for (int w = queue_start(qu, qs); w >= 0; w = queue_next(qu, qs)) {
        const int s = w * kWave + lane;
        const bool valid = s < n;
        const uint4 qi = valid ? quant[s] : make_uint4(0, 0, 0, 0);
        const float Hi = __uint_as_float(qi.w) + skin;
        const float Hi2 = Hi * Hi;
        int c = 0;
        const int64_t base_off = FILL ? ell_off[w] : 0;
        const int cap = (FILL && valid) ? cnt_out[s] : 0;
        int front = 0, back = cap - 1;  // fill cursors: gather pairs, other pairs
        const float G2 = cull_scale(Hi2, Hi2);
        for (int r = rng_off[w]; r < rng_off[w + 1]; ++r) {
            const int2 R = rng[r];
            for (int b = R.x; b < R.y; b += kWave) {
                const int m = min(kWave, R.y - b);
                __syncthreads();
                if (lane < m) sj[lane] = quant[b + lane];
                __syncthreads();
                for (int jj = 0; jj < m; ++jj) {
                    const uint4 qj = sj[jj];
                    const float r2 = cull_r2(qi, qj);
                    const float Hj = __uint_as_float(qj.w) + skin;
                    const float R2 = cull_scale(Hi2, Hj * Hj);
                    if (valid && r2 < R2 && (b + jj) != s) {
                        // the fill pass repeats the count pass exactly; the bound
                        // check keeps every store inside the lane's cnt slots
                        if (FILL && front <= back) {
                            const int k = r2 < G2 ? front++ : back--;
                            nbr[base_off + int64_t(k) * kWave + lane] = uint32_t(b + jj);
                        }
                        ++c;
                    }
                }
            }
        }
        if (!FILL && valid) cnt_out[s] = c;
        if (FILL) {
            // pad the unused slots of the tile's list with a valid index (the
            // lane's own particle, or the tile's first one for lanes past n)
            const uint32_t self = uint32_t(valid ? s : w * kWave);
            for (int k = cap; k < ell_len[w]; ++k) nbr[base_off + int64_t(k) * kWave + lane] = self;
            if (c != cap) {
                // the two passes disagreed: keep every slot a valid index and
                // let the build report the error
                for (int k = front; k <= back; ++k) nbr[base_off + int64_t(k) * kWave + lane] = self;
                atomicAdd(err, 1);
            }
            if (valid) cntg_out[s] = front;
            int mx = front;
            for (int o = 32; o > 0; o >>= 1) mx = max(mx, __shfl_xor(mx, o));
            if (lane == 0) leng_out[w] = mx;
        }
    }
}

// ------------------------------------------------------------------ shared-record slots

// Reorders each tile's lists so that the lanes sharing a neighbour take it in
// the same slot, and records every slot's distinct particles (srec, scnt)
// and each lane's position among them (sidx).  Greedy, one slot at a time:
// among the tile's neighbours, take the one that the most lanes still free in
// this slot need (ties: the smaller index), give it to those lanes, and
// repeat until every lane with entries left holds one; so each lane still
// fills slots 0 .. cnt - 1 and a tile keeps its slot count.  A lane takes its
// gather neighbours (r < H_i) before the others, so the front of its list
// keeps serving the gather passes.  The choice depends only on counts and
// indices, never on the hash layout: the schedule is deterministic.  A tile
// whose neighbour set overflows the table keeps its order with the identity
// sets (64 per slot).
//
// One wave per tile.  The tile's distinct neighbours are collected in an LDS
// hash table, compacted, and held in registers (lane l keeps entries l,
// l + 64, ...), so a pick scans registers only.  Once no neighbour is wanted
// by two free lanes, the greedy would give every free lane its smallest
// wanted neighbour, in increasing order of index: those picks are made at
// once (a minimum per lane through LDS, and ranks for the positions).
constexpr int kSchedHash = 2048;
constexpr int kSchedRegs = kSchedHash / kWave;  // neighbours per lane at most
constexpr uint32_t kSchedEmpty = 0xFFFFFFFFu;

__device__ __forceinline__ unsigned long long readlane64(unsigned long long v, int l) {
    const uint32_t lo = uint32_t(__builtin_amdgcn_readlane(int(uint32_t(v)), l));
    const uint32_t hi = uint32_t(__builtin_amdgcn_readlane(int(uint32_t(v >> 32)), l));
    return (static_cast<unsigned long long>(hi) << 32) | lo;
}

// One of the tile's distinct neighbours with the lanes that need it, in the
// gather and the other part of their lists.
struct SchedEntry {
    unsigned long long gm, bm;
    uint32_t key, pad;
};

// Phase 1, one wave per tile of a batch (tile0 + block): the tile's distinct
// neighbours (an LDS hash table), compacted and written to tbl (kSchedHash
// entries per tile of the batch), their number to tcnt.  A tile whose set
// overflows the table gets the identity schedule here (tcnt = -1).
__global__ __launch_bounds__(64) void k_sched_table(int n, int tile0, const int32_t* __restrict__ cnt,
                                                    const int32_t* __restrict__ cntg,
                                                    const int64_t* __restrict__ ell_off,
                                                    const int32_t* __restrict__ ell_len,
                                                    const uint32_t* __restrict__ nbr, uint32_t* __restrict__ srec,
                                                    uint8_t* __restrict__ sidx, int32_t* __restrict__ scnt,
                                                    SchedEntry* __restrict__ tbl, int32_t* __restrict__ tcnt) {
    __shared__ uint32_t key[kSchedHash];
    __shared__ unsigned long long gm[kSchedHash], bm[kSchedHash];  // lanes needing it: gather, other
    const int bt = blockIdx.x;
    const int w = tile0 + bt;
    const int lane = int(threadIdx.x);
    const int s = w * kWave + lane;
    const bool valid = s < n;
    const int c = valid ? cnt[s] : 0;
    const int cg = valid ? cntg[s] : 0;
    const int len = ell_len[w];
    const int64_t off = ell_off[w];
    for (int t = lane; t < kSchedHash; t += kWave) {
        key[t] = kSchedEmpty;
        gm[t] = 0;
        bm[t] = 0;
    }
    __syncthreads();
    int full = 0;
    for (int k = 0; k < c; ++k) {
        const uint32_t j = nbr[off + int64_t(k) * kWave + lane];
        uint32_t h = (j * 2654435761u) >> 21;
        int probe = 0;
        for (; probe < kSchedHash; ++probe) {
            const uint32_t prev = atomicCAS(&key[h], kSchedEmpty, j);
            if (prev == kSchedEmpty || prev == j) break;
            h = (h + 1) & (kSchedHash - 1);
        }
        if (probe == kSchedHash) {
            full = 1;
            break;
        }
        atomicOr(k < cg ? &gm[h] : &bm[h], 1ull << lane);
    }
    __syncthreads();
    if (__ballot(full) != 0) {  // identity sets: every lane's own entry
        for (int k = 0; k < len; ++k) {
            const int64_t e = off + int64_t(k) * kWave + lane;
            srec[e] = nbr[e];
            sidx[e] = uint8_t(lane);
            if (lane == 0) scnt[(off >> 6) + k] = kWave;
        }
        if (lane == 0) tcnt[bt] = -1;
        return;
    }
    // compact the distinct neighbours to the front of the table (in place: an
    // entry never moves past a row that is still to be read)
    int nd = 0;
    for (int i = 0; i < kSchedRegs; ++i) {
        const int t = lane + kWave * i;
        const uint32_t kk = key[t];
        const unsigned long long g = gm[t], b = bm[t];
        const bool live = kk != kSchedEmpty;
        const unsigned long long lb = __ballot(live);
        const int pos = nd + __popcll(lb & ((1ull << lane) - 1ull));
        __syncthreads();  // the whole row is read before any of it is overwritten
        if (live) {
            key[pos] = kk;
            gm[pos] = g;
            bm[pos] = b;
        }
        nd += __popcll(lb);
    }
    __syncthreads();
    SchedEntry* out = tbl + int64_t(bt) * kSchedHash;
    for (int t = lane; t < nd; t += kWave) out[t] = SchedEntry{gm[t], bm[t], key[t], 0u};
    if (lane == 0) tcnt[bt] = nd;
}

// Phase 2, one wave per listed tile (list holds batch positions): the greedy
// cover of every slot from the tile's neighbour table held in registers
// (kRegs entries per lane at most: tiles are binned by their table size, so
// that small tables run with fewer registers and more waves).
template <int kRegs>
__global__ __launch_bounds__(64) void k_sched_pick(int n, int tile0, const int32_t* __restrict__ list,
                                                   const int32_t* __restrict__ cnt,
                                                   const int32_t* __restrict__ cntg,
                                                   const int64_t* __restrict__ ell_off,
                                                   const int32_t* __restrict__ ell_len, uint32_t* __restrict__ nbr,
                                                   uint32_t* __restrict__ srec, uint8_t* __restrict__ sidx,
                                                   int32_t* __restrict__ scnt, const SchedEntry* __restrict__ tbl,
                                                   const int32_t* __restrict__ tcnt) {
    __shared__ uint32_t tmin[kWave];
    const int bt = list[blockIdx.x];
    const int w = tile0 + bt;
    const int lane = int(threadIdx.x);
    const int s = w * kWave + lane;
    const bool valid = s < n;
    const int c = valid ? cnt[s] : 0;
    const int cg = valid ? cntg[s] : 0;
    const int len = ell_len[w];
    const int64_t off = ell_off[w];
    const uint32_t self = uint32_t(valid ? s : w * kWave);
    const int nd = tcnt[bt];
    const int nk = (nd + kWave - 1) / kWave;  // <= kRegs (binned)
    const SchedEntry* tab = tbl + int64_t(bt) * kSchedHash;
    uint32_t K[kRegs];
    unsigned long long GM[kRegs], BM[kRegs];
#pragma unroll
    for (int i = 0; i < kRegs; ++i) {
        const int t = lane + kWave * i;
        const bool ok = i < nk && t < nd;
        const SchedEntry e = ok ? tab[t] : SchedEntry{0ull, 0ull, kSchedEmpty, 0u};
        K[i] = e.key;
        GM[i] = e.gm;
        BM[i] = e.bm;
    }
    int remg = cg, remb = c - cg;
    const unsigned long long bit = 1ull << lane;
    for (int k = 0; k < len; ++k) {
        const unsigned long long gph = __ballot(remg > 0);
        unsigned long long open = __ballot(remg + remb > 0);
        uint32_t mine = self;
        int mypos = 0, m = 0;
        uint32_t first = 0;
        while (open != 0 && m < kWave) {
            // the neighbour wanted by the most free lanes (ties: smaller index)
            int bc = 0;
            uint32_t bk = kSchedEmpty;
#pragma unroll
            for (int i = 0; i < kRegs; ++i) {
                if (i >= nk) continue;
                const int cv = __popcll(((GM[i] & gph) | (BM[i] & ~gph)) & open);
                if (cv > bc || (cv == bc && K[i] < bk)) {
                    bc = cv;
                    bk = K[i];
                }
            }
            for (int o = kWave / 2; o > 0; o >>= 1) {
                const int oc = __shfl_xor(bc, o);
                const uint32_t ok = uint32_t(__shfl_xor(int(bk), o));
                if (oc > bc || (oc == bc && ok < bk)) {
                    bc = oc;
                    bk = ok;
                }
            }
            bc = __builtin_amdgcn_readfirstlane(bc);
            bk = uint32_t(__builtin_amdgcn_readfirstlane(int(bk)));
            if (bc == 0) break;
            if (bc == 1) {
                // every free lane takes its smallest wanted neighbour; the
                // slot positions follow the neighbours' order
                tmin[lane] = kSchedEmpty;
                __syncthreads();
#pragma unroll
                for (int i = 0; i < kRegs; ++i) {
                    if (i >= nk) continue;
                    const unsigned long long want = ((GM[i] & gph) | (BM[i] & ~gph)) & open;
                    if (want) atomicMin(&tmin[__builtin_ctzll(want)], K[i]);
                }
                __syncthreads();
                const uint32_t mk = tmin[lane];
                const bool taker = (open & bit) != 0;
                int rank = 0;
                for (int l = 0; l < kWave; ++l) rank += ((open >> l) & 1ull) && tmin[l] < mk;
#pragma unroll
                for (int i = 0; i < kRegs; ++i) {
                    if (i >= nk) continue;
                    const unsigned long long want = ((GM[i] & gph) | (BM[i] & ~gph)) & open;
                    if (want && tmin[__builtin_ctzll(want)] == K[i]) {
                        GM[i] &= ~(want & gph);
                        BM[i] &= ~(want & ~gph);
                    }
                }
                if (taker) {
                    mine = mk;
                    mypos = m + rank;
                    if (remg > 0) --remg;
                    else --remb;
                    srec[off + int64_t(k) * kWave + m + rank] = mk;
                }
                const unsigned long long r0 = __ballot(taker && rank == 0);
                if (m == 0) first = uint32_t(__builtin_amdgcn_readlane(int(mk), __builtin_ctzll(r0)));
                m += __popcll(open);
                open = 0;
                __syncthreads();  // tmin is read before the next slot clears it
                break;
            }
            // its owner lane holds the masks: the lanes it goes to
            unsigned long long take = 0;
            bool owner = false;
#pragma unroll
            for (int i = 0; i < kRegs; ++i) {
                if (i >= nk) continue;
                if (K[i] == bk) {
                    owner = true;
                    take = ((GM[i] & gph) | (BM[i] & ~gph)) & open;
                    GM[i] &= ~(take & gph);
                    BM[i] &= ~(take & ~gph);
                }
            }
            take = readlane64(take, __builtin_ctzll(__ballot(owner)));
            if (take & bit) {
                mine = bk;
                mypos = m;
                if (remg > 0) --remg;
                else --remb;
            }
            if (lane == 0) srec[off + int64_t(k) * kWave + m] = bk;
            if (m == 0) first = bk;
            open &= ~take;
            ++m;
        }
        const int64_t e = off + int64_t(k) * kWave + lane;
        nbr[e] = mine;
        sidx[e] = uint8_t(mypos);
        if (lane >= m) srec[e] = m > 0 ? first : self;  // past the set: any valid index
        if (lane == 0) scnt[(off >> 6) + k] = m > 0 ? m : 1;
    }
}

// Tiles of a batch by the register table they need: up to 16 entries per lane
// (list16) or up to 32 (list32); counts[0..1] their numbers (zeroed before).
__global__ void k_sched_bins(int nb, const int32_t* __restrict__ tcnt, int32_t* __restrict__ list16,
                             int32_t* __restrict__ list32, int32_t* __restrict__ counts) {
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= nb) return;
    const int nd = tcnt[b];
    if (nd < 0) return;  // identity schedule, already written
    if (nd <= 16 * kWave) list16[atomicAdd(&counts[0], 1)] = b;
    else list32[atomicAdd(&counts[1], 1)] = b;
}

// Exact FP64 interaction counts over the lists: r < H_i and r < max(H_i, H_j).
__global__ __launch_bounds__(256) void k_count_lists(int n, const uint4* __restrict__ quant,
                                                     const double* __restrict__ Hd,
                                                     const int32_t* __restrict__ cnt,
                                                     const int64_t* __restrict__ ell_off,
                                                     const uint32_t* __restrict__ nbr,
                                                     unsigned long long* out) {
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    unsigned long long c0 = 0, c1 = 0;
    if (s < n) {
        const int w = s / kWave, lane = s % kWave;
        const uint4 qi = quant[s];
        const double Hi = Hd[s];
        for (int k = 0; k < cnt[s]; ++k) {
            const uint32_t j = nbr[ell_off[w] + int64_t(k) * kWave + lane];
            const uint4 qj = quant[j];
            const double dx = sep<double>(qi.x, qj.x), dy = sep<double>(qi.y, qj.y),
                         dz = sep<double>(qi.z, qj.z);
            const double r = sqrt(dx * dx + dy * dy + dz * dz);
            c0 += r < Hi;
            c1 += r < fmax(Hi, Hd[j]);
        }
    }
    for (int o = 32; o > 0; o >>= 1) {
        c0 += __shfl_xor(c0, o);
        c1 += __shfl_xor(c1, o);
    }
    if (lane_id() == 0) {
        atomicAdd(out, c0);
        atomicAdd(out + 1, c1);
    }
}

// FP64 pair counts r < r_fixed over the tiles' candidate ranges.
__global__ __launch_bounds__(64) void k_count_fixed(int n_tiles, int n, const uint4* __restrict__ quant,
                                                    const int32_t* __restrict__ rng_off,
                                                    const int2* __restrict__ rng, double rc,
                                                    unsigned long long* out) {
    const int w = blockIdx.x;
    if (w >= n_tiles) return;
    const int s = w * kWave + lane_id();
    unsigned long long c = 0;
    if (s < n) {
        const uint4 qi = quant[s];
        for (int r = rng_off[w]; r < rng_off[w + 1]; ++r) {
            const int2 R = rng[r];
            for (int j = R.x; j < R.y; ++j) {
                if (j == s) continue;
                const uint4 qj = quant[j];
                const double dx = sep<double>(qi.x, qj.x), dy = sep<double>(qi.y, qj.y),
                             dz = sep<double>(qi.z, qj.z);
                c += sqrt(dx * dx + dy * dy + dz * dz) < rc;
            }
        }
    }
    for (int o = 32; o > 0; o >>= 1) c += __shfl_xor(c, o);
    if (lane_id() == 0) atomicAdd(out, c);
}

// ------------------------------------------------------------------ volume

template <class R, bool kStage16, bool kOff32>
__global__ __launch_bounds__(256) void k_volume(Queue qu, int n, Lists L, const int32_t* __restrict__ perm,
                                                const uint4* __restrict__ quant, const R* __restrict__ h,
                                                const R* __restrict__ m, int chunk, R* __restrict__ V_out,
                                                R* __restrict__ rho_out) {
    constexpr int kStage = stage_stride<uint4, kStage16>();
    extern __shared__ uint4 stage_buf[];  // kStage per wave when staged (stage_bytes)
    const int lane = lane_id();
    QState qs;
    for (int w = queue_start(qu, qs); w >= 0; w = queue_next(qu, qs)) {
        const int s = w * kWave + lane;
        const bool valid = s < n;
        const int i = valid ? perm[s] : 0;
        const uint4 qi = valid ? quant[s] : make_uint4(0, 0, 0, 0);
        const R H = valid ? R(2) * h[i] : R(1);
        const R invHg = (R(1) / H) * R(kInvGrid);  // q from separations in grid units
        const int cnt = valid ? L.cnt[s] : 0;
        const int len = L.len[w];
        ChunkSums<R, 1> S;
        S.zero();
        S.add(0, R(1));  // self term: w(0) = 1
        list_loop<uint4, kOff32, kStage16>(
            L, w, cnt, len, quant, stage_buf + wave_in_block() * kStage,
            [&](const uint4& qj, int k) __attribute__((always_inline)) {
                const R dx = grid_sep<R>(qi.x, qj.x), dy = grid_sep<R>(qi.y, qj.y), dz = grid_sep<R>(qi.z, qj.z);
                const R r = dsqrt(dx * dx + dy * dy + dz * dz);
                R wq, fq;
                wendland(r * invHg, wq, fq);
                S.add(0, k < cnt ? wq : R(0));  // past the count: adds zero
                S.next(k, chunk);
            });
        S.fold();
        if (valid) {
            const R Ssum = S.get(0) * norm_W(H);
            V_out[i] = R(1) / Ssum;
            rho_out[i] = m[i] * Ssum;
        }
    }
}

// ------------------------------------------------------------------ corrections

// Moments over the neighbour list and the FP64 solve; corrections written in
// caller order.
template <class R, bool kOff32, bool kStage16>
__global__ __launch_bounds__(256) void k_moments(Queue qu, int n, Lists L, const int32_t* __restrict__ perm,
                                                 const RecQV<R>* __restrict__ qv,
                                                 const R* __restrict__ h, int chunk, R* __restrict__ A_out,
                                                 R* __restrict__ B_out, R* __restrict__ dA_out,
                                                 R* __restrict__ dB_out,
                                                 unsigned long long* __restrict__ n_fallback,
                                                 double* __restrict__ sums_out) {
    constexpr int kStage = stage_stride<RecQV<R>, kStage16>();
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
        moment_sums<R, kOff32, kStage16>(w, s, valid, L, qv, stage_buf + wave_in_block() * kStage, H, chunk, S, nnb);
        if (valid && sums_out) {
            // kept for the backward (caller order, one row of n per sum)
            for (int e = 0; e < 29; ++e) sums_out[int64_t(e) * n + i] = S[e];
            sums_out[int64_t(29) * n + i] = double(nnb);
        }
        moments_from_sums(S, M);
        if (valid) {
            double Ad, Bd[3], dAd[3], dBd[9];
            const int fb = solve_moments(M, nnb, Ad, Bd, dAd, dBd);
            A_out[i] = R(Ad);
            for (int a = 0; a < 3; ++a) {
                B_out[3 * i + a] = R(Bd[a]);
                dA_out[3 * i + a] = R(dAd[a]);
            }
            for (int k = 0; k < 9; ++k) dB_out[9 * i + k] = R(dBd[k]);
            if (n_fallback && fb) atomicAdd(n_fallback, 1ull);
        }
    }
}

// ------------------------------------------------------------------ forces

// gradient of a particle's corrected kernel at separation y (grid units, from
// that particle); the lane's own particle and its neighbour go through the same
// expression, on exactly negated separations, so that F_ij = -F_ji bit for bit
template <class R, class Rec>
__device__ __forceinline__ void corrected_grad(const Rec& r, R wq, R fq, const R y[3], R G[3]) {
    const R fl = fq * (r.P4s + r.PBs[0] * y[0] + r.PBs[1] * y[1] + r.PBs[2] * y[2]);
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        const R t = r.T0[c] + r.Qs[c] * y[0] + r.Qs[3 + c] * y[1] + r.Qs[6 + c] * y[2];
        G[c] = wq * t + fl * y[c];
    }
}

// What a pair adds to the energy sum.  Symmetric partition: Fv = 2 W_ij, W_ij
// = (v_j - v_i) . F_ij the pair's work, of which i takes half.  Compatible
// partition: i takes f_ij W_ij with f_ij = 1/2 (1 + s_ij),
// s_ij = sgn(W_ij) (u_j - u_i) / (|u_j - u_i| + eps_u (u_i + u_j)), so heating
// goes mostly to the colder particle and cooling comes mostly from the hotter;
// the sum gets (1 + s_ij) Fv.  Both sides of a pair compute the same Fv and
// exactly negated d, so s_ji = -s_ij bit for bit.
template <bool kCompat, class R, class Rec>
__device__ __forceinline__ R energy_term(const Rec& ri, const Rec& rj, R eps_u, R Fv) {
    if constexpr (!kCompat) {
        return Fv;
    } else {
        const R d = rj.u - ri.u;
        const R den = fabs(d) + eps_u * (ri.u + rj.u);
        const R sw = Fv > R(0) ? R(1) : (Fv < R(0) ? R(-1) : R(0));
        const R sh = den > R(0) ? sw * d / den : R(0);
        return Fv + sh * Fv;
    }
}

// One pair of the force pass for lane particle i and neighbour j: adds
// (V_i V_j)(P_i + P_j)(G_i - G_j) (the pair force is -1/2 of it) and its dot
// product with v_i - v_j.
template <bool kCompat, class R>
__device__ __forceinline__ void accel_pair(const RecAcc<R>& ri, const RecAcc<R>& rj, R eps_u, int k, int chunk,
                                           ChunkSums<R, 4>& acc) {
    const R y[3] = {grid_sep<R>(ri.q[0], rj.q[0]), grid_sep<R>(ri.q[1], rj.q[1]),
                    grid_sep<R>(ri.q[2], rj.q[2])};
    const R yo[3] = {-y[0], -y[1], -y[2]};
    const R r = dsqrt(y[0] * y[0] + y[1] * y[1] + y[2] * y[2]);
    R wi, fi, wj, fj;
    wendland(r * ri.invHs, wi, fi);
    wendland(r * rj.invHs, wj, fj);
    R Gi[3], Gj[3];
    corrected_grad(ri, wi, fi, y, Gi);
    corrected_grad(rj, wj, fj, yo, Gj);
    const R coef = (ri.V * rj.V) * (ri.P + rj.P);
    R Fv = R(0);
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        const R F = coef * (Gi[c] - Gj[c]);
        Fv += F * (ri.v[c] - rj.v[c]);
        acc.add(c, F);
    }
    acc.add(3, energy_term<kCompat>(ri, rj, eps_u, Fv));
    acc.next(k, chunk);
}

// The same pair with the artificial viscosity: Q_i + Q_j joins P_i + P_j.
// Per pair, with D_k = dv_k x (velocity units) and s_k = x . D_k, the van
// Leer limiter Phi = max(0, 4 s_i s_j / (s_i + s_j)^2) weights the linear
// reconstruction of both velocities to the pair's midpoint, w = v_i - v_j -
// Phi/2 (D_i + D_j), and mu_k = min(0, h_k (w.x) / (r^2 + eps_q h_k^2)),
// Q_k = rho_k (-C_l c_k mu_k + C_q mu_k^2).  In grid units (x = s y):
// D_k = dvs_k y, s_k carries a common factor 1/s, and
// mu_k = hs_k (w.y) / (|y|^2 + eps_q hs_k^2).  Every quantity is evaluated by
// the same expressions from both sides of the pair (the two Q terms are
// separate statements, added commutatively), so F_ij = -F_ji bit for bit.
template <bool kCompat, class R>
__device__ __forceinline__ void accel_pair_visc(const RecAccV<R>& ri, const RecAccV<R>& rj, R eps_q, R eps_u,
                                                int k, int chunk, ChunkSums<R, 4>& acc) {
    const R y[3] = {grid_sep<R>(ri.q[0], rj.q[0]), grid_sep<R>(ri.q[1], rj.q[1]),
                    grid_sep<R>(ri.q[2], rj.q[2])};
    const R yo[3] = {-y[0], -y[1], -y[2]};
    const R r2 = y[0] * y[0] + y[1] * y[1] + y[2] * y[2];
    const R r = dsqrt(r2);
    R wi, fi, wj, fj;
    wendland(r * ri.invHs, wi, fi);
    wendland(r * rj.invHs, wj, fj);
    R Gi[3], Gj[3];
    corrected_grad(ri, wi, fi, y, Gi);
    corrected_grad(rj, wj, fj, yo, Gj);
    R Di[3], Dj[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        Di[a] = ri.dvs[3 * a] * y[0] + ri.dvs[3 * a + 1] * y[1] + ri.dvs[3 * a + 2] * y[2];
        Dj[a] = rj.dvs[3 * a] * y[0] + rj.dvs[3 * a + 1] * y[1] + rj.dvs[3 * a + 2] * y[2];
    }
    const R si = y[0] * Di[0] + y[1] * Di[1] + y[2] * Di[2];
    const R sj = y[0] * Dj[0] + y[1] * Dj[1] + y[2] * Dj[2];
    const R sp = si * sj;
    const R ss = si + sj;
    const R half_phi = sp > R(0) ? R(2) * sp / (ss * ss) : R(0);
    R wy = R(0);
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const R wa = (ri.v[a] - rj.v[a]) - half_phi * (Di[a] + Dj[a]);
        wy += wa * y[a];
    }
    const R mi = fmin(R(0), ri.hs * wy / (r2 + eps_q * ri.hs * ri.hs));
    const R mj = fmin(R(0), rj.hs * wy / (r2 + eps_q * rj.hs * rj.hs));
    const R qi = mi * (ri.rcq * mi - ri.rcl);
    const R qj = mj * (rj.rcq * mj - rj.rcl);
    const R Q = qi + qj;
    const R coef = (ri.V * rj.V) * ((ri.P + rj.P) + Q);
    R Fv = R(0);
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        const R F = coef * (Gi[c] - Gj[c]);
        Fv += F * (ri.v[c] - rj.v[c]);
        acc.add(c, F);
    }
    acc.add(3, energy_term<kCompat>(ri, rj, eps_u, Fv));
    acc.next(k, chunk);
}

// a_i = -1/2 sum / m_i and du_i/dt = 1/4 (dot-product sum) / m_i; the tile's
// FP64 partial totals go to partials[8 w ...]
template <class R, class Rec>
__device__ __forceinline__ void accel_finish(int w, int s, bool valid, const Rec& ri,
                                             ChunkSums<R, 4>& acc, const int32_t* __restrict__ perm,
                                             const R* __restrict__ m, R* __restrict__ a_out,
                                             R* __restrict__ du_out, double* __restrict__ partials) {
    acc.fold();
    double t[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    if (valid) {
        const int i = perm[s];
        const R mi = m[i];
        R av[3];
        for (int c = 0; c < 3; ++c) {
            av[c] = R(-0.5) * acc.get(c) / mi;
            a_out[3 * i + c] = av[c];
        }
        const R du = R(0.25) * acc.get(3) / mi;
        du_out[i] = du;
        const double md = double(mi);
        const double ax = av[0], ay = av[1], az = av[2], dd = du;
        const double va = double(ri.v[0]) * ax + double(ri.v[1]) * ay + double(ri.v[2]) * az;
        t[0] = md * ax; t[1] = md * ay; t[2] = md * az;
        t[3] = md * (va + dd);
        t[4] = md * sqrt(ax * ax + ay * ay + az * az);
        t[5] = md * (fabs(va) + fabs(dd));
        t[6] = md * dd;
        t[7] = md * va;
    }
#pragma unroll
    for (int k = 0; k < 8; ++k)
        for (int o = 32; o > 0; o >>= 1) t[k] += __shfl_xor(t[k], o);
    if (lane_id() == 0)
        for (int k = 0; k < 8; ++k) partials[8 * w + k] = t[k];
}

template <class R, bool kOff32, bool kCompat>
__global__ __launch_bounds__(256) void k_accel(Queue qu, int n, Lists L, const int32_t* __restrict__ perm,
                                               const RecAcc<R>* __restrict__ rec, const R* __restrict__ m,
                                               R eps_u, int chunk, R* __restrict__ a_out, R* __restrict__ du_out,
                                               double* __restrict__ partials) {
    constexpr int kStage = stage_stride<RecAcc<R>>();
    extern __shared__ uint4 stage_buf[];  // kStage per wave (stage_bytes)
    const int lane = lane_id();
    QState qs;
    for (int w = queue_start(qu, qs); w >= 0; w = queue_next(qu, qs)) {
        const int s = w * kWave + lane;
        const bool valid = s < n;
        const RecAcc<R> ri = rec[valid ? s : 0];
        const int cnt = valid ? L.cnt[s] : 0;
        const int len = L.len[w];
        ChunkSums<R, 4> acc;
        acc.zero();
        staged_list<RecAcc<R>, kOff32>(
            L, w, cnt, len, rec, stage_buf + wave_in_block() * kStage,
            [&](const RecAcc<R>& rj, int k) __attribute__((always_inline)) {
                accel_pair<kCompat>(ri, rj, eps_u, k, chunk, acc);
            });
        accel_finish(w, s, valid, ri, acc, perm, m, a_out, du_out, partials);
    }
}

template <class R, bool kOff32, bool kCompat>
__global__ __launch_bounds__(256) void k_accel_visc(Queue qu, int n, Lists L, const int32_t* __restrict__ perm,
                                                    const RecAccV<R>* __restrict__ rec, const R* __restrict__ m,
                                                    R eps_q, R eps_u, int chunk, R* __restrict__ a_out,
                                                    R* __restrict__ du_out, double* __restrict__ partials) {
    constexpr int kStage = stage_stride<RecAccV<R>>();
    extern __shared__ uint4 stage_buf[];  // kStage per wave (stage_bytes)
    const int lane = lane_id();
    QState qs;
    for (int w = queue_start(qu, qs); w >= 0; w = queue_next(qu, qs)) {
        const int s = w * kWave + lane;
        const bool valid = s < n;
        const RecAccV<R> ri = rec[valid ? s : 0];
        const int cnt = valid ? L.cnt[s] : 0;
        const int len = L.len[w];
        ChunkSums<R, 4> acc;
        acc.zero();
        staged_list<RecAccV<R>, kOff32>(
            L, w, cnt, len, rec, stage_buf + wave_in_block() * kStage,
            [&](const RecAccV<R>& rj, int k) __attribute__((always_inline)) {
                accel_pair_visc<kCompat>(ri, rj, eps_q, eps_u, k, chunk, acc);
            });
        accel_finish(w, s, valid, ri, acc, perm, m, a_out, du_out, partials);
    }
}

// Work-queue coverage: every wave adds one to visits[tile] for each tile the
// queue hands it (the same queue_start / queue_next walk as the pair passes).
__global__ __launch_bounds__(256) void k_queue_visits(Queue qu, int32_t* __restrict__ visits) {
    QState qs;
    for (int w = queue_start(qu, qs); w >= 0; w = queue_next(qu, qs))
        if (lane_id() == 0) atomicAdd(visits + w, 1);
}

// Fixed-order FP64 reduction of the per-tile totals in two stages: block b
// sums tiles [b per, (b + 1) per) (thread t takes every 256th from the start),
// then one block sums the block results.  The order depends only on the tile
// count, never on the schedule that produced the tiles.
constexpr int kTotalsBlocks = 128;

__device__ __forceinline__ void block_sum8(double t[8], double (*red)[8]) {
    for (int k = 0; k < 8; ++k) red[threadIdx.x][k] = t[k];
    __syncthreads();
    for (int st = 128; st > 0; st >>= 1) {
        if (threadIdx.x < st)
            for (int k = 0; k < 8; ++k) red[threadIdx.x][k] += red[threadIdx.x + st][k];
        __syncthreads();
    }
}

__global__ __launch_bounds__(256) void k_totals_blocks(int n_items, int per, const double* __restrict__ in,
                                                       double* __restrict__ out) {
    __shared__ double red[256][8];
    double t[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    const int lo = blockIdx.x * per, hi = min(n_items, lo + per);
    for (int w = lo + int(threadIdx.x); w < hi; w += 256)
        for (int k = 0; k < 8; ++k) t[k] += in[8 * w + k];
    block_sum8(t, red);
    if (threadIdx.x < 8) out[8 * blockIdx.x + threadIdx.x] = red[0][threadIdx.x];
}

}  // namespace

namespace crk {


int pass_scratch(crk_leaves* L, size_t bytes, void** out) {
    if (bytes > L->scratch_bytes)
        return fail(CRK_ENOSPC, "pass needs %zu bytes of scratch, the handle's workspace holds %zu", bytes,
                    L->scratch_bytes);
    *out = L->scratch;
    return CRK_OK;
}

void drop_timed(crk_leaves* L) {
    for (auto& t : L->timed) {
        (void)hipEventDestroy(t.a);
        (void)hipEventDestroy(t.b);
    }
    L->timed.clear();
}

Queue make_queue(const crk_leaves* L, const int32_t* order) {
    // tree order keeps spatially adjacent tiles together (L2 reuse); the
    // longest-first order balances uneven tiles
    const int32_t* ord = L->tune.tile_order == 0 ? L->order_tree : order;
    const int g = L->tune.xcd_groups;
    const int32_t per = int32_t((L->n_tiles + g - 1) / g);
    return Queue{ord, L->counter, int32_t(L->n_tiles), L->tune.persistent, g, per};
}

static int grid_for(const crk_leaves* L, int bw) {
    const int g = L->tune.xcd_groups;
    const int64_t per = (L->n_tiles + g - 1) / g;
    int64_t blocks = g * ((per + bw - 1) / bw);  // one wave per tile
    if (L->tune.persistent) {
        const int64_t cap = int64_t(L->n_cu) * L->tune.waves_per_cu / bw;
        blocks = std::min(blocks, std::max<int64_t>(g, cap / g * g));
    }
    return int(std::max<int64_t>(blocks, 1));
}

// grid for one-wave workgroups (LDS-staged kernels)
int grid_1wave(const crk_leaves* L) { return grid_for(L, 1); }
// grid for block_waves-wave workgroups (list-driven passes)
int grid_nwave(const crk_leaves* L) { return grid_for(L, L->tune.block_waves); }

int check_gas(const crk_leaves* L, const crk_gas* g, bool need_v) {
    if (!L || !g) return fail(CRK_EINVAL, "null handle or gas");
    if (L->n == 0 && g->n == 0) return CRK_OK;  // nothing to do in either mode
    if (!L->hydro) return fail(CRK_ESTATE, "handle was built in fixed-radius mode; CRK passes need h");
    if (g->n != L->n) return fail(CRK_EINVAL, "gas.n = %lld does not match the handle (%lld)",
                                  (long long)g->n, (long long)L->n);
    if (L->n == 0) return CRK_OK;
    if (!g->x || !g->y || !g->z || !g->h) return fail(CRK_EINVAL, "gas positions and h are required");
    if (need_v && (!g->vx || !g->vy || !g->vz || !g->u || !g->m))
        return fail(CRK_EINVAL, "gas velocities, u and m are required");
    return CRK_OK;
}

void reset_queue(crk_leaves* L, hipStream_t st) {
    // only the persistent queue reads the counters
    if (L->tune.persistent) hipLaunchKernelGGL(k_reset, dim3(1), dim3(64), 0, st, L->counter);
}

Lists lists(const crk_leaves* L) {
    return Lists{L->cnt, L->ell_off, L->ell_len, L->nbr, L->srec, L->sidx, L->scnt};
}
Lists lists_gather(const crk_leaves* L) {
    return Lists{L->cnt_gather, L->ell_off, L->ell_len_gather, L->nbr, L->srec, L->sidx, L->scnt};
}

}  // namespace crk

namespace {

template <class R> int volume_impl(crk_leaves* L, const crk_gas* g, R* V, R* rho, hipStream_t st) {
    int rc = pack_positions<R>(L, g->x, g->y, g->z, static_cast<const R*>(g->h), st);
    if (rc) return rc;
    reset_queue(L, st);
    TimeScope ts(L, st, CRK_K_VOLUME);
    const bool st16 = L->tune.stage16 != 0, o32 = off32<uint4>(L);
    // both forms take 32-bit record offsets only where the positions span at most 4 GiB
    auto kern = st16 ? (o32 ? k_volume<R, true, true> : k_volume<R, true, false>)
                     : (o32 ? k_volume<R, false, true> : k_volume<R, false, false>);
    const int bw = L->tune.block_waves;
    const size_t lds = st16 ? stage_bytes<uint4, true>(bw) : size_t(0);
    hipLaunchKernelGGL(kern, dim3(grid_nwave(L)), dim3(kWave * bw), lds, st,
                       make_queue(L, L->order_pair), int(L->n), lists_gather(L), L->perm, L->quant,
                       static_cast<const R*>(g->h), static_cast<const R*>(g->m), L->tune.kahan_chunk, V,
                       rho);
    LAUNCH_CHECK("volume");
    return CRK_OK;
}

template <class R>
int corrections_impl(crk_leaves* L, const crk_gas* g, const R* V, const crk_corr* out,
                     int64_t* n_fallback, hipStream_t st) {
    const int n = int(L->n);
    int rc = pack_positions<R>(L, g->x, g->y, g->z, static_cast<const R*>(g->h), st);
    if (rc) return rc;
    void* sp = nullptr;
    if ((rc = pass_scratch(L, sizeof(RecQV<R>) * size_t(n), &sp))) return rc;
    RecQV<R>* qv = static_cast<RecQV<R>*>(sp);
    {
        TimeScope tp(L, st, CRK_K_PACK);
        hipLaunchKernelGGL(k_pack_qv<R>, dim3((n + 255) / 256), dim3(256), 0, st, n, L->perm, L->quant, V, qv);
    }
    LAUNCH_CHECK("pack position/volume");
    reset_queue(L, st);
    TimeScope ts(L, st, CRK_K_MOMENTS);
    const bool st16 = L->tune.stage16 != 0;
    auto kern = off32<RecQV<R>>(L) ? (st16 ? k_moments<R, true, true> : k_moments<R, true, false>)
                                   : (st16 ? k_moments<R, false, true> : k_moments<R, false, false>);
    const size_t lds = st16 ? stage_bytes<RecQV<R>, true>(L->tune.block_waves)
                            : stage_bytes<RecQV<R>>(L->tune.block_waves);
    hipLaunchKernelGGL(kern, dim3(grid_nwave(L)), dim3(kWave * L->tune.block_waves), lds, st,
                       make_queue(L, L->order_pair), n, lists_gather(L), L->perm, qv,
                       static_cast<const R*>(g->h), L->tune.kahan_chunk, static_cast<R*>(out->A),
                       static_cast<R*>(out->B), static_cast<R*>(out->dA), static_cast<R*>(out->dB),
                       reinterpret_cast<unsigned long long*>(n_fallback), static_cast<double*>(out->M));
    LAUNCH_CHECK("moments");
    return CRK_OK;
}

// Scratch of one force pass: the neighbour records (n), then the FP64 totals
// partials (8 per tile, then 8 per reduction block).
template <class R> size_t accel_scratch_records(int64_t n) {
    return (sizeof(RecAcc<R>) * size_t(n) + 255) / 256 * 256;
}
template <class R> size_t accel_scratch_bytes(int64_t n, int64_t n_tiles) {
    return accel_scratch_records<R>(n) + sizeof(double) * size_t(8 * n_tiles + 8 * kTotalsBlocks);
}

// The force pass with its scratch given: rec holds n records, partials
// 8 (n_tiles + kTotalsBlocks) doubles.
template <class R>
int accel_run(crk_leaves* L, const crk_gas* g, const R* V, const R* rho, const crk_corr* C,
              double gamma, R* a, R* dudt, double* totals, RecAcc<R>* rec, double* partials,
              hipStream_t st, double eps_u = -1.0) {
    const int n = int(L->n);
    int rc = pack_positions<R>(L, g->x, g->y, g->z, static_cast<const R*>(g->h), st);
    if (rc) return rc;
    {
    TimeScope tp(L, st, CRK_K_PACK);
    hipLaunchKernelGGL(k_pack_acc<R>, dim3((n + 255) / 256), dim3(256), 0, st, n, L->perm, L->quant,
                       static_cast<const R*>(g->h), static_cast<const R*>(g->u),
                       static_cast<const R*>(g->vx), static_cast<const R*>(g->vy),
                       static_cast<const R*>(g->vz), V, rho, static_cast<const R*>(C->A),
                       static_cast<const R*>(C->B), static_cast<const R*>(C->dA),
                       static_cast<const R*>(C->dB), R(gamma - 1.0), rec);
    }
    LAUNCH_CHECK("pack_acc");
    reset_queue(L, st);
    {
        TimeScope ts(L, st, CRK_K_ACCEL);
        // eps_u < 0: the symmetric energy partition
        const bool o32 = off32<RecAcc<R>>(L), compat = eps_u >= 0.0;
        auto kern = compat ? (o32 ? k_accel<R, true, true> : k_accel<R, false, true>)
                           : (o32 ? k_accel<R, true, false> : k_accel<R, false, false>);
        const int bw = L->tune.block_waves;
        hipLaunchKernelGGL(kern, dim3(grid_nwave(L)), dim3(kWave * bw), stage_bytes<RecAcc<R>>(bw), st,
                           make_queue(L, L->order_pair), n, lists(L), L->perm, rec,
                           static_cast<const R*>(g->m), R(compat ? eps_u : 0.0), L->tune.kahan_chunk, a, dudt,
                           partials);
    }
    LAUNCH_CHECK("accel");
    if (totals) {
        TimeScope tt(L, st, CRK_K_PACK);
        const int nt = int(L->n_tiles);
        const int per = (nt + kTotalsBlocks - 1) / kTotalsBlocks;
        double* blocks = partials + 8 * int64_t(nt);  // kTotalsBlocks x 8 after the tile partials
        hipLaunchKernelGGL(k_totals_blocks, dim3(kTotalsBlocks), dim3(256), 0, st, nt, per, partials, blocks);
        hipLaunchKernelGGL(k_totals_blocks, dim3(1), dim3(256), 0, st, kTotalsBlocks, kTotalsBlocks, blocks,
                           totals);
        LAUNCH_CHECK("totals");
    }
    return CRK_OK;
}

// The force pass on the handle's workspace.
template <class R>
int accel_impl(crk_leaves* L, const crk_gas* g, const R* V, const R* rho, const crk_corr* C,
               double gamma, R* a, R* dudt, double* totals, hipStream_t st, double eps_u = -1.0) {
    void* sp = nullptr;
    int rc = pass_scratch(L, sizeof(RecAcc<R>) * size_t(L->n), &sp);
    if (rc) return rc;
    return accel_run<R>(L, g, V, rho, C, gamma, a, dudt, totals, static_cast<RecAcc<R>*>(sp), L->partials, st,
                        eps_u);
}

// The force pass with the artificial viscosity (dv: velocity gradients, 9 per
// particle in caller order, from the Extras pass).
template <class R>
int accel_visc_impl(crk_leaves* L, const crk_gas* g, const R* V, const R* rho, const crk_corr* C, const R* dv,
                    const crk_visc* q, double gamma, R* a, R* dudt, double* totals, hipStream_t st,
                    double eps_u = -1.0) {
    const int n = int(L->n);
    int rc = pack_positions<R>(L, g->x, g->y, g->z, static_cast<const R*>(g->h), st);
    if (rc) return rc;
    void* sp = nullptr;
    if ((rc = pass_scratch(L, sizeof(RecAccV<R>) * size_t(n), &sp))) return rc;
    RecAccV<R>* rec = static_cast<RecAccV<R>*>(sp);
    const ViscParams vp{q->Cl, q->Cq, q->eps_q, gamma};
    {
        TimeScope tp(L, st, CRK_K_PACK);
        hipLaunchKernelGGL(k_pack_acc_visc<R>, dim3((n + 255) / 256), dim3(256), 0, st, n, L->perm, L->quant,
                           static_cast<const R*>(g->h), static_cast<const R*>(g->u),
                           static_cast<const R*>(g->vx), static_cast<const R*>(g->vy),
                           static_cast<const R*>(g->vz), V, rho, static_cast<const R*>(C->A),
                           static_cast<const R*>(C->B), static_cast<const R*>(C->dA),
                           static_cast<const R*>(C->dB), dv, R(gamma - 1.0), vp, rec);
    }
    LAUNCH_CHECK("pack_acc_visc");
    reset_queue(L, st);
    {
        TimeScope ts(L, st, CRK_K_ACCEL_VISC);
        const bool o32 = off32<RecAccV<R>>(L), compat = eps_u >= 0.0;
        auto kern = compat ? (o32 ? k_accel_visc<R, true, true> : k_accel_visc<R, false, true>)
                           : (o32 ? k_accel_visc<R, true, false> : k_accel_visc<R, false, false>);
        const int bw = L->tune.block_waves;
        hipLaunchKernelGGL(kern, dim3(grid_nwave(L)), dim3(kWave * bw), stage_bytes<RecAccV<R>>(bw), st,
                           make_queue(L, L->order_pair), n, lists(L), L->perm, rec,
                           static_cast<const R*>(g->m), R(q->eps_q), R(compat ? eps_u : 0.0),
                           L->tune.kahan_chunk, a, dudt, L->partials);
    }
    LAUNCH_CHECK("accel_visc");
    if (totals) {
        TimeScope tt(L, st, CRK_K_PACK);
        const int nt = int(L->n_tiles);
        const int per = (nt + kTotalsBlocks - 1) / kTotalsBlocks;
        double* blocks = L->partials + 8 * int64_t(nt);
        hipLaunchKernelGGL(k_totals_blocks, dim3(kTotalsBlocks), dim3(256), 0, st, nt, per, L->partials, blocks);
        hipLaunchKernelGGL(k_totals_blocks, dim3(1), dim3(256), 0, st, kTotalsBlocks, kTotalsBlocks, blocks,
                           totals);
        LAUNCH_CHECK("totals");
    }
    return CRK_OK;
}

// ---------------------------------------------------------------- force pass without a workspace
// Scratch of crk_accel_energy_noalloc: a fixed array in device memory, one per
// GPU, held from the library's first use on that GPU until the process ends.
// Host code never uses the array's name as an address: the device address is
// looked up once per device (hipGetSymbolAddress, with that device current)
// and kept in noalloc_ptr.
constexpr size_t kNoAllocBytes = size_t(80) << 20;
static __device__ __align__(256) char noalloc_scratch[kNoAllocBytes];
constexpr int kMaxDevices = 64;
std::mutex noalloc_mutex;
void* noalloc_ptr[kMaxDevices] = {};

int noalloc_scratch_of_device(void** out) {
    int dev = 0;
    HIP_TRY(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices) return fail(CRK_EINVAL, "device %d beyond the %d supported", dev, kMaxDevices);
    std::lock_guard<std::mutex> lock(noalloc_mutex);
    if (!noalloc_ptr[dev]) {
        void* p = nullptr;
        HIP_TRY(hipGetSymbolAddress(&p, HIP_SYMBOL(noalloc_scratch)));
        if (!p) return fail(CRK_EHIP, "no device address for the static scratch on device %d", dev);
        noalloc_ptr[dev] = p;
    }
    *out = noalloc_ptr[dev];
    return CRK_OK;
}

template <class R>
int accel_noalloc_impl(crk_leaves* L, const crk_gas* g, const R* V, const R* rho, const crk_corr* C,
                       double gamma, R* a, R* dudt, double* totals, hipStream_t st) {
    const size_t need = accel_scratch_bytes<R>(L->n, L->n_tiles);
    if (need > kNoAllocBytes)
        return fail(CRK_EINVAL, "crk_accel_energy_noalloc: n = %lld needs %zu bytes of scratch; the static "
                    "array holds %zu (use crk_accel_energy)", (long long)L->n, need, kNoAllocBytes);
    void* base = nullptr;
    int rc = noalloc_scratch_of_device(&base);
    if (rc) return rc;
    char* p = static_cast<char*>(base);
    return accel_run<R>(L, g, V, rho, C, gamma, a, dudt, totals, reinterpret_cast<RecAcc<R>*>(p),
                        reinterpret_cast<double*>(p + accel_scratch_records<R>(L->n)), st);
}


}  // namespace

// ====================================================================== C ABI
// ====================================================================== C ABI

extern "C" {

const char* crk_last_error(void) { return crk::g_err.c_str(); }

int crk_timing(crk_leaves* L, int enable) {
    if (!L) return fail(CRK_EINVAL, "null handle");
    HIP_TRY(hipDeviceSynchronize());
    drop_timed(L);
    L->timing = enable != 0;
    return CRK_OK;
}

int crk_kernel_times(crk_leaves* L, double* ms, int64_t* launches) {
    if (!L || !ms || !launches) return fail(CRK_EINVAL, "null argument");
    for (int k = 0; k < CRK_K_COUNT; ++k) { ms[k] = 0.0; launches[k] = 0; }
    for (auto& t : L->timed) {
        HIP_TRY(hipEventSynchronize(t.b));
        float v = 0.f;
        HIP_TRY(hipEventElapsedTime(&v, t.a, t.b));
        ms[t.kind] += v;
        launches[t.kind] += 1;
    }
    return CRK_OK;
}

void crk_leaves_free(crk_leaves* L) {
    if (!L) return;
    drop_timed(L);
    delete L;
}

int crk_queue_visits(crk_leaves* L, int32_t* visits, hipStream_t st) {
    if (!L || !visits) return fail(CRK_EINVAL, "null argument");
    if (L->n_tiles == 0) return CRK_OK;
    reset_queue(L, st);
    hipLaunchKernelGGL(k_queue_visits, dim3(grid_nwave(L)), dim3(kWave * L->tune.block_waves), 0, st,
                       make_queue(L, L->order_pair), visits);
    LAUNCH_CHECK("queue visits");
    return CRK_OK;
}

int crk_leaves_perm(const crk_leaves* L, int32_t* perm, hipStream_t st) {
    if (!L || (!perm && L->n > 0)) return fail(CRK_EINVAL, "null argument");
    if (L->n == 0) return CRK_OK;
    HIP_TRY(hipMemcpyAsync(perm, L->perm, size_t(L->n) * sizeof(int32_t), hipMemcpyDeviceToDevice, st));
    return CRK_OK;
}

int crk_get_tuning(const crk_leaves* L, crk_tuning* out) {
    if (!L || !out) return fail(CRK_EINVAL, "null argument");
    *out = L->tune;
    return CRK_OK;
}

int crk_set_tuning(crk_leaves* L, const crk_tuning* in) {
    if (!L || !in) return fail(CRK_EINVAL, "null argument");
    if (in->persistent != 0 && in->persistent != 1) return fail(CRK_EINVAL, "persistent must be 0 or 1");
    if (in->waves_per_cu < 1 || in->waves_per_cu > 64) return fail(CRK_EINVAL, "waves_per_cu in [1, 64]");
    if (in->kahan_chunk < 1 || in->kahan_chunk > 64 || (in->kahan_chunk & (in->kahan_chunk - 1)))
        return fail(CRK_EINVAL, "kahan_chunk must be a power of two in [1, 64]");
    if (in->block_waves != 1 && in->block_waves != 2 && in->block_waves != 4)
        return fail(CRK_EINVAL, "block_waves must be 1, 2 or 4");
    if (in->xcd_groups < 1 || in->xcd_groups > kMaxGroups) return fail(CRK_EINVAL, "xcd_groups in [1, 16]");
    if (in->tile_order != 0 && in->tile_order != 1) return fail(CRK_EINVAL, "tile_order must be 0 or 1");
    if (in->addr64 != 0 && in->addr64 != 1) return fail(CRK_EINVAL, "addr64 must be 0 or 1");
    if (in->exchange < 0 || in->exchange > 2) return fail(CRK_EINVAL, "exchange must be 0, 1 or 2");
    if (in->stage16 != 0 && in->stage16 != 1) return fail(CRK_EINVAL, "stage16 must be 0 or 1");
    L->tune = *in;
    return CRK_OK;
}

}  // extern "C"

namespace {

// Host state of the last build that stopped for want of workspace: a call that
// repeats it (same sizes and options, same positions and h) resumes from the
// tree and list counts instead of building them again.
struct BuildMemo {
    bool valid = false;
    bool counted = false;
    int64_t n = 0;
    int leaf_max = 0, leaf_min = 0, hydro = 0;
    double r_fixed = 0.0, split_extent = 0.0;
    std::vector<double> hx, hy, hz, H;
    crk::TreeOutput tree;
    std::vector<int32_t> counts;  // list lengths in the tree's order (when counted)
};
thread_local BuildMemo g_memo;

// Workspace layout of a handle: part A (everything that depends only on n and
// the tile count), then the candidate ranges of the tiles (their number
// depends on where the tiles are cut, which the list-length balancing of the
// hydro build changes), then part B: the neighbour lists and their per-slot
// sets (hydro mode, `slots` list slots).  Returns the bytes used; with a null
// base it only measures.
void carve_part_a(crk_leaves* L, Carver& c, int64_t n, int64_t nt) {
    L->counter = c.take<int32_t>(kMaxGroups);
    L->counts = c.take<unsigned long long>(4);
    L->build_err = c.take<int32_t>(kMaxGroups);  // cleared by k_reset
    L->perm = c.take<int32_t>(n);
    L->quant = c.take<uint4>(n);
    L->rng_off = c.take<int32_t>(nt + 1);
    L->order_cull = c.take<int32_t>(nt);
    L->order_pair = c.take<int32_t>(nt);
    L->order_tree = c.take<int32_t>(nt);
    L->partials = c.take<double>(8 * nt + 8 * kTotalsBlocks);
    if (L->hydro) {
        L->Hd = c.take<double>(n);
        L->cnt = c.take<int32_t>(n);
        L->cnt_gather = c.take<int32_t>(n);
        L->ell_off = c.take<int64_t>(nt);
        L->ell_len = c.take<int32_t>(nt);
        L->ell_len_gather = c.take<int32_t>(nt);
    }
    // per-pass scratch, for both precisions: the backward's records (hydro),
    // the masses and upstream adjoints in tree order (gravity)
    L->scratch_bytes = L->hydro ? std::max(crk::backward_scratch_bytes(n, true),
                                           size_t(n) * sizeof(RecAcc<double>))
                                : size_t(n) * 4 * sizeof(double);  // masses and adjoints (gravity)
    if (L->dev_tree) L->scratch_bytes = std::max(L->scratch_bytes, crk::devtree_scratch_bytes(n, nt));
    // the list schedule's neighbour tables (at least one tile at a time)
    if (L->hydro) L->scratch_bytes = std::max(L->scratch_bytes, sizeof(SchedEntry) * kSchedHash + 8192);
    L->scratch = c.take<char>(L->scratch_bytes);
}

void carve_part_b(crk_leaves* L, Carver& c, int64_t slots) {
    L->nbr = c.take<uint32_t>(size_t(slots));
    L->srec = c.take<uint32_t>(size_t(slots));
    L->sidx = c.take<uint8_t>(size_t(slots));
    L->scnt = c.take<int32_t>(size_t(slots / kWave));
}

// slots < 0: no lists (fixed-radius mode, or hydro before the lists are counted)
size_t carve(crk_leaves* L, char* base, int64_t n, int64_t nt, size_t nr, int64_t slots) {
    Carver c(base);
    carve_part_a(L, c, n, nt);
    L->rng = c.take<int2>(nr);
    if (slots >= 0) carve_part_b(L, c, slots);
    return c.used();
}

// Fill pass of the neighbour lists (cnt, ell_off and ell_len in place), tile
// order of the pair passes (longest lists first, from the per-tile lengths
// len) and the shared-record slots.
int fill_lists(crk_leaves* L, const std::vector<int32_t>& len, hipStream_t stream) {
    const int64_t n = L->n, nt = L->n_tiles;
    hipLaunchKernelGGL(k_reset, dim3(1), dim3(64), 0, stream, L->counter);
    hipLaunchKernelGGL(k_reset, dim3(1), dim3(64), 0, stream, L->build_err);
    {
        TimeScope ts(L, stream, CRK_K_CULL);
        hipLaunchKernelGGL(k_cull<true>, dim3(grid_1wave(L)), dim3(kWave), 0, stream,
                           make_queue(L, L->order_cull), int(n), L->quant, L->rng_off, L->rng,
                           L->cnt, L->ell_off, L->ell_len, L->nbr, L->cnt_gather, L->ell_len_gather,
                           L->build_err, float(L->skin));
    }
    if (hipGetLastError() != hipSuccess) return fail(CRK_EHIP, "launch cull fill failed");
    // pair passes: tiles with the longest lists first
    std::vector<int32_t> po(nt);
    std::iota(po.begin(), po.end(), 0);
    std::stable_sort(po.begin(), po.end(), [&](int32_t a, int32_t b) { return len[a] > len[b]; });
    int32_t mismatched = 0;
    if (hipMemcpyAsync(L->order_pair, po.data(), nt * 4, hipMemcpyHostToDevice, stream) != hipSuccess ||
        hipMemcpyAsync(&mismatched, L->build_err, sizeof(int32_t), hipMemcpyDeviceToHost, stream) !=
            hipSuccess ||
        hipStreamSynchronize(stream) != hipSuccess)
        return fail(CRK_EHIP, "list build failed");
    if (mismatched)
        return fail(CRK_EHIP, "neighbour lists: count and fill passes disagree on %d particles", mismatched);
    // shared-record slots: reorder the lists, name each slot's particles; in
    // batches of tiles whose neighbour tables fit the per-pass scratch
    const size_t per_tile = sizeof(SchedEntry) * kSchedHash + 3 * sizeof(int32_t) + 16;
    const int64_t batch = std::min<int64_t>(nt, int64_t((L->scratch_bytes - 4096) / per_tile));
    if (batch < 1) return fail(CRK_EHIP, "list schedule: per-pass scratch of %zu bytes too small", L->scratch_bytes);
    {
        Carver cv(static_cast<char*>(L->scratch));
        SchedEntry* tbl = cv.take<SchedEntry>(size_t(batch) * kSchedHash);
        int32_t* tcnt = cv.take<int32_t>(size_t(batch));
        int32_t* list16 = cv.take<int32_t>(size_t(batch));
        int32_t* list32 = cv.take<int32_t>(size_t(batch));
        int32_t* counts = cv.take<int32_t>(kMaxGroups);  // k_reset clears kMaxGroups
        for (int64_t t0 = 0; t0 < nt; t0 += batch) {
            const int nb = int(std::min<int64_t>(batch, nt - t0));
            int32_t hc[2] = {0, 0};
            {
                TimeScope ts(L, stream, CRK_K_CULL);
                hipLaunchKernelGGL(k_sched_table, dim3(unsigned(nb)), dim3(kWave), 0, stream, int(n), int(t0),
                                   L->cnt, L->cnt_gather, L->ell_off, L->ell_len, L->nbr, L->srec, L->sidx,
                                   L->scnt, tbl, tcnt);
                hipLaunchKernelGGL(k_reset, dim3(1), dim3(64), 0, stream, counts);
                hipLaunchKernelGGL(k_sched_bins, dim3((nb + 255) / 256), dim3(256), 0, stream, nb, tcnt, list16,
                                   list32, counts);
            }
            if (hipGetLastError() != hipSuccess ||
                hipMemcpyAsync(hc, counts, sizeof hc, hipMemcpyDeviceToHost, stream) != hipSuccess ||
                hipStreamSynchronize(stream) != hipSuccess)
                return fail(CRK_EHIP, "list schedule (tables) failed");
            TimeScope ts(L, stream, CRK_K_CULL);
            if (hc[0] > 0)
                hipLaunchKernelGGL(k_sched_pick<16>, dim3(unsigned(hc[0])), dim3(kWave), 0, stream, int(n),
                                   int(t0), list16, L->cnt, L->cnt_gather, L->ell_off, L->ell_len, L->nbr,
                                   L->srec, L->sidx, L->scnt, tbl, tcnt);
            if (hc[1] > 0)
                hipLaunchKernelGGL(k_sched_pick<kSchedRegs>, dim3(unsigned(hc[1])), dim3(kWave), 0, stream,
                                   int(n), int(t0), list32, L->cnt, L->cnt_gather, L->ell_off, L->ell_len, L->nbr,
                                   L->srec, L->sidx, L->scnt, tbl, tcnt);
        }
    }
    if (hipGetLastError() != hipSuccess || hipStreamSynchronize(stream) != hipSuccess)
        return fail(CRK_EHIP, "list schedule failed");
    return CRK_OK;
}

}  // namespace

extern "C" int crk_build_leaf_pairs(int64_t n, const double* x, const double* y, const double* z,
                         const void* h, double r_fixed, int leaf_max, int leaf_min,
                         double split_extent, crk_prec prec, void* ws, size_t ws_bytes,
                         size_t* ws_needed, crk_leaves** out, hipStream_t stream) {
    if (!out || !ws_needed) return fail(CRK_EINVAL, "out and ws_needed must not be NULL");
    *out = nullptr;
    *ws_needed = 0;
    if (n < 0 || n >= (int64_t(1) << 31)) return fail(CRK_EINVAL, "n = %lld out of range [0, 2^31)", (long long)n);
    if (prec != CRK_F32 && prec != CRK_F64) return fail(CRK_EINVAL, "unknown precision");
    if (leaf_max < 1 || leaf_max > (1 << 20)) return fail(CRK_EINVAL, "leaf_max out of range [1, 2^20]");
    if (leaf_min < 1) return fail(CRK_EINVAL, "leaf_min must be >= 1");
    if (n > 0 && !h && !(r_fixed > 0.0 && r_fixed < 0.5))
        return fail(CRK_EINVAL, "fixed radius must be in (0, 1/2) of the box");
    if (h && !(r_fixed >= 0.0 && r_fixed < 0.5))
        return fail(CRK_EINVAL, "list skin (r_fixed in hydro mode) must be in [0, 1/2)");
    if (n > 0 && (!x || !y || !z)) return fail(CRK_EINVAL, "positions are NULL");
    if (ws_bytes > 0 && !ws) return fail(CRK_EINVAL, "ws is NULL but ws_bytes = %zu", ws_bytes);
    if (reinterpret_cast<uintptr_t>(ws) % 256 != 0) return fail(CRK_EINVAL, "ws must be 256-byte aligned");
    const auto t0 = std::chrono::steady_clock::now();

    crk_leaves* L = new crk_leaves();
    L->n = n;
    L->hydro = h != nullptr;
    L->prec = prec;
    L->r_fixed = h ? 0.0 : r_fixed;
    L->skin = h ? r_fixed : 0.0;
    L->ws = static_cast<char*>(ws);
    L->ws_bytes = ws_bytes;
    int dev = 0;
    auto bail = [&](int code) {
        drop_timed(L);
        delete L;
        return code;
    };
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&L->n_cu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
        return bail(fail(CRK_EHIP, "cannot query the device"));
    const int64_t nt = (n + kWave - 1) / kWave;
    L->n_tiles = nt;
    if (n == 0) {
        *ws_needed = carve(L, nullptr, 0, 0, 0, -1);
        if (ws_bytes < *ws_needed) return bail(fail(CRK_ENOSPC, "workspace of %zu bytes, need %zu", ws_bytes, *ws_needed));
        carve(L, L->ws, 0, 0, 0, -1);
        *out = L;
        return CRK_OK;
    }

    // positions (and h) to the host
    std::vector<double> hx(n), hy(n), hz(n), H;
    if (hipMemcpyAsync(hx.data(), x, n * 8, hipMemcpyDeviceToHost, stream) != hipSuccess ||
        hipMemcpyAsync(hy.data(), y, n * 8, hipMemcpyDeviceToHost, stream) != hipSuccess ||
        hipMemcpyAsync(hz.data(), z, n * 8, hipMemcpyDeviceToHost, stream) != hipSuccess)
        return bail(fail(CRK_EHIP, "copying positions to the host failed"));
    if (L->hydro) {
        H.resize(n);
        if (prec == CRK_F32) {
            std::vector<float> hf(n);
            if (hipMemcpyAsync(hf.data(), h, n * 4, hipMemcpyDeviceToHost, stream) != hipSuccess ||
                hipStreamSynchronize(stream) != hipSuccess)
                return bail(fail(CRK_EHIP, "copying h to the host failed"));
            for (int64_t i = 0; i < n; ++i) H[i] = 2.0 * double(hf[i]);
        } else {
            if (hipMemcpyAsync(H.data(), h, n * 8, hipMemcpyDeviceToHost, stream) != hipSuccess ||
                hipStreamSynchronize(stream) != hipSuccess)
                return bail(fail(CRK_EHIP, "copying h to the host failed"));
            for (int64_t i = 0; i < n; ++i) H[i] = 2.0 * H[i];
        }
    }
    if (hipStreamSynchronize(stream) != hipSuccess) return bail(fail(CRK_EHIP, "stream sync failed"));
    std::vector<uint32_t> q[3];
    for (int a = 0; a < 3; ++a) q[a].resize(n);
    double Hmax = 0.0;
    for (int64_t i = 0; i < n; ++i) {
        const double p[3] = {hx[i], hy[i], hz[i]};
        for (int a = 0; a < 3; ++a) {
            if (!std::isfinite(p[a])) return bail(fail(CRK_EINVAL, "non-finite position at %lld", (long long)i));
            const double t = p[a] - std::floor(p[a]);
            const double v = std::floor(t * 4294967296.0 + 0.5);
            q[a][i] = v >= 4294967296.0 ? 0u : uint32_t(v);
        }
        if (L->hydro) {
            if (!(H[i] > 0.0) || !std::isfinite(H[i]))
                return bail(fail(CRK_EINVAL, "h must be positive and finite (particle %lld)", (long long)i));
            Hmax = std::max(Hmax, H[i]);
        }
    }
    if (L->hydro && !(Hmax + L->skin < 0.5))
        return bail(fail(CRK_EINVAL, "2 max(h) + skin = %g must be below half the box", Hmax + L->skin));
    // the tree and the list build see every support widened by the skin
    std::vector<double> Hs;
    if (L->hydro && L->skin > 0.0) {
        Hs.resize(n);
        for (int64_t i = 0; i < n; ++i) Hs[i] = H[i] + L->skin;
    }

    crk::TreeInput tin;
    tin.n = n;
    for (int a = 0; a < 3; ++a) tin.q[a] = q[a].data();
    tin.H = L->hydro ? (Hs.empty() ? H.data() : Hs.data()) : nullptr;
    tin.r_fixed = r_fixed;
    tin.leaf_max = leaf_max;
    tin.leaf_min = leaf_min;
    tin.split_extent = split_extent;
    // the same call as the one that last ran out of workspace: resume from its host state
    BuildMemo& memo = g_memo;
    const bool resume = memo.valid && memo.n == n && memo.leaf_max == leaf_max && memo.leaf_min == leaf_min &&
                        memo.hydro == L->hydro && memo.r_fixed == r_fixed && memo.split_extent == split_extent &&
                        memo.hx == hx && memo.hy == hy && memo.hz == hz && memo.H == H;
    crk::TreeOutput tout;
    std::vector<int32_t> hc;  // list lengths in tree order
    bool counted = false;
    const char* terr = nullptr;
    if (resume) {
        tout = std::move(memo.tree);
        hc = std::move(memo.counts);
        counted = memo.counted;
    } else if (!crk::build_tree(tin, tout, &terr)) {
        return bail(fail(CRK_EINVAL, "tree: %s", terr));
    }
    memo.valid = false;
    auto keep_for_retry = [&](bool with_counts) {
        memo.valid = true;
        memo.counted = with_counts;
        memo.n = n;
        memo.leaf_max = leaf_max;
        memo.leaf_min = leaf_min;
        memo.hydro = L->hydro;
        memo.r_fixed = r_fixed;
        memo.split_extent = split_extent;
        memo.hx = std::move(hx);
        memo.hy = std::move(hy);
        memo.hz = std::move(hz);
        memo.H = std::move(H);
        memo.tree = std::move(tout);
        memo.counts = std::move(hc);
    };
    L->n_leaves = int64_t(tout.leaf_begin.size());
    auto ranges = [](const crk::TreeOutput& t) { return t.rng.size() / 2; };

    // tree-order fixed-point positions and support radii, candidate ranges and
    // the tile orders of one tree order, uploaded (host buffers must outlive
    // the asynchronous copies: they are synchronised before reuse)
    std::vector<uint4> hq(n);
    std::vector<double> hH(L->hydro ? n : 0);
    std::vector<int32_t> order(nt), tree_order(nt);
    std::iota(tree_order.begin(), tree_order.end(), 0);
    auto upload = [&](const crk::TreeOutput& t) -> int {
        const size_t nr = ranges(t);
        for (int64_t s = 0; s < n; ++s) {
            const int32_t i = t.perm[s];
            uint32_t hw = 0;
            if (L->hydro) {
                const float hf = float(H[i]);
                std::memcpy(&hw, &hf, 4);
                hH[s] = H[i];
            }
            hq[s] = make_uint4(q[0][i], q[1][i], q[2][i], hw);
        }
        // longest-processing-time-first order of tiles for the candidate scan
        std::iota(order.begin(), order.end(), 0);
        std::stable_sort(order.begin(), order.end(),
                         [&](int32_t a, int32_t b) { return t.tile_cand[a] > t.tile_cand[b]; });
        if (hipMemcpyAsync(L->perm, t.perm.data(), n * 4, hipMemcpyHostToDevice, stream) != hipSuccess ||
            hipMemcpyAsync(L->quant, hq.data(), n * 16, hipMemcpyHostToDevice, stream) != hipSuccess ||
            hipMemcpyAsync(L->rng_off, t.rng_off.data(), (nt + 1) * 4, hipMemcpyHostToDevice, stream) !=
                hipSuccess ||
            (nr && hipMemcpyAsync(L->rng, t.rng.data(), nr * 8, hipMemcpyHostToDevice, stream) != hipSuccess) ||
            hipMemcpyAsync(L->order_cull, order.data(), nt * 4, hipMemcpyHostToDevice, stream) != hipSuccess ||
            hipMemcpyAsync(L->order_pair, order.data(), nt * 4, hipMemcpyHostToDevice, stream) != hipSuccess ||
            hipMemcpyAsync(L->order_tree, tree_order.data(), nt * 4, hipMemcpyHostToDevice, stream) !=
                hipSuccess ||
            (L->hydro && hipMemcpyAsync(L->Hd, hH.data(), n * 8, hipMemcpyHostToDevice, stream) != hipSuccess) ||
            hipStreamSynchronize(stream) != hipSuccess)
            return fail(CRK_EHIP, "uploading the tree failed");
        L->stats[2] = t.cand_pairs;
        return CRK_OK;
    };
    int rc = CRK_OK;
    L->stats[0] = L->n_leaves;
    L->stats[1] = nt;

    if (!L->hydro) {
        *ws_needed = carve(L, nullptr, n, nt, ranges(tout), -1);
        if (*ws_needed > ws_bytes) {
            keep_for_retry(false);
            return bail(fail(CRK_ENOSPC, "workspace of %zu bytes, need %zu", ws_bytes, *ws_needed));
        }
        carve(L, L->ws, n, nt, ranges(tout), -1);
        if ((rc = upload(tout))) return bail(rc);
    } else {
        L->timing = true;  // the list build is always timed (read by crk_kernel_times)
        if (!counted) {
            // count pass on the first tree, in a workspace without the lists
            *ws_needed = carve(L, nullptr, n, nt, ranges(tout), -1);
            if (*ws_needed > ws_bytes) {
                keep_for_retry(false);  // the lists come on top: not counted yet
                return bail(fail(CRK_ENOSPC, "workspace of %zu bytes, need at least %zu (before the lists)",
                                 ws_bytes, *ws_needed));
            }
            carve(L, L->ws, n, nt, ranges(tout), -1);
            if ((rc = upload(tout))) return bail(rc);
            hipLaunchKernelGGL(k_reset, dim3(1), dim3(64), 0, stream, L->counter);
            {
                TimeScope ts(L, stream, CRK_K_CULL);
                hipLaunchKernelGGL(k_cull<false>, dim3(grid_1wave(L)), dim3(kWave), 0, stream,
                                   make_queue(L, L->order_cull), int(n), L->quant, L->rng_off, L->rng,
                                   L->cnt, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr,
                                   float(L->skin));
            }
            if (hipGetLastError() != hipSuccess) return bail(fail(CRK_EHIP, "launch cull count failed"));
            hc.resize(n);
            if (hipMemcpyAsync(hc.data(), L->cnt, n * 4, hipMemcpyDeviceToHost, stream) != hipSuccess ||
                hipStreamSynchronize(stream) != hipSuccess)
                return bail(fail(CRK_EHIP, "cull count failed"));
            // Tiles of similar list lengths: order every leaf by decreasing count
            // (the leaves, their boxes and every particle's count stay the same;
            // only the tiles and their candidate ranges change), so that a tile's
            // longest list -- the slots all its lanes step through -- is closer
            // to its average one.
            std::vector<int32_t> work(n);
            for (int64_t s = 0; s < n; ++s) work[tout.perm[s]] = hc[s];
            tin.weight = work.data();
            crk::TreeOutput tb;
            if (!crk::build_tree(tin, tb, &terr)) return bail(fail(CRK_EINVAL, "tree: %s", terr));
            if (int64_t(tb.leaf_begin.size()) != L->n_leaves)
                return bail(fail(CRK_EHIP, "tree rebuild changed the leaves"));
            tout = std::move(tb);
            for (int64_t s = 0; s < n; ++s) hc[s] = work[tout.perm[s]];
            counted = true;
        }
        // the final tree and its list lengths (tree order): list offsets per tile
        std::vector<int32_t> len(nt, 0);
        std::vector<int64_t> off(nt, 0);
        int64_t total = 0, entries = 0;
        for (int64_t t = 0; t < nt; ++t) {
            int32_t mx = 0;
            for (int64_t s = t * kWave; s < std::min<int64_t>(n, (t + 1) * kWave); ++s) {
                mx = std::max(mx, hc[s]);
                entries += hc[s];
            }
            len[t] = mx;
            off[t] = total;
            total += int64_t(mx) * kWave;
        }
        *ws_needed = carve(L, nullptr, n, nt, ranges(tout), total);
        if (*ws_needed > ws_bytes) {
            keep_for_retry(true);
            return bail(fail(CRK_ENOSPC, "workspace of %zu bytes, need %zu", ws_bytes, *ws_needed));
        }
        carve(L, L->ws, n, nt, ranges(tout), total);
        if ((rc = upload(tout))) return bail(rc);
        if (hipMemcpyAsync(L->cnt, hc.data(), n * 4, hipMemcpyHostToDevice, stream) != hipSuccess ||
            hipMemcpyAsync(L->ell_off, off.data(), nt * 8, hipMemcpyHostToDevice, stream) != hipSuccess ||
            hipMemcpyAsync(L->ell_len, len.data(), nt * 4, hipMemcpyHostToDevice, stream) != hipSuccess ||
            hipStreamSynchronize(stream) != hipSuccess)
            return bail(fail(CRK_EHIP, "uploading list counts and offsets failed"));
        if ((rc = fill_lists(L, len, stream))) return bail(rc);
        L->stats[3] = entries;
        L->stats[6] = total - entries;
    }
    L->timing = false;
    if (hipStreamSynchronize(stream) != hipSuccess) return bail(fail(CRK_EHIP, "build sync failed"));
    L->stats[7] = std::chrono::duration_cast<std::chrono::microseconds>(
                      std::chrono::steady_clock::now() - t0).count();
    *out = L;
    return CRK_OK;
}

// The same handle built on the device: Morton octree leaves, tile candidate
// ranges and neighbour lists without the positions' round trip to the host.
// A run that stops with CRK_ENOSPC keeps no state: the repeated call rebuilds
// (the build is deterministic, so it reaches the same sizes).
extern "C" int crk_build_leaf_pairs_device(int64_t n, const double* x, const double* y, const double* z,
                                           const void* h, double r_fixed, int leaf_max, crk_prec prec, void* ws,
                                           size_t ws_bytes, size_t* ws_needed, crk_leaves** out,
                                           hipStream_t stream) {
    if (!out || !ws_needed) return fail(CRK_EINVAL, "out and ws_needed must not be NULL");
    *out = nullptr;
    *ws_needed = 0;
    if (n < 0 || n >= (int64_t(1) << 31)) return fail(CRK_EINVAL, "n = %lld out of range [0, 2^31)", (long long)n);
    if (prec != CRK_F32 && prec != CRK_F64) return fail(CRK_EINVAL, "unknown precision");
    if (leaf_max < 1 || leaf_max > kDevLeafMax)
        return fail(CRK_EINVAL, "leaf_max out of range [1, %d] for the device build", kDevLeafMax);
    if (n > 0 && !h && !(r_fixed > 0.0 && r_fixed < 0.5))
        return fail(CRK_EINVAL, "fixed radius must be in (0, 1/2) of the box");
    if (h && !(r_fixed >= 0.0 && r_fixed < 0.5))
        return fail(CRK_EINVAL, "list skin (r_fixed in hydro mode) must be in [0, 1/2)");
    if (n > 0 && (!x || !y || !z)) return fail(CRK_EINVAL, "positions are NULL");
    if (ws_bytes > 0 && !ws) return fail(CRK_EINVAL, "ws is NULL but ws_bytes = %zu", ws_bytes);
    if (reinterpret_cast<uintptr_t>(ws) % 256 != 0) return fail(CRK_EINVAL, "ws must be 256-byte aligned");
    const auto t0 = std::chrono::steady_clock::now();

    crk_leaves* L = new crk_leaves();
    L->n = n;
    L->hydro = h != nullptr;
    L->prec = prec;
    L->r_fixed = h ? 0.0 : r_fixed;
    L->skin = h ? r_fixed : 0.0;
    L->dev_tree = true;
    L->ws = static_cast<char*>(ws);
    L->ws_bytes = ws_bytes;
    int dev = 0;
    auto bail = [&](int code) {
        drop_timed(L);
        delete L;
        return code;
    };
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&L->n_cu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
        return bail(fail(CRK_EHIP, "cannot query the device"));
    const int64_t nt = (n + kWave - 1) / kWave;
    L->n_tiles = nt;
    if (n == 0) {
        *ws_needed = carve(L, nullptr, 0, 0, 0, -1);
        if (ws_bytes < *ws_needed) return bail(fail(CRK_ENOSPC, "workspace of %zu bytes, need %zu", ws_bytes, *ws_needed));
        carve(L, L->ws, 0, 0, 0, -1);
        *out = L;
        return CRK_OK;
    }
    // part A holds the build's temporaries (in the per-pass scratch)
    *ws_needed = carve(L, nullptr, n, nt, 0, -1);
    if (*ws_needed > ws_bytes)
        return bail(fail(CRK_ENOSPC, "workspace of %zu bytes, need at least %zu (before the candidate ranges)",
                         ws_bytes, *ws_needed));
    carve(L, L->ws, n, nt, 0, -1);
    int rc = devtree_leaves(L, x, y, z, h, leaf_max, stream);
    if (rc) return bail(rc);
    L->stats[0] = L->n_leaves;
    L->stats[1] = nt;

    // candidate ranges of the tiles of the current tree order; the tile order
    // of the list build: most candidates first
    std::vector<int64_t> tile_cand;
    std::vector<int32_t> order(nt), tree_order(nt);
    std::iota(tree_order.begin(), tree_order.end(), 0);
    int64_t nr = 0;
    auto ranges_and_orders = [&](int64_t slots) -> int {
        int r = devtree_ranges(L, nullptr, &nr, &tile_cand, stream);
        if (r) return r;
        *ws_needed = carve(L, nullptr, n, nt, size_t(nr), slots);
        if (*ws_needed > ws_bytes)
            return fail(CRK_ENOSPC, "workspace of %zu bytes, need %s%zu", ws_bytes,
                        slots < 0 && L->hydro ? "at least " : "", *ws_needed);
        carve(L, L->ws, n, nt, size_t(nr), slots);
        if ((r = devtree_ranges(L, L->rng, nullptr, nullptr, stream))) return r;
        std::iota(order.begin(), order.end(), 0);
        std::stable_sort(order.begin(), order.end(),
                         [&](int32_t a, int32_t b) { return tile_cand[a] > tile_cand[b]; });
        int64_t cp = 0;
        for (int64_t t = 0; t < nt; ++t) cp += tile_cand[t] * (std::min<int64_t>(n, (t + 1) * kWave) - t * kWave);
        L->stats[2] = cp;
        if (hipMemcpyAsync(L->order_cull, order.data(), nt * 4, hipMemcpyHostToDevice, stream) != hipSuccess ||
            hipMemcpyAsync(L->order_pair, order.data(), nt * 4, hipMemcpyHostToDevice, stream) != hipSuccess ||
            hipMemcpyAsync(L->order_tree, tree_order.data(), nt * 4, hipMemcpyHostToDevice, stream) !=
                hipSuccess ||
            hipStreamSynchronize(stream) != hipSuccess)
            return fail(CRK_EHIP, "uploading the tile orders failed");
        return CRK_OK;
    };
    if ((rc = ranges_and_orders(-1))) return bail(rc);
    if (L->hydro) {
        L->timing = true;  // the list build is always timed (read by crk_kernel_times)
        hipLaunchKernelGGL(k_reset, dim3(1), dim3(64), 0, stream, L->counter);
        {
            TimeScope ts(L, stream, CRK_K_CULL);
            hipLaunchKernelGGL(k_cull<false>, dim3(grid_1wave(L)), dim3(kWave), 0, stream,
                               make_queue(L, L->order_cull), int(n), L->quant, L->rng_off, L->rng, L->cnt,
                               nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, float(L->skin));
        }
        if (hipGetLastError() != hipSuccess) return bail(fail(CRK_EHIP, "launch cull count failed"));
        // tiles of similar list lengths: every leaf by decreasing count (its
        // box stays the same; the tiles and their candidates change)
        if ((rc = devtree_sort_leaves(L, stream))) return bail(rc);
        std::vector<int32_t> len;
        int64_t total = 0, entries = 0;
        if ((rc = devtree_list_layout(L, &total, &entries, &len, stream))) return bail(rc);
        if ((rc = ranges_and_orders(total))) return bail(rc);
        if ((rc = fill_lists(L, len, stream))) return bail(rc);
        L->stats[3] = entries;
        L->stats[6] = total - entries;
    }
    L->timing = false;
    if (hipStreamSynchronize(stream) != hipSuccess) return bail(fail(CRK_EHIP, "build sync failed"));
    L->stats[7] = std::chrono::duration_cast<std::chrono::microseconds>(
                      std::chrono::steady_clock::now() - t0).count();
    *out = L;
    return CRK_OK;
}

extern "C" {

int crk_leaves_stats(crk_leaves* L, int64_t* host_out) {
    if (!L || !host_out) return fail(CRK_EINVAL, "null argument");
    if (!L->counted && L->n > 0) {
        HIP_TRY(hipDeviceSynchronize());
        HIP_TRY(hipMemset(L->counts, 0, 4 * sizeof(unsigned long long)));
        if (L->hydro) {
            hipLaunchKernelGGL(k_count_lists, dim3((L->n + 255) / 256), dim3(256), 0, 0, int(L->n),
                               L->quant, L->Hd, L->cnt, L->ell_off, L->nbr, L->counts);
        } else {
            hipLaunchKernelGGL(k_count_fixed, dim3(L->n_tiles), dim3(64), 0, 0, int(L->n_tiles),
                               int(L->n), L->quant, L->rng_off, L->rng, L->r_fixed, L->counts);
        }
        LAUNCH_CHECK("count");
        unsigned long long c[4];
        HIP_TRY(hipMemcpy(c, L->counts, sizeof c, hipMemcpyDeviceToHost));
        L->stats[4] = int64_t(c[0]);
        L->stats[5] = int64_t(L->hydro ? c[1] : c[0]);
        L->counted = true;
    }
    for (int k = 0; k < 8; ++k) host_out[k] = L->stats[k];
    return CRK_OK;
}

int crk_volume(crk_leaves* L, const crk_gas* g, crk_prec prec, void* V, void* rho, hipStream_t st) {
    int rc = check_gas(L, g, false);
    if (rc) return rc;
    if (L->n == 0) return CRK_OK;
    if (!g->m || !V || !rho) return fail(CRK_EINVAL, "m, V and rho are required");
    if (prec == CRK_F32) return volume_impl<float>(L, g, (float*)V, (float*)rho, st);
    if (prec == CRK_F64) return volume_impl<double>(L, g, (double*)V, (double*)rho, st);
    return fail(CRK_EINVAL, "unknown precision");
}

int crk_corrections(crk_leaves* L, const crk_gas* g, const void* V, crk_prec prec,
                    const crk_corr* out, int64_t* n_fallback, hipStream_t st) {
    int rc = check_gas(L, g, false);
    if (rc) return rc;
    if (L->n == 0) return CRK_OK;
    if (!V || !out || !out->A || !out->B || !out->dA || !out->dB)
        return fail(CRK_EINVAL, "V and all correction outputs are required");
    if (prec == CRK_F32) return corrections_impl<float>(L, g, (const float*)V, out, n_fallback, st);
    if (prec == CRK_F64) return corrections_impl<double>(L, g, (const double*)V, out, n_fallback, st);
    return fail(CRK_EINVAL, "unknown precision");
}

static int accel_entry(bool noalloc, crk_leaves* L, const crk_gas* g, const void* V, const void* rho,
                       const crk_corr* C, double gamma, crk_prec prec, void* a, void* dudt, double* totals,
                       hipStream_t st) {
    int rc = check_gas(L, g, true);
    if (rc) return rc;
    if (L->n == 0) {
        if (totals) {  // a fill kernel, not a memset: callers may capture this call in a graph
            hipLaunchKernelGGL(k_zero8, dim3(1), dim3(64), 0, st, totals);
            LAUNCH_CHECK("zero totals");
        }
        return CRK_OK;
    }
    if (!V || !rho || !C || !C->A || !C->B || !C->dA || !C->dB || !a || !dudt)
        return fail(CRK_EINVAL, "V, rho, corrections, a and dudt are required");
    if (prec == CRK_F32) {
        const float *Vf = (const float*)V, *rf = (const float*)rho;
        return noalloc ? accel_noalloc_impl<float>(L, g, Vf, rf, C, gamma, (float*)a, (float*)dudt, totals, st)
                       : accel_impl<float>(L, g, Vf, rf, C, gamma, (float*)a, (float*)dudt, totals, st);
    }
    if (prec == CRK_F64) {
        const double *Vd = (const double*)V, *rd = (const double*)rho;
        return noalloc ? accel_noalloc_impl<double>(L, g, Vd, rd, C, gamma, (double*)a, (double*)dudt, totals, st)
                       : accel_impl<double>(L, g, Vd, rd, C, gamma, (double*)a, (double*)dudt, totals, st);
    }
    return fail(CRK_EINVAL, "unknown precision");
}

int crk_accel_energy(crk_leaves* L, const crk_gas* g, const void* V, const void* rho,
                     const crk_corr* C, double gamma, crk_prec prec, void* a, void* dudt,
                     double* totals, hipStream_t st) {
    return accel_entry(false, L, g, V, rho, C, gamma, prec, a, dudt, totals, st);
}

int crk_accel_energy_visc(crk_leaves* L, const crk_gas* g, const void* V, const void* rho, const crk_corr* C,
                          const void* dv, const crk_visc* q, double gamma, crk_prec prec, void* a, void* dudt,
                          double* totals, hipStream_t st) {
    int rc = check_gas(L, g, true);
    if (rc) return rc;
    if (!q) return fail(CRK_EINVAL, "viscosity parameters are required");
    if (!(q->Cl >= 0.0) || !(q->Cq >= 0.0) || !(q->eps_q > 0.0))
        return fail(CRK_EINVAL, "viscosity needs Cl >= 0, Cq >= 0 and eps_q > 0");
    if (!(gamma > 1.0)) return fail(CRK_EINVAL, "gamma must exceed 1 (the sound speed)");
    if (L->n == 0) {
        if (totals) {
            hipLaunchKernelGGL(k_zero8, dim3(1), dim3(64), 0, st, totals);
            LAUNCH_CHECK("zero totals");
        }
        return CRK_OK;
    }
    if (!V || !rho || !C || !C->A || !C->B || !C->dA || !C->dB || !dv || !a || !dudt)
        return fail(CRK_EINVAL, "V, rho, corrections, dv, a and dudt are required");
    if (prec == CRK_F32)
        return accel_visc_impl<float>(L, g, (const float*)V, (const float*)rho, C, (const float*)dv, q, gamma,
                                      (float*)a, (float*)dudt, totals, st);
    if (prec == CRK_F64)
        return accel_visc_impl<double>(L, g, (const double*)V, (const double*)rho, C, (const double*)dv, q, gamma,
                                       (double*)a, (double*)dudt, totals, st);
    return fail(CRK_EINVAL, "unknown precision");
}

int crk_accel_energy_compatible(crk_leaves* L, const crk_gas* g, const void* V, const void* rho,
                                const crk_corr* C, const void* dv, const crk_visc* q, double eps_u, double gamma,
                                crk_prec prec, void* a, void* dudt, double* totals, hipStream_t st) {
    int rc = check_gas(L, g, true);
    if (rc) return rc;
    if ((dv == nullptr) != (q == nullptr))
        return fail(CRK_EINVAL, "dv and the viscosity parameters go together (both NULL: no viscosity)");
    if (q && (!(q->Cl >= 0.0) || !(q->Cq >= 0.0) || !(q->eps_q > 0.0)))
        return fail(CRK_EINVAL, "viscosity needs Cl >= 0, Cq >= 0 and eps_q > 0");
    if (!(eps_u >= 0.0) || !std::isfinite(eps_u)) return fail(CRK_EINVAL, "eps_u must be finite and >= 0");
    if (q && !(gamma > 1.0)) return fail(CRK_EINVAL, "gamma must exceed 1 (the sound speed)");
    if (L->n == 0) {
        if (totals) {
            hipLaunchKernelGGL(k_zero8, dim3(1), dim3(64), 0, st, totals);
            LAUNCH_CHECK("zero totals");
        }
        return CRK_OK;
    }
    if (!V || !rho || !C || !C->A || !C->B || !C->dA || !C->dB || !a || !dudt)
        return fail(CRK_EINVAL, "V, rho, corrections, a and dudt are required");
    if (prec == CRK_F32) {
        if (q)
            return accel_visc_impl<float>(L, g, (const float*)V, (const float*)rho, C, (const float*)dv, q, gamma,
                                          (float*)a, (float*)dudt, totals, st, eps_u);
        return accel_impl<float>(L, g, (const float*)V, (const float*)rho, C, gamma, (float*)a, (float*)dudt,
                                 totals, st, eps_u);
    }
    if (prec == CRK_F64) {
        if (q)
            return accel_visc_impl<double>(L, g, (const double*)V, (const double*)rho, C, (const double*)dv, q,
                                           gamma, (double*)a, (double*)dudt, totals, st, eps_u);
        return accel_impl<double>(L, g, (const double*)V, (const double*)rho, C, gamma, (double*)a,
                                  (double*)dudt, totals, st, eps_u);
    }
    return fail(CRK_EINVAL, "unknown precision");
}

int crk_accel_energy_noalloc(crk_leaves* L, const crk_gas* g, const void* V, const void* rho,
                             const crk_corr* C, double gamma, crk_prec prec, void* a, void* dudt,
                             double* totals, hipStream_t st) {
    return accel_entry(true, L, g, V, rho, C, gamma, prec, a, dudt, totals, st);
}

}  // extern "C"
