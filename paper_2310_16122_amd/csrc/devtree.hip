// Device leaf build for MI355X (gfx950): Morton-ordered octree leaves, tile
// boxes and tile candidate ranges computed on the GPU.
//
// The paper's code evaluates short-range interactions between leaves of a
// tree built over the particles (Sec. 3.1).  crk_build_leaf_pairs builds that
// tree on the host (recursive coordinate bisection); crk_build_leaf_pairs_device
// builds an octree on the device instead, without the positions' round trip:
//   1. Morton keys of the fixed-point positions (the top 21 bits per axis),
//      sorted with their indices (radix sort): tree order;
//   2. leaves: each particle's leaf cell is the coarsest octree cell around
//      it that holds at most leaf_max particles (found by binary search of the
//      sorted keys, level by level); consecutive particles whose leaf cells
//      share a parent are cut into leaves of leaf_max, so that every leaf lies
//      inside one cell twice its leaf cell's size;
//   3. leaf and tile boxes (tiles: 64 consecutive particles of tree order) and
//      the largest support radius of each;
//   4. per tile, the leaves whose boxes come within the interaction radius of
//      the tile's box, as merged ranges of tree order: the octree cells of a
//      level fine enough that at most 3 per axis cover the tile's box widened
//      by the largest radius are looked up by key range, and the leaves inside
//      them are tested box against box (periodic gaps), in key order so that a
//      leaf met through two cells is taken once.
// The neighbour lists are then built from these ranges exactly as in the host
// path.  A leaf's particles can be reordered (by decreasing list length, for
// tiles of similar work) without changing its box.

#include <hipcub/hipcub.hpp>

#include "crk_internal.h"
#include "tree.h"

using namespace crk;

namespace {

constexpr int kLevels = 21;  // Morton bits per axis

__device__ __forceinline__ uint64_t spread3(uint32_t v) {
    uint64_t x = v & 0x1fffffu;
    x = (x | (x << 32)) & 0x1f00000000ffffull;
    x = (x | (x << 16)) & 0x1f0000ff0000ffull;
    x = (x | (x << 8)) & 0x100f00f00f00f00full;
    x = (x | (x << 4)) & 0x10c30c30c30c30c3ull;
    x = (x | (x << 2)) & 0x1249249249249249ull;
    return x;
}

__device__ __forceinline__ uint64_t morton3(uint32_t cx, uint32_t cy, uint32_t cz) {
    return (spread3(cx) << 2) | (spread3(cy) << 1) | spread3(cz);
}

__device__ __forceinline__ uint32_t quantize_d(double x) {
    const double t = x - floor(x);  // the same rounding as the host build
    const double v = floor(t * 4294967296.0 + 0.5);
    return v >= 4294967296.0 ? 0u : uint32_t(v);
}

// first position in [lo, hi) whose key is >= v
__device__ __forceinline__ int lower_key(const uint64_t* __restrict__ K, int lo, int hi, uint64_t v) {
    while (lo < hi) {
        const int mid = lo + ((hi - lo) >> 1);
        if (K[mid] < v) lo = mid + 1;
        else hi = mid;
    }
    return lo;
}

// Morton keys of the fixed-point positions; counts invalid inputs (non-finite
// positions, support radii not positive and finite) in *bad and keeps the
// largest support radius 2h (the bits of a positive double order like it)
template <class R>
__global__ void k_keys(int n, const double* __restrict__ x, const double* __restrict__ y,
                       const double* __restrict__ z, const R* __restrict__ h, uint64_t* __restrict__ keys,
                       int32_t* __restrict__ idx, uint4* __restrict__ qin, int32_t* __restrict__ bad,
                       unsigned long long* __restrict__ hmax_bits) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double p[3] = {x[i], y[i], z[i]};
    bool ok = isfinite(p[0]) && isfinite(p[1]) && isfinite(p[2]);
    uint32_t q[3] = {0u, 0u, 0u};
    if (ok)
        for (int a = 0; a < 3; ++a) q[a] = quantize_d(p[a]);
    uint32_t hw = 0u;
    if (h) {
        const double H = 2.0 * double(h[i]);
        if (H > 0.0 && isfinite(H)) {
            atomicMax(hmax_bits, static_cast<unsigned long long>(__double_as_longlong(H)));
            hw = __float_as_uint(float(H));
        } else {
            ok = false;
        }
    }
    if (!ok) atomicAdd(bad, 1);
    qin[i] = make_uint4(q[0], q[1], q[2], hw);
    keys[i] = morton3(q[0] >> (32 - kLevels), q[1] >> (32 - kLevels), q[2] >> (32 - kLevels));
    idx[i] = i;
}

// tree order: permutation, positions, FP64 support radii
template <class R>
__global__ void k_tree_order(int n, const int32_t* __restrict__ sorted_idx, const uint4* __restrict__ qin,
                             const R* __restrict__ h, int32_t* __restrict__ perm, uint4* __restrict__ quant,
                             double* __restrict__ Hd) {
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= n) return;
    const int i = sorted_idx[s];
    perm[s] = i;
    quant[s] = qin[i];
    if (Hd) Hd[s] = 2.0 * double(h[i]);
}

// Leaves: every particle's leaf cell is the coarsest octree cell around it
// holding at most leaf_max particles; its parent cell holds more.  Consecutive
// particles (in key order) whose leaf cells share the parent form a run, cut
// into leaves of leaf_max (the last one shorter): a leaf's box stays inside
// one parent cell, and leaves are not much smaller than leaf_max, which keeps
// the count-ordered tiles (k_leaf_sort) even.  A finest-level cell that still
// holds more than leaf_max particles is a run of its own.
// prange[s]: the range of key order (begin << 32 | end) of s's parent cell.
__global__ void k_leaf_parent(int n, const uint64_t* __restrict__ K, int leaf_max, uint64_t* __restrict__ prange) {
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= n) return;
    const uint64_t key = K[s];
    int lo = 0, hi = n, plo = 0, phi = n;
    int level = 0;
    while (hi - lo > leaf_max && level < kLevels) {
        plo = lo;
        phi = hi;
        ++level;
        const int shift = 3 * (kLevels - level);
        const uint64_t cell = (key >> shift) << shift;
        const uint64_t next = cell + (uint64_t(1) << shift);
        lo = lower_key(K, lo, hi, cell);
        hi = lower_key(K, lo, hi, next);
    }
    if (hi - lo > leaf_max) {  // a finest cell that still holds more
        plo = lo;
        phi = hi;
    }
    prange[s] = (uint64_t(uint32_t(plo)) << 32) | uint32_t(phi);
}

// run_start[s] = s where a run starts, else 0 (a maximum scan then gives every
// position its run's start)
__global__ void k_run_marks(int n, const uint64_t* __restrict__ prange, int32_t* __restrict__ run_start) {
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= n) return;
    run_start[s] = (s == 0 || prange[s] != prange[s - 1]) ? s : 0;
}

// flags[s] = 1 where s starts its leaf
__global__ void k_leaf_flags(int n, const int32_t* __restrict__ run_start, int leaf_max, int32_t* __restrict__ flags) {
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= n) return;
    flags[s] = (s - run_start[s]) % leaf_max == 0 ? 1 : 0;
}

struct MaxOp {
    __device__ __forceinline__ int32_t operator()(int32_t a, int32_t b) const { return a > b ? a : b; }
};

// leaf index of every position (inclusive scan minus one) and each leaf's start
__global__ void k_leaf_index(int n, const int32_t* __restrict__ flags, const int32_t* __restrict__ excl,
                             int32_t* __restrict__ leaf_of, int32_t* __restrict__ leaf_begin,
                             int32_t* __restrict__ n_leaves) {
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= n) return;
    const int id = excl[s] + flags[s] - 1;
    leaf_of[s] = id;
    if (flags[s]) leaf_begin[id] = s;
    if (s == n - 1) {
        leaf_begin[id + 1] = n;
        *n_leaves = id + 1;
    }
}

// Box (fixed point) and largest support radius of a range of tree order.
struct Box {
    uint32_t lo[3], hi[3];
    float hmax;
    int32_t pad;
};

__device__ __forceinline__ Box range_box(const uint4* __restrict__ quant, const double* __restrict__ Hd,
                                         int b, int e) {
    Box bx;
    for (int a = 0; a < 3; ++a) {
        bx.lo[a] = 0xffffffffu;
        bx.hi[a] = 0u;
    }
    double hm = 0.0;
    for (int k = b; k < e; ++k) {
        const uint4 q = quant[k];
        const uint32_t c[3] = {q.x, q.y, q.z};
        for (int a = 0; a < 3; ++a) {
            bx.lo[a] = min(bx.lo[a], c[a]);
            bx.hi[a] = max(bx.hi[a], c[a]);
        }
        if (Hd) hm = fmax(hm, Hd[k]);
    }
    bx.hmax = float(hm);
    bx.pad = 0;
    return bx;
}

__global__ void k_leaf_boxes(const int32_t* __restrict__ n_leaves, const int32_t* __restrict__ leaf_begin,
                             const uint4* __restrict__ quant, const double* __restrict__ Hd,
                             Box* __restrict__ boxes) {
    const int l = blockIdx.x * blockDim.x + threadIdx.x;
    if (l >= *n_leaves) return;
    boxes[l] = range_box(quant, Hd, leaf_begin[l], leaf_begin[l + 1]);
}

__global__ void k_tile_boxes(int n, int nt, const uint4* __restrict__ quant, const double* __restrict__ Hd,
                             Box* __restrict__ boxes) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= nt) return;
    boxes[t] = range_box(quant, Hd, t * kWave, min(n, (t + 1) * kWave));
}

// smallest periodic gap (box units) between two fixed-point intervals
__device__ __forceinline__ double gap1(uint32_t a0, uint32_t a1, uint32_t b0, uint32_t b1) {
    const int64_t P = int64_t(1) << 32;
    int64_t best = P;
    for (int64_t sh = -P; sh <= P; sh += P) {
        const int64_t lo = int64_t(b0) + sh, hi = int64_t(b1) + sh;
        const int64_t g = max(int64_t(0), max(lo - int64_t(a1), int64_t(a0) - hi));
        best = min(best, g);
    }
    return double(best) * kInvGrid;
}

// Candidate ranges of each tile (see the file comment).  FILL = false: counts
// ranges (rcnt[t]) and candidate particles (cand[t]); FILL = true: writes the
// ranges at rng[roff[t] ...].  One thread per tile.
template <bool FILL>
__global__ void k_tile_ranges(int n, int nt, const uint64_t* __restrict__ K, const int32_t* __restrict__ leaf_of,
                              const int32_t* __restrict__ leaf_begin, const Box* __restrict__ lbox,
                              const Box* __restrict__ tbox, double hmax_all, int hydro,
                              double r_fixed, double skin, int32_t* __restrict__ rcnt, int64_t* __restrict__ cand,
                              const int32_t* __restrict__ roff, int2* __restrict__ rng) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= nt) return;
    const Box tb = tbox[t];
    const double margin = kTreeMargin, slack = 4.0 * kInvGrid;
    // the largest radius any pair of this tile can have (the pair's larger support)
    const double Rq = (hydro ? fmax(double(tb.hmax), hmax_all) + skin : r_fixed) * margin + slack;
    double ext = 0.0;
    for (int a = 0; a < 3; ++a) ext = fmax(ext, double(tb.hi[a] - tb.lo[a]) * kInvGrid + 2.0 * Rq);
    // the finest level whose cells exceed half the widened extent (with a
    // little room for rounding): at most 3 cells per axis cover it
    int level = 0;
    while (level < kLevels && ldexp(1.0, -(level + 1)) >= 0.5 * ext * (1.0 + 1e-9)) ++level;
    const int64_t side = int64_t(1) << level;
    int64_t c0[3], nc[3];
    for (int a = 0; a < 3; ++a) {
        const double lo = double(tb.lo[a]) * kInvGrid - Rq, hi = double(tb.hi[a]) * kInvGrid + Rq;
        c0[a] = int64_t(floor(lo * double(side)));
        // 4 bounds the count even if rounding went the wrong way
        nc[a] = min(min(int64_t(floor(hi * double(side))) - c0[a] + 1, side), int64_t(4));
    }
    // the covering cells' Morton prefixes, in increasing order
    uint64_t cells[64];
    int ncell = 0;
    for (int64_t i = 0; i < nc[0]; ++i)
        for (int64_t j = 0; j < nc[1]; ++j)
            for (int64_t k = 0; k < nc[2]; ++k) {
                const uint32_t cx = uint32_t(((c0[0] + i) % side + side) % side);
                const uint32_t cy = uint32_t(((c0[1] + j) % side + side) % side);
                const uint32_t cz = uint32_t(((c0[2] + k) % side + side) % side);
                uint64_t p = morton3(cx, cy, cz);
                int pos = ncell++;
                while (pos > 0 && cells[pos - 1] > p) {
                    cells[pos] = cells[pos - 1];
                    --pos;
                }
                cells[pos] = p;
            }
    const int shift = 3 * (kLevels - level);
    int last = -1, nr = 0;
    int64_t nc_part = 0;
    int open_b = -1, open_e = -1;
    const int base = FILL ? roff[t] : 0;
    const int cap = FILL ? roff[t + 1] - base : 0;  // the count pass's ranges
    auto close = [&]() {
        if (open_b < 0) return;
        if (FILL && nr < cap) rng[base + nr] = make_int2(open_b, open_e);
        ++nr;
        nc_part += open_e - open_b;
        open_b = -1;
    };
    for (int c = 0; c < ncell; ++c) {
        const uint64_t k0 = level == 0 ? 0 : cells[c] << shift;
        const int p0 = level == 0 ? 0 : lower_key(K, 0, n, k0);
        const int p1 = level == 0 ? n : lower_key(K, p0, n, k0 + (uint64_t(1) << shift));
        if (p0 >= p1) continue;
        const int l0 = max(leaf_of[p0], last + 1), l1 = leaf_of[p1 - 1];
        for (int l = l0; l <= l1; ++l) {
            const Box lb = lbox[l];
            double g2 = 0.0;
            for (int a = 0; a < 3; ++a) {
                const double g = gap1(tb.lo[a], tb.hi[a], lb.lo[a], lb.hi[a]);
                g2 += g * g;
            }
            const double R = (hydro ? fmax(double(tb.hmax), double(lb.hmax)) + skin : r_fixed) * margin + slack;
            if (g2 < R * R) {
                const int b = leaf_begin[l], e = leaf_begin[l + 1];
                if (open_b >= 0 && open_e == b) {
                    open_e = e;
                } else {
                    close();
                    open_b = b;
                    open_e = e;
                }
            }
        }
        last = max(last, l1);
    }
    close();
    if (!FILL) {
        rcnt[t] = nr;
        cand[t] = nc_part;
    }
}

// Longest lists first inside every leaf (stable; a leaf's box does not change):
// one workgroup per leaf sorts (count, position) pairs in LDS by bitonic
// merges and permutes the leaf's tree-order arrays.
constexpr int kSortMax = kDevLeafMax;

__global__ __launch_bounds__(256) void k_leaf_sort(const int32_t* __restrict__ leaf_begin, int32_t* __restrict__ perm,
                                                   uint4* __restrict__ quant, double* __restrict__ Hd,
                                                   int32_t* __restrict__ cnt) {
    __shared__ uint64_t key[kSortMax];
    __shared__ uint4 q_s[kSortMax];
    __shared__ double h_s[kSortMax];
    __shared__ int32_t p_s[kSortMax], c_s[kSortMax];
    const int b = leaf_begin[blockIdx.x], e = leaf_begin[blockIdx.x + 1];
    const int m = e - b;
    if (m > kSortMax) return;  // leaves hold at most leaf_max <= kSortMax particles
    int size = 1;
    while (size < m) size <<= 1;
    for (int k = threadIdx.x; k < size; k += blockDim.x) {
        if (k < m) {
            // decreasing count, then increasing position
            key[k] = (uint64_t(0x7fffffffu - uint32_t(cnt[b + k])) << 32) | uint32_t(k);
            q_s[k] = quant[b + k];
            h_s[k] = Hd ? Hd[b + k] : 0.0;
            p_s[k] = perm[b + k];
            c_s[k] = cnt[b + k];
        } else {
            key[k] = ~uint64_t(0);
        }
    }
    __syncthreads();
    for (int len = 2; len <= size; len <<= 1)
        for (int j = len >> 1; j > 0; j >>= 1) {
            for (int k = threadIdx.x; k < size; k += blockDim.x) {
                const int o = k ^ j;
                if (o > k) {
                    const bool up = (k & len) == 0;
                    const uint64_t a = key[k], c = key[o];
                    if ((a > c) == up) {
                        key[k] = c;
                        key[o] = a;
                    }
                }
            }
            __syncthreads();
        }
    for (int k = threadIdx.x; k < m; k += blockDim.x) {
        const int from = int(uint32_t(key[k]));
        quant[b + k] = q_s[from];
        if (Hd) Hd[b + k] = h_s[from];
        perm[b + k] = p_s[from];
        cnt[b + k] = c_s[from];
    }
}

__global__ void k_tile_len(int n, int nt, const int32_t* __restrict__ cnt, int32_t* __restrict__ len,
                           int64_t* __restrict__ slots, int64_t* __restrict__ entries) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= nt) return;
    int mx = 0;
    int64_t sum = 0;
    for (int s = t * kWave; s < min(n, (t + 1) * kWave); ++s) {
        mx = max(mx, cnt[s]);
        sum += cnt[s];
    }
    len[t] = mx;
    slots[t] = int64_t(mx) * kWave;
    entries[t] = sum;
}

}  // namespace

namespace crk {

// Temporaries of the device build, laid out in the handle's per-pass scratch
// (which no pass uses while a build runs); the same (n, tile count) always
// gives the same layout, so the steps of one build share them.
struct DevTree {
    uint64_t *keys_a, *keys_b;  // Morton keys; keys_b sorted (not permuted by the leaf sort)
    int32_t *idx_a, *idx_b, *flags, *excl, *leaf_of, *leaf_begin, *n_leaves, *rcnt, *bad;
    unsigned long long* hmax_bits;
    uint4* qin;
    Box *lbox, *tbox;
    int64_t *cand, *slots, *entries;
    void* cub_tmp;
    size_t cub_bytes;
};

static size_t cub_bytes(int64_t n, int64_t nt) {
    size_t sort_b = 0, scan_b = 0, scan64_b = 0;
    (void)hipcub::DeviceRadixSort::SortPairs(nullptr, sort_b, (uint64_t*)nullptr, (uint64_t*)nullptr,
                                             (int32_t*)nullptr, (int32_t*)nullptr, int(std::max<int64_t>(n, 1)),
                                             0, 3 * kLevels);
    (void)hipcub::DeviceScan::ExclusiveSum(nullptr, scan_b, (int32_t*)nullptr, (int32_t*)nullptr,
                                           int(std::max<int64_t>(n, nt) + 1));
    (void)hipcub::DeviceScan::ExclusiveSum(nullptr, scan64_b, (int64_t*)nullptr, (int64_t*)nullptr,
                                           int(nt + 1));
    size_t max_b = 0;
    (void)hipcub::DeviceScan::InclusiveScan(nullptr, max_b, (int32_t*)nullptr, (int32_t*)nullptr, MaxOp(),
                                            int(std::max<int64_t>(n, 1)));
    return std::max(std::max(sort_b, max_b), std::max(scan_b, scan64_b));
}

static DevTree carve_devtree(char* base, int64_t n, int64_t nt, size_t* used = nullptr) {
    DevTree d;
    Carver c(base);
    d.keys_a = c.take<uint64_t>(n);
    d.keys_b = c.take<uint64_t>(n);
    d.idx_a = c.take<int32_t>(n);
    d.idx_b = c.take<int32_t>(n);
    d.flags = c.take<int32_t>(n + 1);
    d.excl = c.take<int32_t>(n + 1);
    d.leaf_of = c.take<int32_t>(n);
    d.leaf_begin = c.take<int32_t>(n + 1);
    d.n_leaves = c.take<int32_t>(1);
    d.rcnt = c.take<int32_t>(nt + 1);
    d.bad = c.take<int32_t>(1);
    d.hmax_bits = c.take<unsigned long long>(1);
    d.qin = c.take<uint4>(n);
    d.lbox = c.take<Box>(n);
    d.tbox = c.take<Box>(nt);
    d.cand = c.take<int64_t>(nt + 1);
    d.slots = c.take<int64_t>(nt + 1);
    d.entries = c.take<int64_t>(nt);
    d.cub_bytes = cub_bytes(n, nt);
    d.cub_tmp = c.take<char>(d.cub_bytes);
    if (used) *used = c.used();
    return d;
}

size_t devtree_scratch_bytes(int64_t n, int64_t nt) {
    size_t used = 0;
    carve_devtree(nullptr, n, nt, &used);
    return used;
}

static __global__ void k_clear_checks(int32_t* bad, unsigned long long* hmax_bits) {
    if (threadIdx.x == 0) {
        *bad = 0;
        *hmax_bits = 0ull;
    }
}

int devtree_leaves(crk_leaves* L, const double* x, const double* y, const double* z, const void* h,
                   int leaf_max, hipStream_t st) {
    const int n = int(L->n);
    DevTree d = carve_devtree(static_cast<char*>(L->scratch), n, L->n_tiles);
    const dim3 g((n + 255) / 256), b(256);
    hipLaunchKernelGGL(k_clear_checks, dim3(1), dim3(64), 0, st, d.bad, d.hmax_bits);
    if (L->prec == CRK_F32)
        hipLaunchKernelGGL(k_keys<float>, g, b, 0, st, n, x, y, z, static_cast<const float*>(L->hydro ? h : nullptr),
                           d.keys_a, d.idx_a, d.qin, d.bad, d.hmax_bits);
    else
        hipLaunchKernelGGL(k_keys<double>, g, b, 0, st, n, x, y, z,
                           static_cast<const double*>(L->hydro ? h : nullptr), d.keys_a, d.idx_a, d.qin, d.bad,
                           d.hmax_bits);
    LAUNCH_CHECK("morton keys");
    int32_t bad = 0;
    unsigned long long hb = 0;
    HIP_TRY(hipMemcpyAsync(&bad, d.bad, sizeof bad, hipMemcpyDeviceToHost, st));
    HIP_TRY(hipMemcpyAsync(&hb, d.hmax_bits, sizeof hb, hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    if (bad)
        return fail(CRK_EINVAL, "%d particles with a non-finite position or an h that is not positive and finite",
                    bad);
    double hmax = 0.0;
    std::memcpy(&hmax, &hb, sizeof hmax);
    L->hmax = hmax;
    if (L->hydro && !(hmax + L->skin < 0.5))
        return fail(CRK_EINVAL, "2 max(h) + skin = %g must be below half the box", hmax + L->skin);
    size_t tb = d.cub_bytes;
    HIP_TRY(hipcub::DeviceRadixSort::SortPairs(d.cub_tmp, tb, d.keys_a, d.keys_b, d.idx_a, d.idx_b, n, 0,
                                               3 * kLevels, st));
    if (L->prec == CRK_F32)
        hipLaunchKernelGGL(k_tree_order<float>, g, b, 0, st, n, d.idx_b, d.qin,
                           static_cast<const float*>(L->hydro ? h : nullptr), L->perm, L->quant,
                           L->hydro ? L->Hd : nullptr);
    else
        hipLaunchKernelGGL(k_tree_order<double>, g, b, 0, st, n, d.idx_b, d.qin,
                           static_cast<const double*>(L->hydro ? h : nullptr), L->perm, L->quant,
                           L->hydro ? L->Hd : nullptr);
    LAUNCH_CHECK("tree order");
    // keys_a and idx_a are free once the keys are sorted
    hipLaunchKernelGGL(k_leaf_parent, g, b, 0, st, n, d.keys_b, leaf_max, d.keys_a);
    LAUNCH_CHECK("leaf parents");
    hipLaunchKernelGGL(k_run_marks, g, b, 0, st, n, d.keys_a, d.idx_a);
    LAUNCH_CHECK("leaf runs");
    tb = d.cub_bytes;
    HIP_TRY(hipcub::DeviceScan::InclusiveScan(d.cub_tmp, tb, d.idx_a, d.excl, MaxOp(), n, st));
    hipLaunchKernelGGL(k_leaf_flags, g, b, 0, st, n, d.excl, leaf_max, d.flags);
    LAUNCH_CHECK("leaf starts");
    tb = d.cub_bytes;
    HIP_TRY(hipcub::DeviceScan::ExclusiveSum(d.cub_tmp, tb, d.flags, d.excl, n, st));
    hipLaunchKernelGGL(k_leaf_index, g, b, 0, st, n, d.flags, d.excl, d.leaf_of, d.leaf_begin, d.n_leaves);
    LAUNCH_CHECK("leaf index");
    int32_t nl = 0;
    HIP_TRY(hipMemcpyAsync(&nl, d.n_leaves, sizeof nl, hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    if (nl < 1 || nl > n) return fail(CRK_EHIP, "device tree: %d leaves for %d particles", nl, n);
    hipLaunchKernelGGL(k_leaf_boxes, dim3((nl + 255) / 256), b, 0, st, d.n_leaves, d.leaf_begin, L->quant,
                       L->hydro ? L->Hd : nullptr, d.lbox);
    LAUNCH_CHECK("leaf boxes");
    L->n_leaves = nl;
    return CRK_OK;
}

int devtree_ranges(crk_leaves* L, int2* rng, int64_t* total, std::vector<int64_t>* tile_cand, hipStream_t st) {
    const int n = int(L->n);
    const int nt = int(L->n_tiles);
    DevTree d = carve_devtree(static_cast<char*>(L->scratch), n, nt);
    const dim3 gt((nt + 255) / 256), b(256);
    if (!rng) {
        hipLaunchKernelGGL(k_tile_boxes, gt, b, 0, st, n, nt, L->quant, L->hydro ? L->Hd : nullptr, d.tbox);
        LAUNCH_CHECK("tile boxes");
        hipLaunchKernelGGL(k_tile_ranges<false>, gt, b, 0, st, n, nt, d.keys_b, d.leaf_of, d.leaf_begin, d.lbox,
                           d.tbox, L->hmax, L->hydro, L->r_fixed, L->skin, d.rcnt, d.cand, nullptr, nullptr);
        LAUNCH_CHECK("tile ranges (count)");
        size_t tb = d.cub_bytes;
        HIP_TRY(hipcub::DeviceScan::ExclusiveSum(d.cub_tmp, tb, d.rcnt, L->rng_off, nt + 1, st));
        int32_t tot = 0;
        tile_cand->resize(nt);
        HIP_TRY(hipMemcpyAsync(&tot, L->rng_off + nt, sizeof tot, hipMemcpyDeviceToHost, st));
        HIP_TRY(hipMemcpyAsync(tile_cand->data(), d.cand, sizeof(int64_t) * nt, hipMemcpyDeviceToHost, st));
        HIP_TRY(hipStreamSynchronize(st));
        *total = tot;
        return CRK_OK;
    }
    hipLaunchKernelGGL(k_tile_ranges<true>, gt, b, 0, st, n, nt, d.keys_b, d.leaf_of, d.leaf_begin, d.lbox, d.tbox,
                       L->hmax, L->hydro, L->r_fixed, L->skin, nullptr, nullptr, L->rng_off, rng);
    LAUNCH_CHECK("tile ranges (fill)");
    return CRK_OK;
}

int devtree_sort_leaves(crk_leaves* L, hipStream_t st) {
    DevTree d = carve_devtree(static_cast<char*>(L->scratch), L->n, L->n_tiles);
    hipLaunchKernelGGL(k_leaf_sort, dim3(unsigned(L->n_leaves)), dim3(256), 0, st, d.leaf_begin, L->perm, L->quant,
                       L->hydro ? L->Hd : nullptr, L->cnt);
    LAUNCH_CHECK("leaf sort");
    return CRK_OK;
}

int devtree_list_layout(crk_leaves* L, int64_t* slots, int64_t* entries, std::vector<int32_t>* len,
                        hipStream_t st) {
    const int n = int(L->n);
    const int nt = int(L->n_tiles);
    DevTree d = carve_devtree(static_cast<char*>(L->scratch), n, nt);
    hipLaunchKernelGGL(k_tile_len, dim3((nt + 255) / 256), dim3(256), 0, st, n, nt, L->cnt, L->ell_len, d.slots,
                       d.entries);
    LAUNCH_CHECK("tile lengths");
    size_t tb = d.cub_bytes;
    HIP_TRY(hipcub::DeviceScan::ExclusiveSum(d.cub_tmp, tb, d.slots, d.cand, nt + 1, st));
    HIP_TRY(hipMemcpyAsync(L->ell_off, d.cand, sizeof(int64_t) * nt, hipMemcpyDeviceToDevice, st));
    std::vector<int64_t> ent(nt);
    len->resize(nt);
    HIP_TRY(hipMemcpyAsync(slots, d.cand + nt, sizeof(int64_t), hipMemcpyDeviceToHost, st));
    HIP_TRY(hipMemcpyAsync(ent.data(), d.entries, sizeof(int64_t) * nt, hipMemcpyDeviceToHost, st));
    HIP_TRY(hipMemcpyAsync(len->data(), L->ell_len, sizeof(int32_t) * nt, hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    int64_t e = 0;
    for (int64_t v : ent) e += v;
    *entries = e;
    return CRK_OK;
}

}  // namespace crk
