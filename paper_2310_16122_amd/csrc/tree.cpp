// Host-side recursive coordinate bisection (RCB) and per-tile candidate lists.
//
// The paper's CRK-HACC evaluates short-range interactions between leaves of an
// RCB tree, which cuts the number of particle comparisons (Sec. 3.1).  Here
// the tree is built on the host from fixed-point positions: a node is split
// at the median of its longest axis until it holds at most leaf_max particles
// (optionally also until its longest side is at most split_extent, never
// below leaf_min particles).  Tree order then defines tiles of 64 consecutive
// particles -- one wavefront each on the GPU -- and every tile gets the list
// of leaves whose boxes come within the interaction radius of the tile's box,
// merged into contiguous ranges of tree order.

#include "tree.h"

#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstring>

#include <omp.h>

namespace crk {
namespace {

constexpr double kGrid = 4294967296.0;  // 2^32

struct Node {
    uint32_t lo[3], hi[3];
    double hmax;
    int32_t begin, end;
    int32_t left, right;  // -1 for a leaf
};

struct Builder {
    const TreeInput& in;
    int32_t* idx;
    std::vector<Node>& nodes;
    std::atomic<int32_t> next{0};

    Builder(const TreeInput& i, int32_t* x, std::vector<Node>& nd) : in(i), idx(x), nodes(nd) {}

    int32_t build(int32_t b, int32_t e) {
        const int32_t id = next.fetch_add(1);
        Node nd;
        for (int a = 0; a < 3; ++a) { nd.lo[a] = UINT32_MAX; nd.hi[a] = 0; }
        nd.hmax = 0.0;
        for (int32_t k = b; k < e; ++k) {
            const int32_t p = idx[k];
            for (int a = 0; a < 3; ++a) {
                nd.lo[a] = std::min(nd.lo[a], in.q[a][p]);
                nd.hi[a] = std::max(nd.hi[a], in.q[a][p]);
            }
            if (in.H) nd.hmax = std::max(nd.hmax, in.H[p]);
        }
        nd.begin = b;
        nd.end = e;
        nd.left = nd.right = -1;
        const int32_t count = e - b;
        int axis = 0;
        uint32_t ext = 0;
        for (int a = 0; a < 3; ++a) {
            const uint32_t x = nd.hi[a] - nd.lo[a];
            if (x > ext) { ext = x; axis = a; }
        }
        bool split = count > in.leaf_max;
        if (!split && in.split_extent > 0.0 && count >= 2 * in.leaf_min && count >= 2)
            split = double(ext) / kGrid > in.split_extent;
        if (split && count >= 2) {
            // Median split that keeps the current order inside each half: the
            // left half takes the keys below the median and, among keys equal
            // to it, the first ones in the current order.  Rebuilding on
            // particles already in tree order therefore reproduces that order.
            const int32_t mid = b + count / 2;
            const uint32_t* key = in.q[axis];
            std::vector<uint32_t> tmp(count);
            for (int32_t k = 0; k < count; ++k) tmp[k] = key[idx[b + k]];
            std::nth_element(tmp.begin(), tmp.begin() + (mid - b), tmp.end());
            const uint32_t med = tmp[mid - b];
            int32_t need_eq = mid - b;
            for (int32_t k = b; k < e; ++k) need_eq -= key[idx[k]] < med;
            std::vector<int32_t> right;
            right.reserve(e - mid);
            int32_t w = b;
            for (int32_t k = b; k < e; ++k) {
                const int32_t p = idx[k];
                const uint32_t v = key[p];
                if (v < med || (v == med && need_eq-- > 0)) idx[w++] = p;
                else right.push_back(p);
            }
            std::copy(right.begin(), right.end(), idx + w);
            int32_t l = -1, r = -1;
            if (count > 65536) {
#pragma omp task shared(l)
                l = build(b, mid);
#pragma omp task shared(r)
                r = build(mid, e);
#pragma omp taskwait
            } else {
                l = build(b, mid);
                r = build(mid, e);
            }
            nd.left = l;
            nd.right = r;
        }
        nodes[id] = nd;
        return id;
    }
};

// Smallest periodic gap (box units) between two integer intervals on a circle of 2^32.
inline double gap1(uint32_t a0, uint32_t a1, uint32_t b0, uint32_t b1) {
    const int64_t P = int64_t(1) << 32;
    double best = 1e300;
    for (int64_t s = -P; s <= P; s += P) {
        const int64_t lo = int64_t(b0) + s, hi = int64_t(b1) + s;
        int64_t g = std::max<int64_t>(0, std::max<int64_t>(lo - int64_t(a1), int64_t(a0) - hi));
        best = std::min(best, double(g));
    }
    return best / kGrid;
}

}  // namespace

bool build_tree(const TreeInput& in, TreeOutput& out, const char** err) {
    const int64_t n = in.n;
    if (n < 0 || n >= (int64_t(1) << 31)) { *err = "n out of range"; return false; }
    if (in.leaf_max < 1 || in.leaf_max > (1 << 20)) { *err = "leaf_max out of range [1, 2^20]"; return false; }
    out.perm.resize(n);
    for (int64_t i = 0; i < n; ++i) out.perm[i] = int32_t(i);
    out.leaf_begin.clear();
    out.leaf_end.clear();
    out.rng_off.assign(1, 0);
    out.rng.clear();
    out.tile_cand.clear();
    out.cand_pairs = 0;
    if (n == 0) return true;

    // every leaf holds at least min_leaf particles, which bounds the node count
    int64_t min_leaf = std::max(1, (in.leaf_max + 1) / 2);
    if (in.split_extent > 0.0) min_leaf = std::min<int64_t>(min_leaf, std::max(1, in.leaf_min));
    const int64_t max_nodes = 2 * (n / min_leaf + 1) + 8;
    std::vector<Node> nodes(max_nodes);
    Builder bld(in, out.perm.data(), nodes);
    int32_t root = 0;
#pragma omp parallel
#pragma omp single
    root = bld.build(0, int32_t(n));
    const int32_t n_nodes = bld.next.load();
    nodes.resize(n_nodes);

    std::vector<int32_t> leaves;
    for (int32_t k = 0; k < n_nodes; ++k)
        if (nodes[k].left < 0) leaves.push_back(k);
    std::sort(leaves.begin(), leaves.end(),
              [&](int32_t a, int32_t b) { return nodes[a].begin < nodes[b].begin; });
    for (int32_t k : leaves) {
        out.leaf_begin.push_back(nodes[k].begin);
        out.leaf_end.push_back(nodes[k].end);
    }
    if (in.weight) {
        // a leaf's box and radius do not depend on the order inside it
        int32_t* perm = out.perm.data();
        const int32_t* wt = in.weight;
#pragma omp parallel for schedule(dynamic, 64)
        for (int64_t k = 0; k < int64_t(leaves.size()); ++k)
            std::stable_sort(perm + nodes[leaves[k]].begin, perm + nodes[leaves[k]].end,
                             [wt](int32_t a, int32_t b) { return wt[a] > wt[b]; });
    }

    // tiles of kTile consecutive particles in tree order
    const int64_t n_tiles = (n + kTile - 1) / kTile;
    std::vector<std::vector<int32_t>> tile_rng(n_tiles);
    out.tile_cand.assign(n_tiles, 0);
    int64_t cand_pairs = 0;
#pragma omp parallel for schedule(dynamic, 16) reduction(+ : cand_pairs)
    for (int64_t t = 0; t < n_tiles; ++t) {
        const int64_t b = t * kTile, e = std::min<int64_t>(n, b + kTile);
        uint32_t lo[3] = {UINT32_MAX, UINT32_MAX, UINT32_MAX}, hi[3] = {0, 0, 0};
        double hmax = 0.0;
        for (int64_t k = b; k < e; ++k) {
            const int32_t p = out.perm[k];
            for (int a = 0; a < 3; ++a) {
                lo[a] = std::min(lo[a], in.q[a][p]);
                hi[a] = std::max(hi[a], in.q[a][p]);
            }
            if (in.H) hmax = std::max(hmax, in.H[p]);
        }
        std::vector<std::pair<int32_t, int32_t>> found;
        std::vector<int32_t> stack{root};
        while (!stack.empty()) {
            const Node& nd = nodes[stack.back()];
            stack.pop_back();
            double g2 = 0.0;
            for (int a = 0; a < 3; ++a) {
                const double g = gap1(lo[a], hi[a], nd.lo[a], nd.hi[a]);
                g2 += g * g;
            }
            // radius with a small margin (list builds test pairs exactly on the GPU)
            double R = in.H ? std::max(hmax, nd.hmax) : in.r_fixed;
            R = R * kTreeMargin + 4.0 / kGrid;
            if (g2 >= R * R) continue;
            if (nd.left < 0) {
                found.emplace_back(nd.begin, nd.end);
            } else {
                stack.push_back(nd.left);
                stack.push_back(nd.right);
            }
        }
        std::sort(found.begin(), found.end());
        std::vector<int32_t>& r = tile_rng[t];
        int64_t cand = 0;
        for (auto& f : found) {
            if (!r.empty() && r.back() == f.first) r.back() = f.second;
            else { r.push_back(f.first); r.push_back(f.second); }
            cand += f.second - f.first;
        }
        out.tile_cand[t] = cand;
        cand_pairs += cand * (e - b);
    }
    out.cand_pairs = cand_pairs;
    out.rng_off.resize(n_tiles + 1);
    out.rng_off[0] = 0;
    for (int64_t t = 0; t < n_tiles; ++t)
        out.rng_off[t + 1] = out.rng_off[t] + int32_t(tile_rng[t].size() / 2);
    out.rng.resize(2 * size_t(out.rng_off[n_tiles]));
    for (int64_t t = 0; t < n_tiles; ++t)
        std::memcpy(out.rng.data() + 2 * size_t(out.rng_off[t]), tile_rng[t].data(),
                    tile_rng[t].size() * sizeof(int32_t));
    return true;
}

}  // namespace crk
