// Test-only C shim over the host tree builder (compiled with g++ by the tests).
#include <cstring>
#include "tree.h"

extern "C" int tree_shim(long long n, const unsigned* qx, const unsigned* qy, const unsigned* qz,
                         const double* H, double r_fixed, int leaf_max, int leaf_min,
                         double split_extent, int* perm, int* n_leaves, int* rng_off, int* rng,
                         int rng_cap, long long* cand_pairs, const int* weight, int* leaf_begin) {
    crk::TreeInput in;
    in.weight = weight;
    in.n = n; in.q[0] = qx; in.q[1] = qy; in.q[2] = qz; in.H = H; in.r_fixed = r_fixed;
    in.leaf_max = leaf_max; in.leaf_min = leaf_min; in.split_extent = split_extent;
    crk::TreeOutput out;
    const char* err = nullptr;
    if (!crk::build_tree(in, out, &err)) return -1;
    std::memcpy(perm, out.perm.data(), n * sizeof(int));
    *n_leaves = (int)out.leaf_begin.size();
    if (leaf_begin) std::memcpy(leaf_begin, out.leaf_begin.data(), out.leaf_begin.size() * sizeof(int));
    std::memcpy(rng_off, out.rng_off.data(), out.rng_off.size() * sizeof(int));
    if ((int)out.rng.size() > rng_cap) return -2;
    std::memcpy(rng, out.rng.data(), out.rng.size() * sizeof(int));
    *cand_pairs = out.cand_pairs;
    return (int)out.rng.size();
}
