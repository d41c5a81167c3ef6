// Host-side recursive coordinate bisection and tile interaction lists.
#pragma once

#include <cstdint>
#include <vector>

namespace crk {

constexpr int kTile = 64;  // particles per tile = lanes per wavefront
// Radius factor of the box tests that gather a tile's candidates: wide enough
// that every pair the list build accepts (squared radius factor 1 + 1e-5, FP32
// rounding of r^2 and of the radii) lies within it, so that a particle's list
// does not depend on how the particles are cut into leaves and tiles.
constexpr double kTreeMargin = 1.0 + 2.0e-5;

struct TreeInput {
    int64_t n;
    const uint32_t* q[3];   // fixed-point positions (2^-32 box units)
    const double* H;        // support radius per particle (box units), or nullptr
    double r_fixed;         // interaction radius when H == nullptr
    int leaf_max;
    int leaf_min;
    double split_extent;    // box units; <= 0 disables the extent rule
    // optional per-particle work (input index): inside every leaf, particles
    // are ordered by decreasing work (stable), so that each tile of 64 groups
    // lanes of similar list length
    const int32_t* weight = nullptr;
};

struct TreeOutput {
    std::vector<int32_t> perm;         // tree order -> input index
    std::vector<int32_t> leaf_begin;   // leaves as ranges of tree order
    std::vector<int32_t> leaf_end;
    std::vector<int32_t> rng_off;      // per tile: CSR offsets into rng (n_tiles + 1)
    std::vector<int32_t> rng;          // (begin, end) pairs of candidate particle ranges
    std::vector<int64_t> tile_cand;    // candidate particles per tile
    int64_t cand_pairs = 0;            // sum over tiles of (valid lanes * candidates)
};

// Builds the tree and the per-tile candidate ranges.  Returns false with a
// message on invalid input.
bool build_tree(const TreeInput& in, TreeOutput& out, const char** err);

}  // namespace crk
