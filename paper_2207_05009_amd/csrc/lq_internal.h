// Internal declarations shared by the library's HIP sources (not installed).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>

#include "../../include/lumiq.h"

namespace lq {

// Device image of a plenoctree.
//  child: [n_nodes][8] int32 (the descriptor's table, unchanged).
//  child_skip: the same tree with every data leaf whose stored density is
//         below sigma_min removed, and every node left without children
//         removed in turn (leaf indices unchanged).  The plain query marches
//         it: those leaves are never composited (Sec. 6.2, sigma_min), so it
//         visits the composited leaves with the same segments in fewer steps.
//  rows:  [n_leaves][row_elems] in the storage type: sigma, then the SH
//         coefficients of R, G, B (K each), zero padded so that a row is a
//         power-of-two number of bytes >= 64 (one row never straddles a
//         128-byte line when it is <= 128 bytes).
// Level of the dense top grid: for each cell of level kTopLevel the grid
// holds the node covering it (> 0) or, where the tree ends above that level
// in an empty node, minus the level of that node's cell.  One read replaces
// the first kTopLevel steps of a descent.  Trees of depth <= kTopLevel have
// no grid.
constexpr int kTopLevel = 4;
constexpr int kTopCells = 1 << (3 * kTopLevel);

struct DevTree {
    const int32_t *child;
    const int32_t *child_skip;
    const int32_t *top;        // [kTopCells] grid of `child`, or null
    const int32_t *top_skip;   // [kTopCells] grid of `child_skip`, or null
    const void *rows;
    int32_t depth, sh_degree, K, storage;
    int32_t n_nodes, n_leaves, row_elems, pad;
    float l_max, sigma_min, alpha_max, pad2;
};

// Ray counters of one query launch (two contiguous ranges of the batch per
// accelerator die, see octree_kernels.h).
constexpr int kQueryCounters = 16;

struct QueryArgs {
    const float *o, *d;
    int64_t n;
    float *rgb, *alpha;
    int model;
    uint32_t flags;
    // trace outputs (nullptr when not tracing)
    uint32_t *count;
    uint64_t *hash;
    int32_t *term_idx;
    uint32_t *n_comp;
    uint32_t *n_steps;
    uint32_t *leaf_ids;
    int32_t max_ids;
    // ray i of the launch is index[i] of the arrays (null: i itself), and
    // the launch covers *n_dev rays when n_dev is set (n is then a bound)
    const int64_t *index;
    const unsigned long long *n_dev;
    // camera batch: when img_w > 0 the n = img_w * img_h rays are the pixels
    // of a row-major image and the waves take them up in 8 x 8 pixel tiles
    // (tile_order_pixel); excludes index
    uint32_t img_w, img_h;
    // kQueryCounters device counters for the launch, or null: the launcher
    // then allocates them stream-ordered
    unsigned long long *counters;
};

// Pixel taken up at position v (< w h) of a camera batch's tile order, a
// bijection of [0, w h): whole 8 x 8 tiles first, tile by tile along each
// band of 8 rows (a tile row-major inside), then the pixels right of the
// last whole tile of each band, then the rows below the last whole band,
// both row-major.  A wave's 64 lanes thus take one tile: neighbouring
// pixels, whose rays cross mostly the same octree nodes.  w h < 2^32.
__host__ __device__ inline uint32_t tile_order_pixel(uint32_t v, uint32_t w, uint32_t h) {
    const uint32_t w8 = w & ~7u, h8 = h & ~7u;   // columns and rows of whole tiles
    const uint32_t n_tiled = h8 * w8;
    if (v < n_tiled) {                           // then w8 >= 8
        const uint32_t band = v / (8u * w8), j = v - band * (8u * w8);
        const uint32_t p = j & 63u;
        return (band * 8u + (p >> 3)) * w + (j >> 6) * 8u + (p & 7u);
    }
    v -= n_tiled;
    const uint32_t ws = w - w8, n_side = h8 * ws;
    if (v < n_side) {                            // then ws >= 1
        const uint32_t r = v / ws;
        return r * w + w8 + (v - r * ws);
    }
    return h8 * w + (v - n_side);
}

// launch the emission query; returns hipSuccess or the launch error
hipError_t launch_query(const DevTree &t, const QueryArgs &a, bool trace, hipStream_t s);
// several trees of one storage type and SH degree (2 or 3) in one launch;
// trees/offsets are device arrays
hipError_t launch_query_multi(int storage, int sh_degree, const DevTree *trees, const int64_t *offsets,
                              int n_trees, const QueryArgs &a, hipStream_t s);

// FP32 -> storage conversions used by the loader (round to nearest even)
uint16_t f32_to_f16_rne(float x);
uint16_t f32_to_bf16_rne(float x);

void set_error(const std::string &msg);

// a device array on `device` holding `bytes` from ptr on (else an error
// status, with the message set)
lq_status check_device_array(const void *ptr, size_t bytes, int device, const char *name);
// device of a tree
int octree_device(const lq_octree *t);

// emission query (default flags) over rays in the library's own device
// scratch (no pointer checks: the caller made the arrays): the rays listed
// in index[0 .. *n_dev) of o/d, writing rgb and alpha at those rays
lq_status query_scratch(const lq_octree *t, const float *o, const float *d, int64_t n_max, const int64_t *index,
                        const unsigned long long *n_dev, float *rgb, float *alpha, int model, hipStream_t s);

// emission query (linear model, default flags) of the rays listed in
// index[0 .. *n_dev) of origins/dirs, writing rgb at those rays
lq_status query_indexed(const lq_octree *tree, const float *o, const float *d, int64_t n_max,
                        const int64_t *index, const unsigned long long *n_dev, float *rgb, hipStream_t s);

}  // namespace lq
