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
};

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

// emission query (linear model, default flags) of the rays listed in
// index[0 .. *n_dev) of origins/dirs, writing rgb at those rays
lq_status query_indexed(const lq_octree *tree, const float *o, const float *d, int64_t n_max,
                        const int64_t *index, const unsigned long long *n_dev, float *rgb, hipStream_t s);

}  // namespace lq
