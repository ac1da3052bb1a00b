// octree_query.hip -- launch of the emission query on gfx950.
//
// One work-item per ray; the per-ray march (traversal with exact decisions,
// float32 compositing) is march_ray() in march.h.
#include "march.h"

namespace lq {
namespace {

template <int ST, int DEG, bool ACC64, bool TRACE>
__global__ __launch_bounds__(256) void k_query(const DevTree t, const QueryArgs a) {
    __shared__ int32_t s_path[10 * 256];   // per-lane node path, [level][lane]
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= a.n) return;
    RayOut r;
    uint32_t *ids = TRACE && a.max_ids > 0 ? a.leaf_ids + (size_t)i * a.max_ids : nullptr;
    march_ray<ST, DEG, ACC64, TRACE>(t, a.o + 3 * i, a.d + 3 * i, a.model, a.flags, r, ids,
                                     TRACE ? a.max_ids : 0, s_path + threadIdx.x, 256);
    if (a.rgb) {
        a.rgb[3 * i] = r.rgb[0];
        a.rgb[3 * i + 1] = r.rgb[1];
        a.rgb[3 * i + 2] = r.rgb[2];
    }
    if (a.alpha) a.alpha[i] = r.alpha;
    if (TRACE) {
        a.count[i] = r.count;
        a.hash[i] = r.hash;
        a.term_idx[i] = r.term_idx;
        a.n_comp[i] = r.n_comp;
        if (a.n_steps) a.n_steps[i] = r.n_steps;
    }
}

template <int ST, int DEG>
hipError_t launch_deg(const DevTree &t, const QueryArgs &a, bool trace, hipStream_t s) {
    const int block = 256;
    const int64_t grid = (a.n + block - 1) / block;
    const bool acc64 = (a.flags & LQ_FP64_ACCUM) != 0;
    if (trace && acc64) hipLaunchKernelGGL((k_query<ST, DEG, true, true>), dim3(grid), dim3(block), 0, s, t, a);
    else if (trace) hipLaunchKernelGGL((k_query<ST, DEG, false, true>), dim3(grid), dim3(block), 0, s, t, a);
    else if (acc64) hipLaunchKernelGGL((k_query<ST, DEG, true, false>), dim3(grid), dim3(block), 0, s, t, a);
    else hipLaunchKernelGGL((k_query<ST, DEG, false, false>), dim3(grid), dim3(block), 0, s, t, a);
    return hipGetLastError();
}

template <int ST>
hipError_t launch_st(const DevTree &t, const QueryArgs &a, bool trace, hipStream_t s) {
    switch (t.sh_degree) {
        case 0: return launch_deg<ST, 0>(t, a, trace, s);
        case 1: return launch_deg<ST, 1>(t, a, trace, s);
        case 2: return launch_deg<ST, 2>(t, a, trace, s);
        case 3: return launch_deg<ST, 3>(t, a, trace, s);
        case 4: return launch_deg<ST, 4>(t, a, trace, s);
    }
    return hipErrorInvalidValue;
}

}  // namespace

int row_bytes(int storage, int K) { return row_bytes_for(storage == LQ_F32 ? 4 : 2, K); }

hipError_t launch_query(const DevTree &t, const QueryArgs &a, bool trace, hipStream_t s) {
    if (a.n == 0) return hipSuccess;
    switch (t.storage) {
        case LQ_F32: return launch_st<LQ_F32>(t, a, trace, s);
        case LQ_F16: return launch_st<LQ_F16>(t, a, trace, s);
        case LQ_BF16: return launch_st<LQ_BF16>(t, a, trace, s);
    }
    return hipErrorInvalidValue;
}

}  // namespace lq
