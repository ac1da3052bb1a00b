// octree_query.hip -- dispatch of the emission query by storage type (the
// kernels are in octree_kernels.h, one translation unit per storage type).
#include "march.h"

namespace lq {

hipError_t launch_query_f32(const DevTree &t, const QueryArgs &a, bool trace, hipStream_t s);
hipError_t launch_query_f16(const DevTree &t, const QueryArgs &a, bool trace, hipStream_t s);
hipError_t launch_query_bf16(const DevTree &t, const QueryArgs &a, bool trace, hipStream_t s);
hipError_t launch_query_multi_f32(int, const DevTree *, const int64_t *, int, const QueryArgs &, hipStream_t);
hipError_t launch_query_multi_f16(int, const DevTree *, const int64_t *, int, const QueryArgs &, hipStream_t);
hipError_t launch_query_multi_bf16(int, const DevTree *, const int64_t *, int, const QueryArgs &, hipStream_t);

int row_bytes(int storage, int K) { return row_bytes_for(storage == LQ_F32 ? 4 : 2, K); }

hipError_t launch_query(const DevTree &t, const QueryArgs &a, bool trace, hipStream_t s) {
    if (a.n == 0) return hipSuccess;
    switch (t.storage) {
        case LQ_F32: return launch_query_f32(t, a, trace, s);
        case LQ_F16: return launch_query_f16(t, a, trace, s);
        case LQ_BF16: return launch_query_bf16(t, a, trace, s);
    }
    return hipErrorInvalidValue;
}

hipError_t launch_query_multi(int storage, int sh_degree, const DevTree *trees, const int64_t *offsets, int n_trees,
                              const QueryArgs &a, hipStream_t s) {
    if (a.n == 0) return hipSuccess;
    switch (storage) {
        case LQ_F32: return launch_query_multi_f32(sh_degree, trees, offsets, n_trees, a, s);
        case LQ_F16: return launch_query_multi_f16(sh_degree, trees, offsets, n_trees, a, s);
        case LQ_BF16: return launch_query_multi_bf16(sh_degree, trees, offsets, n_trees, a, s);
    }
    return hipErrorInvalidValue;
}

}  // namespace lq
