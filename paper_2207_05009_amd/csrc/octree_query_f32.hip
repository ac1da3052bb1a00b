// octree_query_f32.hip -- f32 storage instantiations of the query kernels.
#include "octree_kernels.h"

namespace lq {

hipError_t launch_query_f32(const DevTree &t, const QueryArgs &a, bool trace, hipStream_t s) {
    return launch_st<LQ_F32>(t, a, trace, s);
}

hipError_t launch_query_multi_f32(int sh_degree, const DevTree *trees, const int64_t *offsets, int n_trees,
                                   const QueryArgs &a, hipStream_t s) {
    return launch_multi_st<LQ_F32>(sh_degree, trees, offsets, n_trees, a, s);
}

}  // namespace lq
