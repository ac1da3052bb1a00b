// octree_query_f16.hip -- f16 storage instantiations of the query kernels.
#include "octree_kernels.h"

namespace lq {

hipError_t launch_query_f16(const DevTree &t, const QueryArgs &a, bool trace, hipStream_t s) {
    return launch_st<LQ_F16>(t, a, trace, s);
}

hipError_t launch_query_multi_f16(int sh_degree, const DevTree *trees, const int64_t *offsets, int n_trees,
                                   const QueryArgs &a, hipStream_t s) {
    return launch_multi_st<LQ_F16>(sh_degree, trees, offsets, n_trees, a, s);
}

}  // namespace lq
