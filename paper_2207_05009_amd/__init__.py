"""MI355X (gfx950) luminaire emission query: a C-ABI HIP library
(liblumiq.so, include/lumiq.h) and its thin Python binding."""
from .lumiq import (LQ_BF16, LQ_EXP, LQ_F16, LQ_F32, LQ_FP64_ACCUM, LQ_LINEAR, Surrogate, query_multi,
                    LQ_NO_EARLY_TERM, LQ_NO_SIGMA_SKIP, LQ_TRACE_PRUNED, LumiqError, Octree, check, distill_leaves, lib,
                    octree_from_leaves, version)

__all__ = ["LQ_BF16", "LQ_EXP", "LQ_F16", "LQ_F32", "LQ_FP64_ACCUM", "LQ_LINEAR", "Surrogate", "query_multi",
           "LQ_NO_EARLY_TERM", "LQ_NO_SIGMA_SKIP", "LQ_TRACE_PRUNED", "LumiqError", "Octree", "check", "distill_leaves", "lib",
           "octree_from_leaves", "version"]
