"""The allocation-free query entry point (lq_query_radiance_noalloc),
called through the C ABI, against lq_query_radiance: bit-identical results
on two calls in a row, the second with fewer rays (the shared counter
array keeps the first call's contents and must be cleared by the second)."""
import ctypes as C
import sys

import numpy as np
import pytest

import inputs

pytestmark = pytest.mark.gpu


def _say(msg):
    print(f"[gpu] {msg}", flush=True)
    sys.stdout.flush()


def _dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def test_noalloc_query_matches_query(c0_tree):
    import torch
    import paper_2207_05009_amd as lq
    L = lq.lib()
    L.lq_query_radiance_noalloc.argtypes = L.lq_query_radiance.argtypes
    L.lq_query_radiance_noalloc.restype = C.c_int
    oct_ = lq.Octree(c0_tree, "f32")
    stream = C.c_void_p(torch.cuda.current_stream().cuda_stream)
    calls = [(65536, 1, 0, lq.LQ_LINEAR), (1000, 2, 0, lq.LQ_LINEAR), (4099, 3, lq.LQ_NO_EARLY_TERM, lq.LQ_EXP)]
    for n, seed, flags, model in calls:
        _say(f"no-alloc query: {n} rays, seed {seed}, flags {flags}, model {model}")
        o, d = inputs.rays.sphere_to_cube(n, seed)
        O, D = _dev(o), _dev(d)
        out = {}
        for name in ("lq_query_radiance", "lq_query_radiance_noalloc"):
            rgb = torch.full((n, 3), float("nan"), device="cuda")
            alpha = torch.full((n,), float("nan"), device="cuda")
            st = getattr(L, name)(oct_.handle, C.c_void_p(O.data_ptr()), C.c_void_p(D.data_ptr()), n,
                                  C.c_void_p(rgb.data_ptr()), C.c_void_p(alpha.data_ptr()), model, flags,
                                  stream)
            assert st == 0, L.lq_last_error()
            torch.cuda.synchronize()
            out[name] = (rgb, alpha)
        ref, got = out["lq_query_radiance"], out["lq_query_radiance_noalloc"]
        assert not bool(torch.isnan(got[0]).any()) and not bool(torch.isnan(got[1]).any())
        assert torch.equal(got[0], ref[0]) and torch.equal(got[1], ref[1])
    # argument errors as in lq_query_radiance; n = 0 is a no-op
    assert L.lq_query_radiance_noalloc(oct_.handle, None, None, 0, None, None, 0, 0, None) == 0
    assert L.lq_query_radiance_noalloc(None, None, None, 4, None, None, 0, 0, None) == -1
    oct_.free()
