"""The C ABI without a GPU: the library loads, exports every declared entry
point, and rejects malformed input before touching a device."""
import ctypes as C
import os
import re

import numpy as np
import pytest

import inputs

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "lumiq.h")


@pytest.fixture(scope="module")
def L():
    from paper_2207_05009_amd import lumiq
    if not os.path.exists(lumiq.LIB_PATH):
        from paper_2207_05009_amd import build
        build.build()
    return lumiq.lib()


def _declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(lq_[a-z0-9_]+)\s*\(", text)))


def test_exports_every_declared_symbol(L):
    names = _declared()
    assert "lq_query_radiance" in names and "lq_load_octree" in names
    for n in names:
        assert hasattr(L, n), n
    assert L.lq_version().startswith(b"lumiq")


def _desc(tree):
    from paper_2207_05009_amd.lumiq import OctreeDesc
    child = np.ascontiguousarray(tree.child, np.int32)
    sig = np.ascontiguousarray(tree.sigma, np.float32)
    sh = np.ascontiguousarray(tree.sh, np.float32)
    keep = (child, sig, sh)
    d = OctreeDesc(tree.depth, tree.sh_degree, child.shape[0], sig.shape[0], tree.l_max,
                   tree.sigma_min, tree.alpha_max, child.ctypes.data,
                   sig.ctypes.data if sig.size else None, sh.ctypes.data if sh.size else None)
    return d, keep


def _load(L, desc):
    h = C.c_void_p()
    st = L.lq_load_octree_desc(C.byref(desc), 0, 0, C.byref(h))
    return st, h


def test_descriptor_validation(L):
    tree = inputs.random_tree(3, 0.3, seed=1)
    d, keep = _desc(tree)
    assert L.lq_load_octree_desc(None, 0, 0, C.byref(C.c_void_p())) == -1
    h = C.c_void_p()
    assert L.lq_load_octree_desc(C.byref(d), 9, 0, C.byref(h)) == -1      # storage
    bad = _desc(tree)[0]
    bad.max_depth = 0
    assert _load(L, bad)[0] == -2
    bad = _desc(tree)[0]
    bad.sh_degree = 5
    assert _load(L, bad)[0] == -2
    # corrupt child tables
    for mutate in ("oob_node", "oob_leaf", "leaf_too_high", "repeat", "unreachable"):
        t2 = inputs.random_tree(3, 0.3, seed=1)
        ch = t2.child.copy()
        internal = np.nonzero(ch > 0)
        leaves = np.nonzero(ch < 0)
        if mutate == "oob_node":
            ch[internal[0][0], internal[1][0]] = ch.shape[0] + 5
        elif mutate == "oob_leaf":
            ch[leaves[0][0], leaves[1][0]] = -(t2.n_leaves + 3)
        elif mutate == "leaf_too_high":
            ch[0, np.nonzero(ch[0] > 0)[0][0]] = -1
        elif mutate == "repeat":
            r, c = internal[0][1], internal[1][1]
            ch[r, c] = ch[internal[0][0], internal[1][0]]
        elif mutate == "unreachable":
            ch[0, np.nonzero(ch[0] > 0)[0][0]] = 0
        t2.child = ch
        dd, k2 = _desc(t2)
        st, _ = _load(L, dd)
        assert st == -2, mutate
        assert L.lq_last_error()


def test_file_loader_errors(L, tmp_path):
    h = C.c_void_p()
    assert L.lq_load_octree(str(tmp_path / "missing").encode(), 0, 0, C.byref(h)) == -7
    p = tmp_path / "bad.lqot"
    p.write_bytes(b"NOPE" + bytes(60))
    assert L.lq_load_octree(str(p).encode(), 0, 0, C.byref(h)) == -2
    tree = inputs.random_tree(2, 0.5, seed=2)
    good = tmp_path / "t.lqot"
    inputs.treefile.save(tree, str(good))
    raw = good.read_bytes()
    (tmp_path / "trunc.lqot").write_bytes(raw[:-7])
    assert L.lq_load_octree(str(tmp_path / "trunc.lqot").encode(), 0, 0, C.byref(h)) == -2


def test_no_device_is_reported(L):
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    tree = inputs.random_tree(2, 0.5, seed=3)
    d, keep = _desc(tree)
    st, h = _load(L, d)
    assert st == -4 and b"device" in L.lq_last_error()


def test_query_argument_errors(L):
    assert L.lq_query_radiance(None, None, None, 4, None, None, 0, 0, None) == -1
    assert b"tree" in L.lq_last_error()


def test_image_query_argument_errors(L):
    assert L.lq_query_radiance_image(None, None, None, -1, 4, None, None, 0, 0, None) == -1
    assert b"width" in L.lq_last_error()
    assert L.lq_query_radiance_image(None, None, None, 65536, 32768, None, None, 0, 0, None) == -1
    assert b"2^31" in L.lq_last_error()
    assert L.lq_query_radiance_image(None, None, None, 4, 4, None, None, 0, 0, None) == -1
    assert b"tree" in L.lq_last_error()


def test_proxy_irradiance_argument_errors(L):
    assert L.lq_proxy_irradiance(None, None, None, 4, None, 8, None, 0, None, None, None) == -1
    assert b"tree" in L.lq_last_error()


def test_distillation_rejects_bad_fields(L):
    """lq_distill_leaves checks its field before touching a device."""
    from paper_2207_05009_amd import lumiq
    from inputs.trees import field_params
    p = field_params(inputs.TreeSpec(depth=3, n_blobs=4, n_shells=1, sh_degree=2, seed=1, occupancy=0.3))
    n = C.c_int64()
    assert L.lq_distill_leaves(None, 3, 0.01, 16, 0, 0, 0, None, None, None, C.byref(n), None) == -1
    desc, keep = lumiq.field_desc(p)
    assert L.lq_distill_leaves(C.byref(desc), 11, 0.01, 16, 0, 0, 0, None, None, None, C.byref(n), None) == -1
    assert L.lq_distill_leaves(C.byref(desc), 3, 0.0, 16, 0, 0, 0, None, None, None, C.byref(n), None) == -1
    assert L.lq_distill_leaves(C.byref(desc), 3, 0.01, 0, 0, 0, 0, None, None, None, C.byref(n), None) == -1
    desc.n_blobs = 33
    assert L.lq_distill_leaves(C.byref(desc), 3, 0.01, 16, 0, 0, 0, None, None, None, C.byref(n), None) == -5
    desc.n_blobs = 4
    desc.sh_degree = 5
    assert L.lq_distill_leaves(C.byref(desc), 3, 0.01, 16, 0, 0, 0, None, None, None, C.byref(n), None) == -5
    bad = dict(p)
    bad["emission"] = np.asarray(p["emission"]) * 0.0
    d2, keep2 = lumiq.field_desc(bad)
    assert L.lq_distill_leaves(C.byref(d2), 3, 0.01, 16, 0, 0, 0, None, None, None, C.byref(n), None) == -1
    assert b"radiance" in L.lq_last_error()
    bad = dict(p)
    bad["radii"] = np.asarray(p["radii"]) * 0.0 + 1e-4
    d3, keep3 = lumiq.field_desc(bad)
    assert L.lq_distill_leaves(C.byref(d3), 3, 0.01, 16, 0, 0, 0, None, None, None, C.byref(n), None) == -1
    assert b"radius" in L.lq_last_error()
    h = C.c_void_p()
    assert L.lq_octree_from_leaves(11, 2, None, None, None, 0, 2048.0, 0.1, 0.9, 0, 0, C.byref(h)) == -1
    assert L.lq_octree_download(None, None, None, None) == -1
