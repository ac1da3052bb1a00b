"""GPU parity of the emission query (through the C ABI) against the oracle."""
import sys

import numpy as np
import pytest

import inputs
from oracle import core
from tests import parity

pytestmark = pytest.mark.gpu


def _say(msg):
    print(f"[gpu] {msg}", flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def lq():
    import torch
    import paper_2207_05009_amd as lq
    assert torch.cuda.is_available()
    lq.lib()
    return lq


def _dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def _run_trace(oct_, o, d, model, flags=0, max_ids=0):
    import torch
    out = oct_.trace(_dev(o), _dev(d), model=model, flags=flags, max_ids=max_ids)
    torch.cuda.synchronize()
    return parity.to_numpy(out)


@pytest.mark.parametrize("model", ["linear", "exp"])
def test_small_config_full_parity(lq, c0_tree, model):
    o, d = inputs.rays.sphere_to_cube(65536, 1)
    _say(f"small config, 65536 rays, depth 6, model={model}")
    oct_ = lq.Octree(c0_tree, "f32")
    m = 0 if model == "linear" else 1
    orc = core.query(c0_tree, o, d, model=m, max_ids=160)
    assert orc["count"].max() <= 160
    g = _run_trace(oct_, o, d, model, max_ids=160)
    rep = parity.compare(g, orc, c0_tree.l_max)
    _say(f"report {rep}")
    assert rep["ok"], rep


@pytest.mark.parametrize("depth", [1, 2, 3, 4, 5])
def test_adversarial_rays_small_trees(lq, depth):
    tree = inputs.random_tree(depth, 0.4, seed=50 + depth)
    o1, d1 = inputs.rays.adversarial(depth, seed=60 + depth, n=400)
    rng = np.random.default_rng(depth)
    o2 = (rng.normal(size=(400, 3)) * 2.5).astype(np.float32)
    d2 = (rng.uniform(-1.1, 1.1, size=(400, 3)) - o2).astype(np.float32)
    o, d = np.concatenate([o1, o2]), np.concatenate([d1, d2])
    _say(f"adversarial rays, depth {depth}, n={len(o)}")
    oct_ = lq.Octree(tree, "f32")
    mx = 3 * (1 << depth) + 4
    for model, m in (("linear", 0), ("exp", 1)):
        for flags in (0, lq.LQ_NO_EARLY_TERM):
            orc = parity.oracle_for(tree, o, d, m, flags, max_ids=mx)
            g = _run_trace(oct_, o, d, model, flags, max_ids=mx)
            rep = parity.compare(g, orc, tree.l_max)
            assert rep["ok"], (model, flags, rep)


def test_flags_and_fp64_accumulation(lq, c0_tree):
    o, d = inputs.rays.sphere_to_cube(8192, 2)
    oct_ = lq.Octree(c0_tree, "f32")
    for flags in (lq.LQ_NO_EARLY_TERM, lq.LQ_NO_SIGMA_SKIP, lq.LQ_NO_EARLY_TERM | lq.LQ_NO_SIGMA_SKIP,
                  lq.LQ_FP64_ACCUM, lq.LQ_FP64_ACCUM | lq.LQ_NO_EARLY_TERM):
        for model, m in (("linear", 0), ("exp", 1)):
            _say(f"flags={flags} model={model}")
            orc = parity.oracle_for(c0_tree, o, d, m, flags, max_ids=160)
            g = _run_trace(oct_, o, d, model, flags, max_ids=160)
            rep = parity.compare(g, orc, c0_tree.l_max)
            assert rep["ok"], (flags, model, rep)
            if flags & lq.LQ_FP64_ACCUM:
                # FP64 accumulation leaves only the float32 leaf inputs' error
                assert rep["max_rel"] < 2e-5, rep


def test_radiance_kernel_matches_trace_kernel(lq, c0_tree):
    """The plain query marches the table without sub-sigma_min leaves; it
    composites the same leaves over the same segments as the trace, so the
    outputs agree (bit-exactly except where a segment's entry is an edge or
    corner crossing, whose tie may be represented by another axis)."""
    import torch
    o, d = inputs.rays.sphere_to_cube(65536, 3)
    oct_ = lq.Octree(c0_tree, "f32")
    _say("query vs trace outputs")
    for model in ("linear", "exp"):
        rgb, alpha = oct_.query(_dev(o), _dev(d), model=model)
        t = oct_.trace(_dev(o), _dev(d), model=model)
        torch.cuda.synchronize()
        err = parity.rel_err(rgb.cpu().numpy().astype(np.float64), t["rgb"].cpu().numpy(), c0_tree.l_max)
        assert err.max() < 1e-6, err.max()
        assert float((alpha - t["alpha"]).abs().max()) < 1e-6
        same = (rgb == t["rgb"]).all(1)
        assert float(same.float().mean()) > 0.999
        # with every leaf composited both march the full table: bit-identical
        f = lq.LQ_NO_SIGMA_SKIP
        rgb, alpha = oct_.query(_dev(o), _dev(d), model=model, flags=f)
        t = oct_.trace(_dev(o), _dev(d), model=model, flags=f)
        torch.cuda.synchronize()
        assert torch.equal(rgb, t["rgb"]) and torch.equal(alpha, t["alpha"])


@pytest.mark.parametrize("storage", ["f32", "f16", "bf16"])
def test_plain_query_parity(lq, c0_tree, storage):
    """The production entry point (no records) against the oracle."""
    import torch
    o, d = inputs.rays.sphere_to_cube(65536, 8)
    oct_ = lq.Octree(c0_tree, storage)
    for model, m in (("linear", 0), ("exp", 1)):
        _say(f"plain query {storage} {model}")
        rgb, alpha = oct_.query(_dev(o), _dev(d), model=model)
        torch.cuda.synchronize()
        orc = core.query(c0_tree, o, d, model=m, storage=storage)
        g = {"rgb": rgb.cpu().numpy(), "alpha": alpha.cpu().numpy()}
        amb = orc["alt_valid"].astype(bool)
        e_main = parity.rel_err(g["rgb"].astype(np.float64), orc["L"], c0_tree.l_max).max(1)
        e_alt = parity.rel_err(g["rgb"].astype(np.float64), orc["alt_L"], c0_tree.l_max).max(1)
        err = np.where(amb, np.minimum(e_main, e_alt), e_main)
        assert err.max() < parity.RTOL, (storage, model, err.max())


@pytest.mark.parametrize("deg", [0, 1, 2, 3, 4])
def test_sh_degrees_parity(lq, deg):
    """Every SH degree the library takes (0..4), each storage, both
    transmittance models: trace records bit-exact and radiance within the
    tolerance against the oracle, and the plain query equal to the trace
    kernel's radiance."""
    import torch
    tree = inputs.random_tree(5, 0.35, seed=90 + deg, sh_degree=deg)
    o, d = inputs.rays.sphere_to_cube(20000, 91 + deg)
    for storage in ("f32", "f16", "bf16"):
        oct_ = lq.Octree(tree, storage)
        for model, m in (("linear", 0), ("exp", 1)):
            _say(f"SH degree {deg} {storage} {model}")
            g = _run_trace(oct_, o, d, model)
            orc = core.query(tree, o, d, model=m, storage=storage)
            rep = parity.compare(g, orc, tree.l_max)
            assert rep["ok"], (deg, storage, model, rep)
            rgb, _ = oct_.query(_dev(o), _dev(d), model=model)
            torch.cuda.synchronize()
            assert np.array_equal(rgb.cpu().numpy(), g["rgb"]), (deg, storage, model)
        oct_.free()


def test_threshold_ambiguous_rays_match_a_candidate(lq):
    """Hand-built rows of leaves put 1 - T within 1e-4 of alpha_max at the
    first or second stop test, above or below it (down to 1e-7 away): the
    GPU's float32 compositing may decide either way, and its records and
    radiance must equal one of the oracle's two candidates (Sec. 6.2)."""
    from tests import test_oracle_ambiguous as amb
    n_alt = 0
    for model, name in ((core.LINEAR, "linear"), (core.EXP, "exp")):
        for amb_test in (0, 1):
            for offset in (4e-5, -4e-5, 1e-6, -1e-6, 1e-7, -1e-7):
                sig, _ = amb._densities(model, amb_test, offset)
                tree = amb._tree(sig)
                orc = core.query(tree, amb.O, amb.D, model=model, max_ids=8)
                assert orc["alt_valid"][0] == 1
                oct_ = lq.Octree(tree, "f32")
                g = _run_trace(oct_, amb.O, amb.D, name, max_ids=8)
                rep = parity.compare(g, orc, tree.l_max)
                assert rep["ok"], (name, amb_test, offset, rep)
                n_alt += rep["n_alt"]
                oct_.free()
    _say(f"threshold-ambiguous rays: {n_alt} of 24 matched the second candidate")
    # two ambiguous tests in a row (the second leaf's density is below
    # sigma_min: the skip is off): stop at either, or continue through both
    outcomes = {}
    for model, name in ((core.LINEAR, "linear"), (core.EXP, "exp")):
        for offsets in ((-6e-5, 3e-5), (-8e-5, -2e-5), (2e-5, 7e-5), (-1e-7, 1e-7), (-3e-7, -1e-7)):
            sig, _ = amb._densities_two(model, *offsets)
            tree = amb._tree(sig)
            oct_ = lq.Octree(tree, "f32")
            g = _run_trace(oct_, amb.O, amb.D, name, lq.LQ_NO_SIGMA_SKIP, max_ids=8)
            c = core.candidates(tree, amb.O, amb.D, model=model, opts=core.NO_SKIP)
            assert int(c["valid"][0].sum()) == 3
            assert parity.match_candidates(g, c, tree.l_max)[0], (name, offsets, g)
            outcomes[int(g["term_idx"][0])] = outcomes.get(int(g["term_idx"][0]), 0) + 1
            oct_.free()
    _say(f"two ambiguous tests: the GPU stopped at tests {outcomes}")


@pytest.mark.parametrize("depth", [2, 3, 5])
def test_pruned_table_trace(lq, depth):
    """The trace of the sigma_min-pruned table (what the production query
    marches) against the oracle marching its own pruned tree with the skip
    off: records bit-exact on adversarial and random rays, every storage."""
    tree = inputs.random_tree(depth, 0.5, seed=30 + depth, sigma_range=(0.02, 50.0))
    o1, d1 = inputs.rays.adversarial(depth, seed=40 + depth, n=400)
    o2, d2 = inputs.rays.sphere_to_cube(3000, 45 + depth)
    o, d = np.concatenate([o1, o2]), np.concatenate([d1, d2])
    mx = 3 * (1 << depth) + 4
    for storage in ("f32", "f16", "bf16"):
        oct_ = lq.Octree(tree, storage)
        pt = core.pruned_tree(tree, storage)
        for model, m in (("linear", 0), ("exp", 1)):
            for flags in (0, lq.LQ_NO_EARLY_TERM):
                _say(f"pruned-table trace, depth {depth}, {storage} {model} flags={flags}")
                g = _run_trace(oct_, o, d, model, flags | lq.LQ_TRACE_PRUNED, max_ids=mx)
                opts = core.NO_SKIP | (core.NO_STOP if flags else 0)
                orc = core.query(pt, o, d, model=m, opts=opts, storage=storage, max_ids=mx)
                rep = parity.compare(g, orc, tree.l_max)
                assert rep["ok"], (storage, model, flags, rep)
        oct_.free()


def test_empty_tree_and_misses(lq):
    import torch
    tree = inputs.empty_tree(4)
    oct_ = lq.Octree(tree, "f32")
    o, d = inputs.rays.sphere_to_cube(4096, 4)
    _say("empty tree")
    rgb, alpha = oct_.query(_dev(o), _dev(d))
    torch.cuda.synchronize()
    assert float(rgb.abs().max()) == 0.0 and float(alpha.abs().max()) == 0.0
    # rays that miss, non-finite rays, zero directions
    full = inputs.uniform_tree(2, 3.0, np.zeros((3, 9)))
    oct2 = lq.Octree(full, "f32")
    o = np.array([[3, 3, 3], [0, 0, 5], [np.nan, 0, 0], [0, 0, 0], [-3, 0.5, 0.5]], np.float32)
    d = np.array([[1, 0, 0], [0, 0, 1], [1, 0, 0], [0, 0, 0], [1, 0, np.inf]], np.float32)
    rgb, alpha = oct2.query(_dev(o), _dev(d))
    torch.cuda.synchronize()
    assert float(rgb.abs().max()) == 0.0 and float(alpha.abs().max()) == 0.0


def test_uniform_cube_closed_form(lq):
    import math
    import torch
    sig = 0.75
    tree = inputs.uniform_tree(3, sig, np.array([[-2.0]] * 3))
    oct_ = lq.Octree(tree, "f32")
    rng = np.random.default_rng(9)
    o = rng.normal(size=(2048, 3))
    o = (3 * o / np.linalg.norm(o, axis=1, keepdims=True)).astype(np.float32)
    tgt = rng.uniform(-0.9, 0.9, size=(2048, 3))
    d = (tgt - o).astype(np.float32)
    _say("uniform cube closed form")
    rgb, alpha = oct_.query(_dev(o), _dev(d), model="exp", flags=lq.LQ_NO_EARLY_TERM)
    torch.cuda.synchronize()
    od, dd = o.astype(np.float64), d.astype(np.float64)
    with np.errstate(divide="ignore"):
        t0 = (-1 - od) / dd
        t1 = (1 - od) / dd
    tin = np.minimum(t0, t1).max(1)
    tout = np.maximum(t0, t1).min(1)
    chord = (tout - tin) * np.linalg.norm(dd, axis=1)
    phi = tree.l_max / (1 + math.exp(2.0 * 0.5 / math.sqrt(math.pi)))
    ref = phi * (1 - np.exp(-sig * chord))
    err = np.abs(rgb.cpu().numpy()[:, 0] - ref) / ref
    assert err.max() < 1e-4, err.max()


@pytest.mark.parametrize("storage", ["f16", "bf16"])
def test_reduced_precision_storage(lq, c0_tree, storage):
    o, d = inputs.rays.sphere_to_cube(16384, 5)
    oct_ = lq.Octree(c0_tree, storage)
    _say(f"storage {storage}")
    orc_q = core.query(c0_tree, o, d, model=0, storage=storage, max_ids=160)
    g = _run_trace(oct_, o, d, "linear", max_ids=160)
    rep = parity.compare(g, orc_q, c0_tree.l_max)
    assert rep["ok"], rep
    # stated (not bounded) error against the float32 tree
    orc32 = core.query(c0_tree, o, d, model=0)
    err = parity.rel_err(g["rgb"].astype(np.float64), orc32["L"], c0_tree.l_max)
    _say(f"{storage} vs fp32 tree: max {err.max():.3e} p99 {np.quantile(err, 0.99):.3e}")


def test_direction_scaling_bit_identical(lq, c0_tree):
    o, d = inputs.rays.sphere_to_cube(16384, 6)
    oct_ = lq.Octree(c0_tree, "f32")
    _say("power-of-two scaling")
    ref = _run_trace(oct_, o, d, "linear", max_ids=160)
    for k in (-30, -2, 5, 40):
        g = _run_trace(oct_, o, (d * np.float32(2.0 ** k)).astype(np.float32), "linear", max_ids=160)
        for key in ("rgb", "alpha", "count", "hash", "term_idx", "leaf_ids"):
            assert np.array_equal(g[key], ref[key]), (k, key)


@pytest.mark.parametrize("wh", [(1, 1), (7, 5), (8, 8), (13, 11), (64, 3), (3, 64), (100, 37), (517, 259)])
def test_camera_batch_order_is_bit_identical(lq, c0_tree, wh):
    """The camera-batch entry point takes rays up in 8x8 pixel tiles (then
    the columns and rows beyond the last whole tile); each ray's result is
    that of the batch-order query: every pixel written once, bit-identical,
    whatever the image's remainder modulo 8 and whatever the flags."""
    import torch
    w, h = wh
    o, d = inputs.rays.pinhole(w, h)
    _say(f"camera batch order, {w}x{h}")
    oct_ = lq.Octree(c0_tree, "f32")
    O, D = _dev(o), _dev(d)
    for model in ("linear", "exp"):
        for flags in (0, lq.LQ_NO_EARLY_TERM, lq.LQ_NO_SIGMA_SKIP, lq.LQ_FP64_ACCUM):
            ref_rgb, ref_alpha = oct_.query(O, D, model=model, flags=flags)
            rgb = torch.full((w * h, 3), float("nan"), device="cuda")
            alpha = torch.full((w * h,), float("nan"), device="cuda")
            oct_.query_image(O, D, w, h, model=model, flags=flags, rgb=rgb, alpha=alpha)
            torch.cuda.synchronize()
            assert torch.equal(rgb, ref_rgb) and torch.equal(alpha, ref_alpha), (model, flags)
    e = torch.empty((0, 3), device="cuda")
    assert oct_.query_image(e, e, 0, 5)[0].shape == (0, 3)


@pytest.mark.parametrize("storage", ["f32", "f16"])
def test_full_size_camera_batch_order(lq, c1_tree, storage):
    """The 2048x2048 camera batch through the camera-batch entry point:
    bit-identical to the batch-order query on every ray."""
    import torch
    o, d = inputs.rays.pinhole(2048, 2048)
    _say(f"full-size camera batch in tile order, {storage}")
    oct_ = lq.Octree(c1_tree, storage)
    O, D = _dev(o), _dev(d)
    ref_rgb, ref_alpha = oct_.query(O, D)
    rgb, alpha = oct_.query_image(O, D, 2048, 2048)
    torch.cuda.synchronize()
    assert torch.equal(rgb, ref_rgb) and torch.equal(alpha, ref_alpha)


def test_abi_rejects_bad_pointers(lq, c0_tree):
    import ctypes as C
    import torch
    oct_ = lq.Octree(c0_tree, "f32")
    o = torch.zeros((16, 3), device="cuda")
    d = torch.ones((16, 3), device="cuda")
    rgb = torch.zeros((16, 3), device="cuda")
    L = lq.lib()
    host = np.zeros((16, 3), np.float32)
    _say("ABI pointer checks")
    st = L.lq_query_radiance(oct_.handle, C.c_void_p(host.ctypes.data), C.c_void_p(d.data_ptr()), 16,
                             C.c_void_p(rgb.data_ptr()), None, 0, 0, None)
    assert st == -1 and b"device pointer" in L.lq_last_error()
    small = torch.zeros((4, 3), device="cuda")
    st = L.lq_query_radiance(oct_.handle, C.c_void_p(o.data_ptr()), C.c_void_p(d.data_ptr()), 1 << 22,
                             C.c_void_p(small.data_ptr()), None, 0, 0, None)
    assert st == -1
    st = L.lq_query_radiance(oct_.handle, C.c_void_p(o.data_ptr()), C.c_void_p(d.data_ptr()), 16,
                             C.c_void_p(rgb.data_ptr()), None, 7, 0, None)
    assert st == -1
    st = L.lq_query_radiance(oct_.handle, C.c_void_p(o.data_ptr()), C.c_void_p(d.data_ptr()), 16,
                             C.c_void_p(rgb.data_ptr()), None, 0, 1 << 9, None)
    assert st == -1
    assert L.lq_query_radiance(oct_.handle, None, None, 0, None, None, 0, 0, None) == 0
    # the pruned-table flag belongs to the trace, and only with the stop flag
    st = L.lq_query_radiance(oct_.handle, C.c_void_p(o.data_ptr()), C.c_void_p(d.data_ptr()), 16,
                             C.c_void_p(rgb.data_ptr()), None, 0, lq.LQ_TRACE_PRUNED, None)
    assert st == -1
    with pytest.raises(lq.LumiqError):
        oct_.trace(o, d, flags=lq.LQ_TRACE_PRUNED | lq.LQ_FP64_ACCUM)
