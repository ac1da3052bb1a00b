"""Pins for the oracle's leaf sequence: three independent exact traversals
agree with each other and with the FP64 C march, on adversarial rays."""
import math

import numpy as np
import pytest

import inputs
from oracle import core, exact


def _dlen(d):
    d = [float(v) for v in d]
    return math.sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2])


def _ids(segs):
    return [s[1] for s in segs]


def _random_rays(n, seed):
    rng = np.random.default_rng(seed)
    o = rng.normal(size=(n, 3)) * 2.5
    d = rng.uniform(-1.1, 1.1, size=(n, 3)) - o
    return o.astype(np.float32), d.astype(np.float32)


@pytest.mark.parametrize("depth", [1, 2, 3])
def test_bruteforce_dda_octree_and_c_march_agree(depth):
    tree = inputs.random_tree(depth, 0.45, seed=depth)
    o1, d1 = inputs.rays.adversarial(depth, seed=depth, n=160)
    o2, d2 = _random_rays(80, 100 + depth)
    o, d = np.concatenate([o1, o2]), np.concatenate([d1, d2])
    maxid = 3 * (1 << depth) + 4
    for model in (core.LINEAR, core.EXP):
        r = core.query(tree, o, d, model=model, opts=core.NO_STOP, max_ids=maxid,
                       exact_fallback=True)
        for i in range(len(o)):
            bf = brute = exact.brute_force(tree, o[i], d[i], tree.leaf_cells)
            dda = exact.dense_dda(tree, o[i], d[i], tree.leaf_cells)
            oc, _ = exact.march_octree(tree, o[i], d[i])
            assert _ids(bf) == _ids(dda) == _ids(oc), i
            assert [s[2:] for s in brute] == [s[2:] for s in oc]
            n = r["count"][i]
            assert n == len(oc)
            assert list(r["leaf_ids"][i, :n]) == _ids(oc)
            assert int(r["hash"][i]) == exact.fnv(_ids(oc))
            dl = _dlen(d[i])
            if dl > 0 and math.isfinite(dl):
                Y = core.sh_eval(tree.sh_degree, -d[i].astype(np.float64) / dl)
                c = exact.composite(tree, oc, d[i], Y, model, no_stop=True)
                # the C march's leaf lengths come from FP64 crossing parameters
                # (error ~1e-16 |t|), i.e. ~1e-9 relative on a leaf cut near
                # its corner; the exact march's come from exact differences
                np.testing.assert_allclose(r["L"][i], c["L"], rtol=1e-8, atol=1e-300)
                assert r["alpha"][i] == pytest.approx(c["alpha"], rel=1e-8, abs=1e-300)


@pytest.mark.parametrize("depth", [4, 5])
def test_dense_dda_matches_c_march_deeper(depth):
    tree = inputs.random_tree(depth, 0.3, seed=10 + depth)
    o, d = inputs.rays.adversarial(depth, seed=20 + depth, n=96)
    r = core.query(tree, o, d, opts=core.NO_STOP, max_ids=3 * (1 << depth) + 4)
    for i in range(len(o)):
        dda = exact.dense_dda(tree, o[i], d[i], tree.leaf_cells)
        n = r["count"][i]
        assert list(r["leaf_ids"][i, :n]) == _ids(dda), i


def test_c_march_matches_exact_march_on_small_config(c0_tree):
    o, d = inputs.rays.sphere_to_cube(200, 21)
    r = core.query(c0_tree, o, d, model=core.EXP, max_ids=256, exact_fallback=False)
    assert r["n_exact"] == 0
    for i in range(len(o)):
        oc, visited = exact.march_octree(c0_tree, o[i], d[i])
        Y = core.sh_eval(2, -d[i].astype(np.float64) / _dlen(d[i]))
        c = exact.composite(c0_tree, oc, d[i], Y, core.EXP)
        n = r["count"][i]
        assert list(r["leaf_ids"][i, :n]) == c["ids"]
        assert r["term_idx"][i] == c["term_idx"]
        assert r["n_nodes"][i] == visited or r["term_idx"][i] >= 0
        np.testing.assert_allclose(r["L"][i], c["L"], rtol=1e-8, atol=1e-300)


def test_exact_fallback_is_used_for_degenerate_rays():
    # rays through grid vertices tie exactly: the FP64 march must defer them
    tree = inputs.random_tree(3, 0.5, seed=3)
    o, d = inputs.rays.adversarial(3, seed=5, n=200)
    r = core.query(tree, o, d, max_ids=32)
    assert r["n_exact"] > 0
    for i in range(len(o)):
        oc, _ = exact.march_octree(tree, o[i], d[i])
        n = r["count"][i]
        full = exact.brute_force(tree, o[i], d[i], tree.leaf_cells)
        assert list(r["leaf_ids"][i, :n]) == _ids(full)[:n]


def test_leaf_split_leaves_radiance_unchanged():
    # splitting every data leaf into 8 identical children (depth D -> D+1)
    base = inputs.random_tree(3, 0.5, seed=33)
    cells = np.asarray(base.leaf_cells)
    kids, sig, sh = [], [], []
    for j in range(8):
        off = np.array([j & 1, (j >> 1) & 1, (j >> 2) & 1])
        kids.append(2 * cells + off)
        sig.append(base.sigma)
        sh.append(base.sh)
    split = inputs.tree_from_cells(4, np.concatenate(kids), np.concatenate(sig),
                                   np.concatenate(sh))
    o, d = _random_rays(300, 34)
    for model in (core.LINEAR, core.EXP):
        a = core.query(base, o, d, model=model, opts=core.NO_STOP)
        b = core.query(split, o, d, model=model, opts=core.NO_STOP)
        np.testing.assert_allclose(a["L"], b["L"], rtol=1e-11, atol=1e-12)
        np.testing.assert_allclose(a["alpha"], b["alpha"], rtol=1e-11, atol=1e-13)


def test_power_of_two_direction_scaling_is_bit_identical(c0_tree):
    o, d = inputs.rays.sphere_to_cube(2000, 35)
    ref = core.query(c0_tree, o, d, max_ids=64)
    for k in (-40, -3, 7, 50):
        r = core.query(c0_tree, o, (d * np.float32(2.0 ** k)).astype(np.float32), max_ids=64)
        for key in ("L", "alpha", "count", "hash", "term_idx", "leaf_ids"):
            assert np.array_equal(r[key], ref[key]), (k, key)


def test_sliding_origin_along_ray(c0_tree):
    # dyadic rays so that o - 4 d is exact in float32
    rng = np.random.default_rng(36)
    n = 500
    d = (rng.integers(-512, 513, size=(n, 3)) / 512.0).astype(np.float32)
    d[np.all(d == 0, axis=1)] = np.float32([1, 0, 0])
    tgt = (rng.integers(-900, 900, size=(n, 3)) / 1024.0)
    o = (tgt - 3.0 * d).astype(np.float32)
    o2 = (o - 4.0 * d).astype(np.float32)
    assert np.array_equal(o2.astype(np.float64), o.astype(np.float64) - 4.0 * d.astype(np.float64))
    # both origins must lie outside the proxy
    out = (np.abs(o).max(1) > 1) & (np.abs(o2).max(1) > 1)
    a = core.query(c0_tree, o[out], d[out])
    b = core.query(c0_tree, o2[out], d[out])
    assert np.array_equal(a["hash"], b["hash"])
    np.testing.assert_allclose(a["L"], b["L"], rtol=1e-11, atol=1e-12)


def test_exact_path_records_match_fp64_path(c0_tree):
    o, d = inputs.rays.sphere_to_cube(400, 37)
    for model in (core.LINEAR, core.EXP):
        a = core.query(c0_tree, o, d, model=model, max_ids=160)
        b = core.query(c0_tree, o, d, model=model, max_ids=160, force_exact=True)
        assert a["n_exact"] == 0
        for key in ("count", "hash", "term_idx", "n_comp", "n_nodes", "leaf_ids"):
            assert np.array_equal(a[key], b[key]), key
        np.testing.assert_allclose(a["L"], b["L"], rtol=1e-8, atol=1e-300)


@pytest.mark.parametrize("storage", ["f32", "f16", "bf16"])
def test_pruned_tree_structure_and_march(c0_tree, storage):
    """The pruned tree (the table the production query marches) holds
    exactly the leaves whose stored density is >= sigma_min, every internal
    node has a child, and marching it with the skip off composites the same
    leaves over the same segments as marching the whole tree with the skip
    on (Sec. 6.2): identical FP64 radiance, alpha, stop, and the leaf count
    of the pruned march equals the composited count of the full one."""
    for tree in (c0_tree, inputs.random_tree(4, 0.5, seed=7, sigma_range=(0.02, 50.0))):
        p = core.pruned_tree(tree, storage)
        kept = core.dequantize(tree.sigma, storage) >= float(np.float32(0.1))
        leaves = -p.child[p.child < 0] - 1
        assert np.array_equal(np.sort(leaves), np.nonzero(kept)[0])
        assert np.all((p.child != 0).any(1)) or p.n_nodes == 1
        # every node below the root is referenced exactly once
        refs = p.child[p.child > 0]
        assert np.array_equal(np.sort(refs), np.arange(1, p.n_nodes))
        assert p.n_nodes <= tree.n_nodes
        o, d = inputs.rays.sphere_to_cube(3000, 17)
        for model in (core.LINEAR, core.EXP):
            a = core.query(tree, o, d, model=model, storage=storage)
            b = core.query(p, o, d, model=model, opts=core.NO_SKIP, storage=storage)
            assert np.array_equal(a["L"], b["L"]) and np.array_equal(a["alpha"], b["alpha"])
            assert np.array_equal(a["n_comp"], b["count"]) and np.array_equal(b["count"], b["n_comp"])
            stopped = a["term_idx"] >= 0
            assert np.array_equal(stopped, b["term_idx"] >= 0)
            assert np.all(b["term_idx"][stopped] == b["count"][stopped] - 1)
            assert np.all(b["n_nodes"] <= a["n_nodes"])
