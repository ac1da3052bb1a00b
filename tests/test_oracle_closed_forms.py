"""Closed forms and invariants that pin the oracle's compositing
(Sec. 4.1, Eqs. 3-5; Sec. 4.2, Eq. 6; Sec. 6.2 heuristics)."""
import math
from fractions import Fraction as Fr

import numpy as np
import pytest
import scipy.special as sps

import inputs
from oracle import core, exact

LMAX = inputs.L_MAX


def _chords(o, d, lo, hi):
    """Textbook slab test: parameter interval of o + t d inside the box
    [lo, hi] (exact rationals), clipped to t >= 0."""
    t0, t1 = Fr(0), None
    for a in range(3):
        oa, da = Fr(float(o[a])), Fr(float(d[a]))
        if da == 0:
            assert lo[a] <= oa < hi[a]
            continue
        u, v = (Fr(lo[a]) - oa) / da, (Fr(hi[a]) - oa) / da
        t0 = max(t0, min(u, v))
        t1 = max(u, v) if t1 is None else min(t1, max(u, v))
    return t0, t1


def _dlen(d):
    d = [float(v) for v in d]
    return math.sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2])


def _real_sh_scipy(l, m, w):
    th, ph = math.acos(max(-1.0, min(1.0, w[2]))), math.atan2(w[1], w[0])
    c = sps.sph_harm_y(l, abs(m), th, ph)
    if m == 0:
        return c.real
    return math.sqrt(2) * (-1) ** m * (c.real if m > 0 else c.imag)


def _phi(row, w):
    deg = int(round(math.sqrt(len(row)))) - 1
    x = sum(float(row[l * l + l + m]) * _real_sh_scipy(l, m, w)
            for l in range(deg + 1) for m in range(-l, l + 1))
    return LMAX / (1.0 + math.exp(-x))


def _rays_through_cube(n, seed):
    rng = np.random.default_rng(seed)
    o = rng.normal(size=(n, 3))
    o = 3.0 * o / np.linalg.norm(o, axis=1, keepdims=True)
    tgt = rng.uniform(-0.9, 0.9, size=(n, 3))
    d = tgt - o
    return o.astype(np.float32), (d / np.linalg.norm(d, axis=1, keepdims=True)).astype(np.float32)


@pytest.mark.parametrize("model", [core.LINEAR, core.EXP])
@pytest.mark.parametrize("deg", [0, 2])
def test_uniform_cube(model, deg):
    rng = np.random.default_rng(10 + deg)
    K = (deg + 1) ** 2
    sig = 0.75
    rows = rng.normal(0, 1.0, size=(3, K))
    rows[:, 0] -= 4.0
    tree = inputs.uniform_tree(2, sig, rows)
    o, d = _rays_through_cube(64, 3)
    r = core.query(tree, o, d, model=model, opts=core.NO_STOP | core.NO_SKIP)
    for i in range(len(o)):
        t0, t1 = _chords(o[i], d[i], (-1, -1, -1), (1, 1, 1))
        chord = float(t1 - t0) * _dlen(d[i])
        a = 1.0 - math.exp(-float(np.float32(sig)) * chord) if model == core.EXP else min(
            1.0, float(np.float32(sig)) * chord)
        w = -np.asarray(d[i], np.float64) / _dlen(d[i])
        for c in range(3):
            assert r["L"][i, c] == pytest.approx(_phi(tree.sh[0, c], w) * a, rel=1e-12)
        assert r["alpha"][i] == pytest.approx(a, rel=1e-12)


def test_degree0_radiance_independent_of_direction():
    # a uniform cube of SH degree 0 seen along chords of equal length
    tree = inputs.uniform_tree(3, 2.0, np.array([[-3.0]] * 3))
    o = np.array([[-3, 0.1, 0.2], [0.1, -3, 0.2], [0.2, 0.1, 3], [3, -0.1, -0.2]], np.float32)
    d = np.array([[1, 0, 0], [0, 1, 0], [0, 0, -1], [-1, 0, 0]], np.float32)
    r = core.query(tree, o, d, model=core.EXP, opts=core.NO_STOP)
    assert np.all(r["L"] == r["L"][0, 0])
    ref = LMAX / (1 + math.exp(3.0 * 0.5 / math.sqrt(math.pi))) * (1 - math.exp(-2.0 * 2.0))
    assert r["L"][0, 0] == pytest.approx(ref, rel=1e-13)


def test_emission_direction_is_minus_d():
    # emission concentrated toward +z: a ray travelling down (d = -z) sees
    # omega = +z, the bright side (Sec. 4.1: the ray is x - omega t)
    row = np.zeros(9)
    row[0], row[2] = -2.0, 4.0             # k = 2 is (l=1, m=0), proportional to z
    tree = inputs.uniform_tree(1, 5.0, np.array([row] * 3))
    o = np.array([[0.1, 0.2, 3.0], [0.1, 0.2, -3.0]], np.float32)
    d = np.array([[0, 0, -1], [0, 0, 1]], np.float32)
    r = core.query(tree, o, d, model=core.EXP, opts=core.NO_STOP)
    y00, y10 = 0.5 / math.sqrt(math.pi), math.sqrt(3 / (4 * math.pi))
    a = 1 - math.exp(-5.0 * 2.0)
    up = LMAX / (1 + math.exp(-(-2.0 * y00 + 4.0 * y10))) * a
    down = LMAX / (1 + math.exp(-(-2.0 * y00 - 4.0 * y10))) * a
    assert r["L"][0, 0] == pytest.approx(up, rel=1e-13)
    assert r["L"][1, 0] == pytest.approx(down, rel=1e-13)
    assert up > 10 * down


@pytest.mark.parametrize("model", [core.LINEAR, core.EXP])
def test_two_leaf_closed_form_and_order(model):
    # cells A = (0,0,0) and B = (1,0,0) of a depth-1 tree, degree-0 emission
    sA, sB = float(np.float32(0.9)), 3.0
    cA, cB = -6.0, 1.5
    tree = inputs.tree_from_cells(1, [[0, 0, 0], [1, 0, 0]], [sA, sB],
                                  np.array([[[cA]] * 3, [[cB]] * 3]))
    y00 = 0.5 / math.sqrt(math.pi)
    phiA, phiB = LMAX / (1 + math.exp(-cA * y00)), LMAX / (1 + math.exp(-cB * y00))
    for sgn in (1.0, -1.0):
        o = np.array([[-3.0 * sgn, -0.47, -0.53]], np.float32)
        d = np.array([[sgn, 0.0123, -0.0211]], np.float32)
        d /= np.linalg.norm(d)
        r = core.query(tree, o, d, model=model, opts=core.NO_STOP | core.NO_SKIP)
        dl = _dlen(d[0])
        ta = _chords(o[0], d[0], (-1, -1, -1), (0, 0, 0))
        tb = _chords(o[0], d[0], (0, -1, -1), (1, 0, 0))
        dA, dB = float(ta[1] - ta[0]) * dl, float(tb[1] - tb[0]) * dl
        first, second = ((sA, dA, phiA), (sB, dB, phiB)) if sgn > 0 else ((sB, dB, phiB), (sA, dA, phiA))
        if model == core.EXP:
            w1 = 1 - math.exp(-first[0] * first[1])
            w2 = (1 - w1) * (1 - math.exp(-second[0] * second[1]))
        else:
            w1 = min(1.0, first[0] * first[1])
            w2 = min(1.0 - w1, second[0] * second[1])
        ref = w1 * first[2] + w2 * second[2]
        assert r["L"][0, 0] == pytest.approx(ref, rel=1e-12)
        assert r["alpha"][0] == pytest.approx(w1 + w2, rel=1e-12)
        assert r["count"][0] == 2


def test_empty_tree_returns_zero():
    tree = inputs.empty_tree(5)
    o, d = inputs.rays.sphere_to_cube(500, 7)
    for model in (core.LINEAR, core.EXP):
        r = core.query(tree, o, d, model=model)
        assert np.all(r["L"] == 0) and np.all(r["alpha"] == 0) and np.all(r["count"] == 0)


def test_sigma_min_skip_and_boundary():
    # sigma below 0.1f is skipped; exactly 0.1f is composited
    below = inputs.uniform_tree(2, np.nextafter(np.float32(0.1), np.float32(0)), np.zeros((3, 1)))
    at = inputs.uniform_tree(2, np.float32(0.1), np.zeros((3, 1)))
    o, d = _rays_through_cube(16, 5)
    rb = core.query(below, o, d)
    ra = core.query(at, o, d)
    assert np.all(rb["L"] == 0) and np.all(rb["count"] > 0)
    assert np.all(ra["L"] > 0) and np.all(ra["n_comp"] == ra["count"])
    rn = core.query(below, o, d, opts=core.NO_SKIP)
    assert np.all(rn["L"] > 0)


def test_alpha_max_stop():
    # dense uniform cube: the march stops at the first leaf where 1 - T >= 0.9
    tree = inputs.uniform_tree(3, 8.0, np.zeros((3, 1)))
    o, d = _rays_through_cube(64, 6)
    for model in (core.LINEAR, core.EXP):
        r = core.query(tree, o, d, model=model)
        free = core.query(tree, o, d, model=model, opts=core.NO_STOP)
        for i in range(len(o)):
            segs, _ = exact.march_octree(tree, o[i], d[i])
            Y = core.sh_eval(0, -d[i].astype(np.float64) / _dlen(d[i]))
            c = exact.composite(tree, segs, d[i], Y, model)
            if free["alpha"][i] >= 0.9:
                assert r["term_idx"][i] == r["count"][i] - 1 >= 0
                assert r["alpha"][i] >= np.float32(0.9)
                assert len(c["alphas"]) < 2 or c["alphas"][-2] < np.float32(0.9)
            else:
                assert r["term_idx"][i] == -1


def test_invariants_on_small_config(c0_tree):
    o, d = inputs.rays.sphere_to_cube(4096, 11)
    for model in (core.LINEAR, core.EXP):
        r = core.query(c0_tree, o, d, model=model)
        assert np.all((r["alpha"] >= 0) & (r["alpha"] <= 1))
        assert np.all(r["L"] >= 0)
        assert np.all(r["L"] <= LMAX * r["alpha"][:, None] * (1 + 1e-12) + 1e-300)
        # stop only (no skip) vs fully heuristic-free: identical prefix weights
        stop = core.query(c0_tree, o, d, model=model, opts=core.NO_SKIP)
        free = core.query(c0_tree, o, d, model=model, opts=core.NO_SKIP | core.NO_STOP)
        gap = free["L"] - stop["L"]
        tstop = 1.0 - stop["alpha"]
        assert np.all(gap >= -1e-9 * (1 + free["L"]))
        assert np.all(gap <= LMAX * tstop[:, None] + 1e-9 * (1 + free["L"]))


def test_weights_sum_to_alpha_and_transmittance_never_increases(c0_tree):
    o, d = inputs.rays.sphere_to_cube(300, 12)
    for model in (core.LINEAR, core.EXP):
        for i in range(len(o)):
            segs, _ = exact.march_octree(c0_tree, o[i], d[i])
            Y = core.sh_eval(2, -d[i].astype(np.float64) / _dlen(d[i]))
            c = exact.composite(c0_tree, segs, d[i], Y, model, no_stop=True)
            assert all(w >= 0 for w in c["weights"])
            assert sum(c["weights"]) == pytest.approx(c["alpha"], rel=1e-12, abs=1e-15)
            al = c["alphas"]
            assert all(b >= a for a, b in zip(al, al[1:]))


def test_storage_dequantisation_matches_torch():
    import torch
    rng = np.random.default_rng(0)
    x = np.concatenate([rng.normal(0, 30, 20000), 10.0 ** rng.uniform(-9, 4, 20000),
                        [0.0, -0.0, 1e-40, 65504.0, 1.00390625, 1.01171875]]).astype(np.float32)
    t = torch.from_numpy(x)
    assert np.array_equal(core.dequantize(x, "bf16"), t.to(torch.bfloat16).double().numpy())
    assert np.array_equal(core.dequantize(x, "f16"), t.to(torch.float16).double().numpy())
