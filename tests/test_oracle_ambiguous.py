"""Pins of the oracle's second candidate for threshold-ambiguous rays.

The alpha_max stop (Sec. 6.2, "Performance vs Quality") is tested after
every composited leaf: stop once 1 - T >= alpha_max (float32 0.9).  When a
test lands within eta = 1e-4 of the threshold, float32 compositing on the
GPU may take the other branch, so the oracle also returns the outcome with
that one test inverted (alt_*).  Here a ray crosses a row of hand-built
leaves whose densities put 1 - T just above or just below the threshold at a
chosen test; both candidates are checked against the closed forms of the
linear (Sec. 4.1, Eq. 4) and exponential models: stop at the ambiguous leaf,
or composite the next leaf too and stop there.  Both oracle paths are
pinned: the FP64 march and the exact-rational re-run.
"""
import math
from fractions import Fraction as Fr

import numpy as np
import pytest

import inputs
from oracle import core

LMAX = inputs.L_MAX
AMAX = float(np.float32(0.9))
Y00 = 0.5 / math.sqrt(math.pi)
DEPTH = 2
# the row of leaves: cells x = 0..3 at y-cell 1, z-cell 1 of a depth-2 tree
CELLS = [(x, 1, 1) for x in range(4)]
DC = [-1.0, 2.0, 0.5, -3.0]          # degree-0 coefficient of each leaf
O = np.array([[-3.0, -0.26, -0.24]], np.float32)
D = np.array([[1.0, 0.001, -0.002]], np.float32)


def _morton(x, y, z):
    m = 0
    for b in range(DEPTH):
        m |= ((x >> b) & 1) << (3 * b) | ((y >> b) & 1) << (3 * b + 1) | ((z >> b) & 1) << (3 * b + 2)
    return m


def _fnv(ids):
    h = 14695981039346656037
    for i in ids:
        h = ((h ^ i) * 1099511628211) % (1 << 64)
    return h


def _deltas():
    """Chord length of the ray in each leaf cell (exact slab test, times |d|)."""
    o = [Fr(float(v)) for v in O[0]]
    d = [Fr(float(v)) for v in D[0]]
    dl = math.sqrt(sum(float(v) ** 2 for v in D[0]))
    out = []
    for (cx, cy, cz) in CELLS:
        lo = [Fr(-1) + Fr(c, 2) for c in (cx, cy, cz)]
        t0, t1 = Fr(-10 ** 9), Fr(10 ** 9)
        for a in range(3):
            u, v = (lo[a] - o[a]) / d[a], (lo[a] + Fr(1, 2) - o[a]) / d[a]
            t0, t1 = max(t0, min(u, v)), min(t1, max(u, v))
        assert t1 > t0 > 0
        out.append(float(t1 - t0) * dl)
    return out


def _phi(c):
    return LMAX / (1.0 + math.exp(-c * Y00))


def _closed(sig, dlt, model, stop_at):
    """Radiance and alpha of compositing leaves 0..stop_at (Eq. 4 or
    Beer-Lambert), each weighted by its drop of transmittance."""
    T, L = 1.0, 0.0
    for i in range(stop_at + 1):
        if model == core.LINEAR:
            w = min(T, sig[i] * dlt[i])
        else:
            w = T * (1.0 - math.exp(-sig[i] * dlt[i]))
        L += w * _phi(DC[i])
        T -= w
    return L, 1.0 - T


def _tree(sig):
    sh = np.array([[[c]] * 3 for c in DC], np.float32)
    return inputs.tree_from_cells(DEPTH, CELLS, np.array(sig, np.float32), sh)


def _densities(model, amb_test, offset):
    """float32 densities that put 1 - T at AMAX + offset after leaf
    amb_test, about 0.5 after the leaves before it, and past the threshold
    after the next one."""
    dlt = _deltas()
    sig = [0.0] * 4
    if model == core.LINEAR:
        if amb_test == 1:
            sig[0] = 0.5 / dlt[0]
        prior = sum(sig[i] * dlt[i] for i in range(amb_test))
        sig[amb_test] = (AMAX + offset - prior) / dlt[amb_test]
    else:
        if amb_test == 1:
            sig[0] = -math.log(0.5) / dlt[0]
        prior = sum(sig[i] * dlt[i] for i in range(amb_test))
        sig[amb_test] = (-math.log(1.0 - AMAX - offset) - prior) / dlt[amb_test]
    sig[amb_test + 1] = 40.0           # the next leaf saturates: 1 - T >= 0.9 after it
    for i in range(amb_test + 2, 4):
        sig[i] = 1.0
    return [float(np.float32(s)) for s in sig], dlt


def _check(r, i, L, alpha, count, term, ids, prefix=""):
    assert r[prefix + "L"][i, 0] == pytest.approx(L, rel=1e-12)
    assert r[prefix + "alpha"][i] == pytest.approx(alpha, rel=1e-12)
    key = {"count": "count", "term": "term_idx", "hash": "hash"}
    if prefix:
        key = {"count": "alt_count", "term": "alt_term", "hash": "alt_hash"}
    assert int(r[key["count"]][i]) == count
    assert int(r[key["term"]][i]) == term
    assert int(r[key["hash"]][i]) == _fnv(ids)


@pytest.mark.parametrize("exact_path", [False, True])
@pytest.mark.parametrize("model", [core.LINEAR, core.EXP])
@pytest.mark.parametrize("amb_test", [0, 1])
@pytest.mark.parametrize("offset", [4e-5, -4e-5])
def test_both_candidates_closed_form(exact_path, model, amb_test, offset):
    sig, dlt = _densities(model, amb_test, offset)
    tree = _tree(sig)
    # the premise: the test at leaf amb_test is within eta of the threshold,
    # on the side `offset` says, and the next leaf saturates
    _, a_amb = _closed(sig, dlt, model, amb_test)
    assert abs(a_amb - AMAX) <= core.ETA and (a_amb >= AMAX) == (offset > 0)
    _, a_next = _closed(sig, dlt, model, amb_test + 1)
    assert a_next >= AMAX + core.ETA
    r = core.query(tree, O, D, model=model, force_exact=exact_path)
    assert r["alt_valid"][0] == 1
    ids = [_morton(*c) for c in CELLS]
    stop_here = _closed(sig, dlt, model, amb_test)
    stop_next = _closed(sig, dlt, model, amb_test + 1)
    here = (stop_here[0], stop_here[1], amb_test + 1, amb_test, ids[:amb_test + 1])
    nxt = (stop_next[0], stop_next[1], amb_test + 2, amb_test + 1, ids[:amb_test + 2])
    canon, alt = (here, nxt) if offset > 0 else (nxt, here)
    _check(r, 0, *canon)
    _check(r, 0, *alt, prefix="alt_")


@pytest.mark.parametrize("model", [core.LINEAR, core.EXP])
def test_clear_margin_has_no_second_candidate(model):
    for offset in (3e-4, -3e-4):
        sig, dlt = _densities(model, 1, offset)
        r = core.query(_tree(sig), O, D, model=model)
        assert r["alt_valid"][0] == 0
        term = 1 if offset > 0 else 2
        assert r["term_idx"][0] == term
        L, a = _closed(sig, dlt, model, term)
        assert r["L"][0, 0] == pytest.approx(L, rel=1e-12)
        assert r["alpha"][0] == pytest.approx(a, rel=1e-12)


def test_no_stop_has_no_second_candidate():
    sig, _ = _densities(core.LINEAR, 1, 4e-5)
    r = core.query(_tree(sig), O, D, model=core.LINEAR, opts=core.NO_STOP)
    assert r["alt_valid"][0] == 0 and r["term_idx"][0] == -1 and r["count"][0] == 4


def _densities_two(model, first_offset, second_offset):
    """Densities putting 1 - T at AMAX + first_offset after leaf 0 and at
    AMAX + second_offset after leaf 1 (two ambiguous tests in a row), then a
    saturating leaf."""
    dlt = _deltas()
    a0, a1 = AMAX + first_offset, AMAX + second_offset
    if model == core.LINEAR:
        s0, s1 = a0 / dlt[0], (a1 - a0) / dlt[1]
    else:
        s0 = -math.log(1.0 - a0) / dlt[0]
        s1 = (-math.log(1.0 - a1) + math.log(1.0 - a0)) / dlt[1]
    sig = [s0, s1, 40.0, 1.0]
    return [float(np.float32(s)) for s in sig], dlt


@pytest.mark.parametrize("exact_path", [False, True])
@pytest.mark.parametrize("model", [core.LINEAR, core.EXP])
@pytest.mark.parametrize("offsets", [(-6e-5, 3e-5), (-8e-5, -2e-5), (2e-5, 7e-5)])
def test_every_outcome_of_two_ambiguous_tests(exact_path, model, offsets):
    """Two stop tests in a row within eta of the threshold: each may go
    either way, so the valid outcomes are stop at the first, stop at the
    second, or continue through both (and stop at the saturating third
    leaf).  candidates() lists exactly these, in that order after the
    continue-through one, each equal to its closed form; the canonical
    outcome of query() is one of them.  (The second leaf adds under 1e-4 to
    1 - T, so its density is below sigma_min: the skip is off here.)"""
    sig, dlt = _densities_two(model, *offsets)
    a0, a1 = _closed(sig, dlt, model, 0)[1], _closed(sig, dlt, model, 1)[1]
    assert abs(a0 - AMAX) <= core.ETA and abs(a1 - AMAX) <= core.ETA
    assert _closed(sig, dlt, model, 2)[1] >= AMAX + core.ETA
    tree = _tree(sig)
    c = core.candidates(tree, O, D, model=model, opts=core.NO_SKIP, force_exact=exact_path)
    assert list(c["valid"][0]) == [1, 1, 1, 0, 0, 0, 0, 0]
    ids = [_morton(*cell) for cell in CELLS]
    for slot, stop_at in ((0, 2), (1, 0), (2, 1)):
        L, a = _closed(sig, dlt, model, stop_at)
        assert c["L"][0, slot, 0] == pytest.approx(L, rel=1e-12)
        assert c["alpha"][0, slot] == pytest.approx(a, rel=1e-12)
        assert c["count"][0, slot] == stop_at + 1 and c["term_idx"][0, slot] == stop_at
        assert int(c["hash"][0, slot]) == _fnv(ids[:stop_at + 1])
    r = core.query(tree, O, D, model=model, opts=core.NO_SKIP)
    canon = 0 if offsets[0] >= 0 else (1 if offsets[1] >= 0 else 2)
    assert r["term_idx"][0] == canon
    # one clear test: a single candidate, the canonical outcome
    sig1, _ = _densities(model, 1, 3e-4)
    c1 = core.candidates(_tree(sig1), O, D, model=model, force_exact=exact_path)
    assert list(c1["valid"][0]) == [1, 0, 0, 0, 0, 0, 0, 0] and c1["term_idx"][0, 0] == 1
