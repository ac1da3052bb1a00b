"""Exact-rational ray traversal for the oracle (test infrastructure only).

Three independent ways to obtain the leaf sequence of one ray, all in exact
rational arithmetic (fractions.Fraction; every float32 input is a dyadic
rational, so nothing is rounded):

  march_octree  the oracle's octree march (locate the point just after t by
                descending from the root, jump to the node's exit) -- the same
                steps as the FP64 C march, used for rays whose FP64 decisions
                fell inside the filter;
  brute_force   every data leaf's ray-cube interval, kept when it has positive
                length, sorted by entry parameter (small trees);
  dense_dda     Amanatides & Woo grid stepping over every max-depth cell
                (1987), stepping all tied axes at once (small trees).

A leaf sequence is a list of (leaf_index, morton_id, t_enter, t_exit) with
exact Fraction parameters.  composite() turns one into radiance in FP64 with
the same formulas as the C march (Sec. 4.1, Eqs. 3-5; Sec. 4.2, Eq. 6;
Sec. 6.2 heuristics).
"""
from __future__ import annotations

import math
from fractions import Fraction as Fr

import numpy as np

FNV_OFFSET = 14695981039346656037
FNV_PRIME = 1099511628211
MASK64 = (1 << 64) - 1


def fnv(ids) -> int:
    h = FNV_OFFSET
    for i in ids:
        h = ((h ^ int(i)) * FNV_PRIME) & MASK64
    return h


def _morton(x: int, y: int, z: int) -> int:
    m = 0
    for b in range(10):
        m |= ((x >> b) & 1) << (3 * b)
        m |= ((y >> b) & 1) << (3 * b + 1)
        m |= ((z >> b) & 1) << (3 * b + 2)
    return m


class _Ray:
    def __init__(self, o, d, depth):
        self.of = [float(v) for v in o]
        self.df = [float(v) for v in d]
        self.o = [Fr(v) for v in self.of]
        self.d = [Fr(v) for v in self.df]
        self.N = 1 << depth
        self.h = Fr(2, self.N)

    def plane(self, k):
        return -1 + k * self.h

    def tcross(self, a, P):
        return (P - self.o[a]) / self.d[a]

    def clip(self):
        """Exact [t_start, t_out] of the ray inside [-1,1)^3, or None."""
        if not all(math.isfinite(v) for v in self.of + self.df):
            return None
        if all(v == 0.0 for v in self.df):
            return None
        t_in, t_out = None, None
        for a in range(3):
            if self.d[a] == 0:
                if not (-1 <= self.o[a] < 1):
                    return None
                continue
            t0, t1 = self.tcross(a, Fr(-1)), self.tcross(a, Fr(1))
            tn, tf = min(t0, t1), max(t0, t1)
            t_in = tn if t_in is None else max(t_in, tn)
            t_out = tf if t_out is None else min(t_out, tf)
        t_start = max(Fr(0), t_in)
        if not (t_out > t_start):
            return None
        return t_start, t_out


def march_octree(tree, o, d, with_ordinals=False):
    """Octree march in exact arithmetic.  Returns (segments, n_nodes_visited)
    and, with with_ordinals, the 1-based node ordinal of every segment."""
    r = _Ray(o, d, tree.depth)
    span = r.clip()
    if span is None:
        return ([], 0, []) if with_ordinals else ([], 0)
    t, t_out = span
    N = r.N
    child = tree.child
    segs = []
    ordinals = []
    visited = 0
    while t < t_out:
        node, level = 0, 0
        lo = [0, 0, 0]
        while True:
            half = N >> (level + 1)
            octant = 0
            for a in range(3):
                P = r.plane(lo[a] + half)
                if r.d[a] == 0:
                    up = r.o[a] >= P
                elif r.d[a] > 0:
                    up = t >= r.tcross(a, P)
                else:
                    up = t < r.tcross(a, P)
                if up:
                    octant |= 1 << a
                    lo[a] += half
            c = int(child[node, octant])
            level += 1
            if c > 0:
                node = c
                continue
            break
        visited += 1
        size = N >> level
        t_next = None
        for a in range(3):
            if r.d[a] == 0:
                continue
            k = lo[a] + size if r.d[a] > 0 else lo[a]
            ta = r.tcross(a, r.plane(k))
            t_next = ta if t_next is None else min(t_next, ta)
        t_next = min(t_next, t_out)
        assert t_next > t
        if c < 0:
            segs.append((-c - 1, _morton(*lo), t, t_next))
            ordinals.append(visited)
        t = t_next
    return (segs, visited, ordinals) if with_ordinals else (segs, visited)


def brute_force(tree, o, d, leaf_cells):
    """All data leaves, exact intervals, positive length, sorted by entry."""
    r = _Ray(o, d, tree.depth)
    span = r.clip()
    if span is None:
        return []
    t_start, t_out = span
    out = []
    for leaf, (x, y, z) in enumerate(np.asarray(leaf_cells).tolist()):
        lo_t, hi_t = t_start, t_out
        ok = True
        for a, q in enumerate((x, y, z)):
            lo_p, hi_p = r.plane(q), r.plane(q + 1)
            if r.d[a] == 0:
                if not (lo_p <= r.o[a] < hi_p):
                    ok = False
                    break
                continue
            t0, t1 = r.tcross(a, lo_p), r.tcross(a, hi_p)
            lo_t = max(lo_t, min(t0, t1))
            hi_t = min(hi_t, max(t0, t1))
        if ok and hi_t > lo_t:
            out.append((leaf, _morton(x, y, z), lo_t, hi_t))
    out.sort(key=lambda s: s[2])
    return out


def dense_dda(tree, o, d, leaf_cells):
    """Cell-by-cell grid stepping over the full 2^D grid."""
    r = _Ray(o, d, tree.depth)
    span = r.clip()
    if span is None:
        return []
    t, t_out = span
    N = r.N
    lookup = {tuple(c): i for i, c in enumerate(np.asarray(leaf_cells).tolist())}
    # cell containing the point just after t
    q = [0, 0, 0]
    for a in range(3):
        if r.d[a] == 0:
            p = r.o[a]
            k = math.floor((p + 1) / r.h)
        else:
            p = r.o[a] + t * r.d[a]
            k = math.floor((p + 1) / r.h)
            if r.d[a] < 0 and p == r.plane(k):
                k -= 1       # on a plane, moving down: the lower cell
        q[a] = min(max(k, 0), N - 1)
    t_max = [None] * 3
    for a in range(3):
        if r.d[a] != 0:
            k = q[a] + 1 if r.d[a] > 0 else q[a]
            t_max[a] = r.tcross(a, r.plane(k))
    out = []
    while t < t_out:
        cand = [t_max[a] for a in range(3) if t_max[a] is not None]
        t_next = min(min(cand), t_out)
        leaf = lookup.get((q[0], q[1], q[2]))
        if leaf is not None and t_next > t:
            out.append((leaf, _morton(*q), t, t_next))
        if t_next >= t_out:
            break
        for a in range(3):
            if t_max[a] is not None and t_max[a] == t_next:
                step = 1 if r.d[a] > 0 else -1
                q[a] += step
                k = q[a] + 1 if r.d[a] > 0 else q[a]
                t_max[a] = r.tcross(a, r.plane(k))
        t = t_next
        if not all(0 <= v < N for v in q):
            break
    return out


FORCE_CONTINUE = 1 << 30


def composite(tree, segs, d, Y, model, no_stop=False, no_skip=False, flip_test=-1,
              sigma=None, sh=None, eta=1e-4, force_stop=None):
    """FP64 compositing of an exact leaf sequence.  Returns a dict with L,
    alpha, count, hash, term_idx, n_comp, first_amb_test, amb_tests (the
    stop tests within eta of the threshold).  flip_test inverts one stop
    test; force_stop takes another valid outcome of a threshold-ambiguous
    ray: continue at every ambiguous test before test force_stop and stop
    there (FORCE_CONTINUE: continue at every ambiguous test)."""
    sigma = tree.sigma.astype(np.float64) if sigma is None else sigma
    sh = tree.sh.astype(np.float64) if sh is None else sh
    df = [float(v) for v in d]
    dlen = math.sqrt(df[0] * df[0] + df[1] * df[1] + df[2] * df[2])
    smin = float(np.float32(tree.sigma_min))
    amax = float(np.float32(tree.alpha_max))
    K = sh.shape[-1]
    Tr = 1.0
    L = [0.0, 0.0, 0.0]
    ids = []
    term = -1
    n_comp = 0
    tests = 0
    first_amb = -1
    weights, alphas = [], []
    amb_tests = []
    for (leaf, mid, t0, t1) in segs:
        ids.append(mid)
        sig = float(sigma[leaf])
        if no_skip or sig >= smin:
            delta = float(t1 - t0) * dlen
            if model == 0:
                tau = sig * delta
                w = tau if tau < Tr else Tr
            else:
                w = -Tr * math.expm1(-sig * delta)
            for c in range(3):
                x = 0.0
                for k in range(K):
                    x += float(sh[leaf, c, k]) * Y[k]
                phi = tree.l_max / (1.0 + math.exp(-x))
                L[c] += w * phi
            Tr -= w
            n_comp += 1
            weights.append(w)
            alphas.append(1.0 - Tr)
            if not no_stop:
                alpha = 1.0 - Tr
                stop = alpha >= amax
                amb = abs(alpha - amax) <= eta
                if amb:
                    amb_tests.append(tests)
                    if first_amb < 0:
                        first_amb = tests
                if tests == flip_test:
                    stop = not stop
                if force_stop is not None:
                    if tests == force_stop:
                        stop = True
                    elif amb:
                        stop = False
                tests += 1
                if stop:
                    term = len(ids) - 1
                    break
    return {"L": L, "alpha": 1.0 - Tr, "count": len(ids), "hash": fnv(ids), "ids": ids,
            "term_idx": term, "n_comp": n_comp, "first_amb_test": first_amb, "amb_tests": amb_tests,
            "weights": weights, "alphas": alphas}
