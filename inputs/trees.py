"""Seeded synthetic luminaire plenoctrees.

This module only manufactures input data (a density field sampled at voxel
centres, pruned into a sparse octree, plus per-leaf spherical-harmonic
coefficients).  It holds none of the query's arithmetic: no ray geometry, no
SH evaluation, no compositing.  Both the CPU oracle and the GPU library read
the arrays it returns.

Field (stands in for the distilled NeRF of Sec. 5, "Creating the plenoctree"):

    log sigma(x) = ln(1e-3) + sum_k a_k exp(-|x - c_k|^2 / (2 r_k^2)),
    sigma = min(exp(log sigma), 50)

with c_k ~ U[-0.7, 0.7]^3, r_k = s * U(0.08, 0.3), a_k = U(0.5, 1) ln(5e4).
A voxel is kept iff sigma at its centre is >= 0.01 (the prune threshold of
Sec. 5); optional thin shells (two finest voxels thick, sigma = 50) stand in
for glass.  All data leaves sit at the maximum depth.  The radius scale s is
set by bisection on a coarse grid to reach a target occupancy.

Emission is smooth per blob: blob k has a magnitude m_k ~ logU(1e-2, 1e3) and a
tint rgb_k ~ U(0.2, 1)^3; a leaf blends them with Gaussian weights.  The DC
coefficient is the logit of the blended magnitude over L_max, divided by the
constant degree-0 basis value 1/(2 sqrt(pi)); higher coefficients are
blob-weighted N(0, 0.5^2) draws.

Octree layout (shared convention with the file format):
  child[n_nodes][8] int32: > 0 internal node index, < 0 -(leaf + 1), 0 empty.
  Node 0 is the root; nodes are in breadth-first order, Morton order within a
  level.  Octant index = bx | by << 1 | bz << 2.  Leaves are numbered in
  Morton order of their cells (x bit i -> bit 3i, y -> 3i+1, z -> 3i+2).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

L_MAX = 2048.0
SIGMA_MIN = 0.1          # render-time skip threshold (Sec. 6.2)
ALPHA_MAX = 0.9          # render-time saturation threshold (Sec. 6.2)
PRUNE_SIGMA = 0.01       # extraction prune threshold (Sec. 5)
SIGMA_CLAMP = 50.0
LOG_BASE = math.log(1e-3)
# occupied iff ln(1e-3) + S >= ln(0.01)  <=>  S >= ln(10)
OCC_S = math.log(PRUNE_SIGMA) - LOG_BASE


@dataclass
class TreeSpec:
    depth: int
    n_blobs: int = 8
    n_shells: int = 0
    sh_degree: int = 2
    seed: int = 0
    occupancy: float | None = 0.30      # target occupied fraction of the blob field
    scale: float | None = None          # explicit radius scale (skips bisection)
    l_max: float = L_MAX


@dataclass
class Tree:
    depth: int
    sh_degree: int
    l_max: float
    child: np.ndarray            # int32 [n_nodes, 8]
    sigma: np.ndarray            # float32 [n_leaves]
    sh: np.ndarray               # float32 [n_leaves, 3, K]
    leaf_cells: np.ndarray       # int32 [n_leaves, 3] (x, y, z) cell coords, Morton order
    sigma_min: float = SIGMA_MIN
    alpha_max: float = ALPHA_MAX
    meta: dict = field(default_factory=dict)

    @property
    def n_nodes(self) -> int:
        return int(self.child.shape[0])

    @property
    def n_leaves(self) -> int:
        return int(self.sigma.shape[0])

    @property
    def K(self) -> int:
        return (self.sh_degree + 1) ** 2


# --------------------------------------------------------------------------
# Morton codes
# --------------------------------------------------------------------------
def _part1by2(v: np.ndarray) -> np.ndarray:
    v = v.astype(np.uint64) & np.uint64(0x3FF)
    v = (v | (v << np.uint64(16))) & np.uint64(0x030000FF)
    v = (v | (v << np.uint64(8))) & np.uint64(0x0300F00F)
    v = (v | (v << np.uint64(4))) & np.uint64(0x030C30C3)
    v = (v | (v << np.uint64(2))) & np.uint64(0x09249249)
    return v


def morton3(x, y, z) -> np.ndarray:
    return _part1by2(np.asarray(x)) | (_part1by2(np.asarray(y)) << np.uint64(1)) | (
        _part1by2(np.asarray(z)) << np.uint64(2))


def _compact1by2(v: np.ndarray) -> np.ndarray:
    v = v.astype(np.uint64) & np.uint64(0x09249249)
    v = (v | (v >> np.uint64(2))) & np.uint64(0x030C30C3)
    v = (v | (v >> np.uint64(4))) & np.uint64(0x0300F00F)
    v = (v | (v >> np.uint64(8))) & np.uint64(0x030000FF)
    v = (v | (v >> np.uint64(16))) & np.uint64(0x3FF)
    return v


def demorton3(code: np.ndarray):
    code = np.asarray(code, dtype=np.uint64)
    return (_compact1by2(code), _compact1by2(code >> np.uint64(1)),
            _compact1by2(code >> np.uint64(2)))


# --------------------------------------------------------------------------
# Octree from a set of occupied finest cells
# --------------------------------------------------------------------------
def build_octree(depth: int, codes: np.ndarray) -> np.ndarray:
    """Child table for the sparse octree whose occupied max-depth cells have
    the given Morton codes.  Returns int32 [n_nodes, 8]."""
    if depth < 1 or depth > 10:
        raise ValueError("depth must be in [1, 10]")
    codes = np.unique(np.asarray(codes, dtype=np.uint64))
    levels = [None] * (depth + 1)
    levels[depth] = codes
    for lvl in range(depth - 1, -1, -1):
        levels[lvl] = np.unique(levels[lvl + 1] >> np.uint64(3))
    levels[0] = np.zeros(1, dtype=np.uint64)           # the root always exists
    base = [0] * (depth + 1)
    acc = 0
    for lvl in range(depth):
        base[lvl] = acc
        acc += levels[lvl].size
    n_nodes = acc
    child = np.zeros((n_nodes, 8), dtype=np.int32)
    for lvl in range(depth):
        kids = levels[lvl + 1]
        if kids.size == 0:
            continue
        parent = kids >> np.uint64(3)
        octant = (kids & np.uint64(7)).astype(np.int64)
        pidx = np.searchsorted(levels[lvl], parent).astype(np.int64)
        idx = np.arange(kids.size, dtype=np.int64)
        if lvl + 1 < depth:
            val = base[lvl + 1] + idx
        else:
            val = -(idx + 1)
        child[base[lvl] + pidx, octant] = val.astype(np.int32)
    return child


# --------------------------------------------------------------------------
# Field
# --------------------------------------------------------------------------
def cell_centres(depth: int) -> np.ndarray:
    n = 1 << depth
    return -1.0 + (np.arange(n, dtype=np.float64) + 0.5) * (2.0 / n)


def _profile(xs: np.ndarray, c: float, r: float) -> np.ndarray:
    # libm exp per sample so the occupancy pattern does not depend on the
    # host's SIMD exp implementation
    inv = 1.0 / (2.0 * r * r)
    return np.array([math.exp(-((x - c) ** 2) * inv) for x in xs.tolist()])


@dataclass
class _Params:
    centres: np.ndarray   # [nb, 3]
    u: np.ndarray         # [nb]
    amp: np.ndarray       # [nb]
    shells: np.ndarray    # [ns, 4]  (cx, cy, cz, R)
    mag: np.ndarray       # [nb]
    tint: np.ndarray      # [nb, 3]
    hi: np.ndarray        # [nb, 3, K-1]


def _draw_params(spec: TreeSpec) -> _Params:
    rng = np.random.default_rng(spec.seed)
    nb = spec.n_blobs
    K = (spec.sh_degree + 1) ** 2
    centres = rng.uniform(-0.7, 0.7, size=(nb, 3))
    u = rng.uniform(0.08, 0.3, size=nb)
    amp = rng.uniform(0.5, 1.0, size=nb) * math.log(5e4)
    shells = np.zeros((spec.n_shells, 4))
    if spec.n_shells:
        shells[:, :3] = rng.uniform(-0.5, 0.5, size=(spec.n_shells, 3))
        shells[:, 3] = rng.uniform(0.25, 0.6, size=spec.n_shells)
    mag = 10.0 ** rng.uniform(-2.0, 3.0, size=nb)
    tint = rng.uniform(0.2, 1.0, size=(nb, 3))
    hi = rng.normal(0.0, 0.5, size=(nb, 3, max(K - 1, 0)))
    return _Params(centres, u, amp, shells, mag, tint, hi)


def _blob_sum_slabs(depth: int, p: _Params, s: float, on_slab):
    """Evaluate S(x) = sum_k a_k g_k(x) at every cell centre, z-slab by z-slab,
    in a fixed summation order, and hand each slab to on_slab(z0, S)."""
    n = 1 << depth
    xs = cell_centres(depth)
    r = s * p.u
    gx = [_profile(xs, p.centres[k, 0], r[k]) for k in range(len(r))]
    gy = [_profile(xs, p.centres[k, 1], r[k]) for k in range(len(r))]
    gz = [_profile(xs, p.centres[k, 2], r[k]) for k in range(len(r))]
    plane = [np.multiply.outer(gy[k], gx[k]) for k in range(len(r))]   # [y, x]
    zc = max(1, min(n, (1 << 22) // (n * n) or 1))
    for z0 in range(0, n, zc):
        z1 = min(n, z0 + zc)
        S = np.zeros((z1 - z0, n, n))
        for k in range(len(r)):
            S += (p.amp[k] * gz[k][z0:z1])[:, None, None] * plane[k][None]
        on_slab(z0, S)


def _occupied_fraction(depth: int, p: _Params, s: float) -> float:
    tot = [0]

    def cb(z0, S):
        tot[0] += int(np.count_nonzero(S >= OCC_S))

    _blob_sum_slabs(depth, p, s, cb)
    return tot[0] / float(1 << (3 * depth))


def _solve_scale(spec: TreeSpec, p: _Params) -> float:
    if spec.scale is not None:
        return float(spec.scale)
    probe = min(spec.depth, 6)
    lo, hi = 0.05, 8.0
    for _ in range(40):
        mid = math.sqrt(lo * hi)
        if _occupied_fraction(probe, p, mid) < spec.occupancy:
            lo = mid
        else:
            hi = mid
    return math.sqrt(lo * hi)


def field_params(spec: TreeSpec) -> dict:
    """Parameters of the continuous field the tree of `spec` samples (the
    stand-in for a trained radiance field that a plenoctree is distilled
    from): blob centres, radii (with the solved scale), log-density
    amplitudes, per-blob emission (magnitude times tint) and higher SH
    coefficients, shells (centre, radius) of half-width one finest voxel at
    the spec's depth, base log-density, density clamp, L_max, SH degree."""
    p = _draw_params(spec)
    s = _solve_scale(spec, p) if spec.n_blobs else 1.0
    K = (spec.sh_degree + 1) ** 2
    return {"centres": p.centres.copy(), "radii": s * p.u, "amps": p.amp.copy(),
            "emission": p.mag[:, None] * p.tint, "hi": p.hi.reshape(spec.n_blobs, 3, K - 1).copy(),
            "shells": p.shells.copy(), "shell_half_width": 2.0 / (1 << spec.depth),
            "log_base": LOG_BASE, "sigma_max": SIGMA_CLAMP, "l_max": float(spec.l_max),
            "sh_degree": spec.sh_degree}


def make_tree(spec: TreeSpec) -> Tree:
    """Generate the seeded synthetic plenoctree described by spec."""
    depth = spec.depth
    n = 1 << depth
    h = 2.0 / n
    K = (spec.sh_degree + 1) ** 2
    p = _draw_params(spec)
    s = _solve_scale(spec, p) if spec.n_blobs else 1.0
    xs = cell_centres(depth)

    occ_cells = []
    occ_logs = []

    def cb(z0, S):
        zz, yy, xx = np.nonzero(S >= OCC_S)
        occ_cells.append(np.stack([xx, yy, zz + z0], axis=1).astype(np.int32))
        occ_logs.append(LOG_BASE + S[zz, yy, xx])

    if spec.n_blobs:
        _blob_sum_slabs(depth, p, s, cb)
    cells = np.concatenate(occ_cells) if occ_cells else np.zeros((0, 3), np.int32)
    logs = np.concatenate(occ_logs) if occ_logs else np.zeros(0)
    sig = np.minimum(np.exp(logs), SIGMA_CLAMP)

    if spec.n_shells:
        shell_cells = []
        for (cx, cy, cz, R) in p.shells:
            zc = max(1, (1 << 22) // (n * n) or 1)
            dy2 = (xs - cy) ** 2
            dx2 = (xs - cx) ** 2
            for z0 in range(0, n, zc):
                z1 = min(n, z0 + zc)
                dz2 = (xs[z0:z1] - cz) ** 2
                dist = np.sqrt(dz2[:, None, None] + dy2[None, :, None] + dx2[None, None, :])
                zz, yy, xx = np.nonzero(np.abs(dist - R) < h)
                shell_cells.append(np.stack([xx, yy, zz + z0], axis=1).astype(np.int32))
        sc = np.concatenate(shell_cells) if shell_cells else np.zeros((0, 3), np.int32)
        # shells override the blob density
        all_cells = np.concatenate([cells, sc])
        all_sig = np.concatenate([sig, np.full(len(sc), SIGMA_CLAMP)])
        codes_all = morton3(all_cells[:, 0], all_cells[:, 1], all_cells[:, 2])
        # keep the last occurrence (shell wins)
        order = np.argsort(codes_all, kind="stable")
        codes_sorted = codes_all[order]
        last = np.ones(len(order), dtype=bool)
        last[:-1] = codes_sorted[1:] != codes_sorted[:-1]
        keep = order[last]
        cells, sig = all_cells[keep], all_sig[keep]

    codes = morton3(cells[:, 0], cells[:, 1], cells[:, 2])
    order = np.argsort(codes, kind="stable")
    codes, cells, sig = codes[order], cells[order], sig[order]
    child = build_octree(depth, codes)

    # emission: per-blob smooth SH
    nl = cells.shape[0]
    sh = np.zeros((nl, 3, K), dtype=np.float64)
    if nl and spec.n_blobs:
        pos = -1.0 + (cells.astype(np.float64) + 0.5) * h
        r = s * p.u
        chunk = 1 << 20
        for a in range(0, nl, chunk):
            b = min(nl, a + chunk)
            d2 = ((pos[a:b, None, :] - p.centres[None, :, :]) ** 2).sum(-1)   # [m, nb]
            lw = -d2 / (2.0 * r * r)[None, :]
            lw -= lw.max(axis=1, keepdims=True)
            w = np.exp(lw)
            w /= w.sum(axis=1, keepdims=True)
            E = w @ (p.mag[:, None] * p.tint)                                  # [m, 3]
            frac = E / spec.l_max
            sh[a:b, :, 0] = np.log(frac / (1.0 - frac)) * (2.0 * math.sqrt(math.pi))
            if K > 1:
                sh[a:b, :, 1:] = np.einsum("mk,kcj->mcj", w, p.hi)
    return Tree(depth=depth, sh_degree=spec.sh_degree, l_max=float(spec.l_max),
                child=child, sigma=sig.astype(np.float32), sh=sh.astype(np.float32),
                leaf_cells=cells.astype(np.int32),
                meta={"scale": s, "seed": spec.seed, "n_blobs": spec.n_blobs,
                      "n_shells": spec.n_shells})


# --------------------------------------------------------------------------
# Hand-built trees for closed-form tests
# --------------------------------------------------------------------------
def tree_from_cells(depth: int, cells, sigma, sh, l_max: float = L_MAX,
                    sh_degree: int | None = None) -> Tree:
    """Tree whose data leaves are exactly the given max-depth cells."""
    cells = np.asarray(cells, dtype=np.int64).reshape(-1, 3)
    sigma = np.asarray(sigma, dtype=np.float32).reshape(-1)
    sh = np.asarray(sh, dtype=np.float32)
    if sh.ndim == 2:
        sh = sh[:, None, :].repeat(3, axis=1)
    if sh_degree is None:
        sh_degree = int(round(math.sqrt(sh.shape[-1]))) - 1
    codes = morton3(cells[:, 0], cells[:, 1], cells[:, 2])
    order = np.argsort(codes, kind="stable")
    child = build_octree(depth, codes[order])
    return Tree(depth=depth, sh_degree=sh_degree, l_max=float(l_max), child=child,
                sigma=sigma[order], sh=sh[order].astype(np.float32),
                leaf_cells=cells[order].astype(np.int32))


def uniform_tree(depth: int, sigma: float, sh_row, l_max: float = L_MAX) -> Tree:
    """Every max-depth cell occupied with the same density and SH row."""
    n = 1 << depth
    g = np.arange(n)
    zz, yy, xx = np.meshgrid(g, g, g, indexing="ij")
    cells = np.stack([xx.ravel(), yy.ravel(), zz.ravel()], axis=1)
    sh_row = np.asarray(sh_row, dtype=np.float32)
    if sh_row.ndim == 1:
        sh_row = np.repeat(sh_row[None, :], 3, axis=0)
    sh = np.repeat(sh_row[None], len(cells), axis=0)
    return tree_from_cells(depth, cells, np.full(len(cells), sigma), sh, l_max)


def empty_tree(depth: int, sh_degree: int = 2, l_max: float = L_MAX) -> Tree:
    K = (sh_degree + 1) ** 2
    return Tree(depth=depth, sh_degree=sh_degree, l_max=l_max,
                child=np.zeros((1, 8), dtype=np.int32),
                sigma=np.zeros(0, np.float32), sh=np.zeros((0, 3, K), np.float32),
                leaf_cells=np.zeros((0, 3), np.int32))


def random_tree(depth: int, p_occ: float, seed: int, sh_degree: int = 2,
                l_max: float = L_MAX, sigma_range=(0.02, 50.0)) -> Tree:
    """I.i.d. occupancy and values: an adversarial structure for traversal tests."""
    rng = np.random.default_rng(seed)
    n = 1 << depth
    occ = rng.random((n, n, n)) < p_occ            # [z, y, x]
    zz, yy, xx = np.nonzero(occ)
    cells = np.stack([xx, yy, zz], axis=1)
    K = (sh_degree + 1) ** 2
    lo, hi = sigma_range
    sigma = np.exp(rng.uniform(math.log(lo), math.log(hi), size=len(cells)))
    sh = rng.normal(0.0, 1.5, size=(len(cells), 3, K))
    sh[:, :, 0] += rng.uniform(-20.0, 0.0, size=(len(cells), 3))
    return tree_from_cells(depth, cells, sigma, sh, l_max, sh_degree)


# --------------------------------------------------------------------------
# Workload configurations
# --------------------------------------------------------------------------
C0_TREE = TreeSpec(depth=6, n_blobs=8, n_shells=0, sh_degree=2, seed=0, occupancy=0.30)
# about 6M occupied leaves at 512^3 (4.5% of the cells, shells included)
C1_TREE = TreeSpec(depth=9, n_blobs=16, n_shells=4, sh_degree=2, seed=10, occupancy=0.040)


def cached_tree(spec: TreeSpec, cache_dir: str | None = None) -> Tree:
    """make_tree(spec), memoised as an .npz file (default: $LUMIQ_CACHE or
    <tmp>/lumiq_inputs) so that several processes on one machine generate a
    large tree once."""
    import hashlib
    import os
    import tempfile
    cache_dir = cache_dir or os.environ.get("LUMIQ_CACHE") or os.path.join(
        tempfile.gettempdir(), "lumiq_inputs")
    key = hashlib.sha1(repr(spec).encode()).hexdigest()[:16]
    path = os.path.join(cache_dir, f"tree_{key}.npz")
    if os.path.exists(path):
        try:
            z = np.load(path, allow_pickle=False)
            return Tree(depth=int(z["depth"]), sh_degree=int(z["sh_degree"]),
                        l_max=float(z["l_max"]), child=z["child"], sigma=z["sigma"], sh=z["sh"],
                        leaf_cells=z["leaf_cells"], meta={"cached": path})
        except Exception:
            pass
    t = make_tree(spec)
    os.makedirs(cache_dir, exist_ok=True)
    tmp = path + f".{os.getpid()}.tmp.npz"
    np.savez(tmp, depth=t.depth, sh_degree=t.sh_degree, l_max=t.l_max, child=t.child,
             sigma=t.sigma, sh=t.sh, leaf_cells=t.leaf_cells)
    os.replace(tmp, path)
    return t
