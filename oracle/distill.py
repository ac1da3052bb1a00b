"""FP64 oracle of the plenoctree distillation (test infrastructure only).

Only tests/, the smoke check and the benchmark's CPU leg use this module;
the GPU library never imports it.

Sec. 5, "Creating the plenoctree": the octree is extracted from a
continuous radiance field by (1) one density sample at the centre of every
voxel of the finest grid, (2) pruning the voxels whose centre density is
below 0.01, (3) averaging, for each voxel kept, the density and the SH
coefficients of 256 further samples at uniformly random positions inside the
voxel (against aliasing at discontinuities), and an octree over the kept
voxels whose empty octants collapse bottom-up.

The continuous field stands in for the trained network (no dataset or
trained model is available): a sum of Gaussian blobs in log-density plus
thin spherical shells of constant density,

    sigma(x) = sigma_max                              if | |x - s_j| - R_j | < w for a shell j
             = min(exp(ln_base + sum_k a_k g_k(x)), sigma_max)   otherwise,
    g_k(x)   = exp(-|x - c_k|^2 / (2 r_k^2)),

and SH emission coefficients blended by the normalised blob weights
w_k(x) = g_k(x) / sum_j g_j(x) (a softmax of -|x - c_k|^2 / (2 r_k^2)):

    E_c(x)     = sum_k w_k(x) e_kc                 (e_kc: blob k's radiance, channel c)
    coef_c0(x) = logit(E_c(x) / L_max) / Y_00,     Y_00 = 1 / (2 sqrt(pi))
    coef_cj(x) = sum_k w_k(x) h_kcj                 (j >= 1: SH index l^2 + l + m)

so that L_max sigmoid(coef_c0 Y_00) = E_c at every point (Sec. 4.2, Eq. 6).

Random positions: Philox4x32-10 (Salmon, Moraes, Dror and Shaw, "Parallel
random numbers: as easy as 1, 2, 3", SC 2011), counter (Morton code of the
voxel, sample index, 0, 0), key (seed low, seed high 32 bits); the first
three output words u give the offsets (u >> 8) 2^-24 in [0, 1) along x, y,
z.  The GPU library implements the same published generator on its side.

Occupancy is decided in FP64; a voxel whose centre value lies within a
relative 1e-9 of the threshold (or of a shell's boundary) is reported as
ambiguous: either decision is valid there.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

M0, M1 = 0xD2511F53, 0xCD9E8D57
W0, W1 = 0x9E3779B9, 0xBB67AE85
MASK32 = np.uint64(0xFFFFFFFF)
AMBIGUOUS_REL = 1e-9
Y00 = 0.5 / math.sqrt(math.pi)


# ---------------------------------------------------------------- Philox
def philox4x32_10(c0, c1, c2, c3, k0, k1):
    """Philox4x32 with 10 rounds on arrays of 32-bit counters (uint64 arrays
    holding 32-bit values) and a 32-bit key pair.  Returns four arrays."""
    c = [np.asarray(v, dtype=np.uint64) & MASK32 for v in (c0, c1, c2, c3)]
    k0, k1 = np.uint64(int(k0) & 0xFFFFFFFF), np.uint64(int(k1) & 0xFFFFFFFF)
    m0, m1 = np.uint64(M0), np.uint64(M1)
    for _ in range(10):
        p0 = c[0] * m0                 # < 2^64: exact in uint64
        p1 = c[2] * m1
        hi0, lo0 = p0 >> np.uint64(32), p0 & MASK32
        hi1, lo1 = p1 >> np.uint64(32), p1 & MASK32
        c = [(hi1 ^ c[1] ^ k0) & MASK32, lo1, (hi0 ^ c[3] ^ k1) & MASK32, lo0]
        k0 = (k0 + np.uint64(W0)) & MASK32
        k1 = (k1 + np.uint64(W1)) & MASK32
    return c


def unit_offsets(codes, n_samples, seed):
    """[n_voxels, n_samples, 3] offsets in [0, 1) of the sample positions."""
    codes = np.asarray(codes, dtype=np.uint64)
    j = np.arange(n_samples, dtype=np.uint64)
    c0 = np.repeat(codes, n_samples)
    c1 = np.tile(j, codes.size)
    z = np.zeros_like(c0)
    u = philox4x32_10(c0, c1, z, z, seed & 0xFFFFFFFF, seed >> 32)
    out = np.stack([(u[a] >> np.uint64(8)).astype(np.float64) * 2.0 ** -24 for a in range(3)], axis=-1)
    return out.reshape(codes.size, n_samples, 3)


# ---------------------------------------------------------------- field
@dataclass
class Field:
    centres: np.ndarray        # [nb, 3]
    radii: np.ndarray          # [nb]
    amps: np.ndarray           # [nb]
    emission: np.ndarray       # [nb, 3]  e_kc
    hi: np.ndarray             # [nb, 3, K - 1]
    shells: np.ndarray         # [ns, 4]  centre, radius
    shell_half_width: float
    log_base: float
    sigma_max: float
    l_max: float
    sh_degree: int

    @property
    def K(self) -> int:
        return (self.sh_degree + 1) ** 2


def _blob_terms(f: Field, x):
    """-|x - c_k|^2 / (2 r_k^2) for every point and blob: [n, nb]."""
    d2 = ((x[:, None, :] - f.centres[None, :, :]) ** 2).sum(-1)
    return -d2 / (2.0 * f.radii[None, :] ** 2)


def _in_shell(f: Field, x):
    """(inside any shell [n] bool, distance of | |x - s| - R | to w [n]
    for the nearest shell boundary, for the ambiguity test)."""
    inside = np.zeros(x.shape[0], bool)
    margin = np.full(x.shape[0], np.inf)
    for (sx, sy, sz, R) in f.shells:
        dist = np.sqrt(((x - np.array([sx, sy, sz])) ** 2).sum(-1))
        e = np.abs(dist - R)
        inside |= e < f.shell_half_width
        margin = np.minimum(margin, np.abs(e - f.shell_half_width))
    return inside, margin


def log_density_sum(f: Field, x):
    """S(x) = sum_k a_k g_k(x) (the log-density above ln_base)."""
    return (f.amps[None, :] * np.exp(_blob_terms(f, x))).sum(1)


def density(f: Field, x):
    inside, _ = _in_shell(f, x)
    s = np.minimum(np.exp(f.log_base + log_density_sum(f, x)), f.sigma_max)
    return np.where(inside, f.sigma_max, s)


def sh_coefficients(f: Field, x):
    """[n, 3, K] SH coefficients of the emission at x."""
    lw = _blob_terms(f, x)
    lw = lw - lw.max(1, keepdims=True)
    w = np.exp(lw)
    w /= w.sum(1, keepdims=True)
    E = w @ f.emission                                   # [n, 3]
    frac = E / f.l_max
    out = np.zeros((x.shape[0], 3, f.K))
    out[:, :, 0] = (np.log(frac) - np.log1p(-frac)) / Y00
    if f.K > 1:
        out[:, :, 1:] = np.einsum("nk,kcj->ncj", w, f.hi)
    return out


# ---------------------------------------------------------------- Morton
def morton_decode(codes):
    codes = np.asarray(codes, dtype=np.uint64)
    xyz = []
    for a in range(3):
        v = np.zeros(codes.shape, np.int64)
        for b in range(10):
            v |= ((codes >> np.uint64(3 * b + a)) & np.uint64(1)).astype(np.int64) << b
        xyz.append(v)
    return np.stack(xyz, axis=-1)


def morton_encode(x, y, z):
    m = np.zeros(np.shape(x), np.uint64)
    for b in range(10):
        for a, v in enumerate((x, y, z)):
            m |= ((np.asarray(v, np.uint64) >> np.uint64(b)) & np.uint64(1)) << np.uint64(3 * b + a)
    return m


# ---------------------------------------------------------------- steps
def centre_decisions(f: Field, depth: int, codes, prune_sigma: float = 0.01):
    """Step (1) for the given voxels (Morton codes): whether each is kept
    (centre density >= prune_sigma, or inside a shell), and whether the
    decision is ambiguous (either decision valid), as centre_occupancy
    decides them."""
    codes = np.asarray(codes, dtype=np.uint64)
    thr = math.log(prune_sigma) - f.log_base
    kept, near = _centre_decide(f, depth, thr, codes)
    return kept, near


def _centre_decide(f, depth, thr, codes):
    h = 2.0 / (1 << depth)
    q = morton_decode(codes)
    x = -1.0 + (q + 0.5) * h
    S = log_density_sum(f, x)
    inside, margin = _in_shell(f, x)
    keep = inside | (S >= thr)
    near = (np.abs(S - thr) <= AMBIGUOUS_REL * max(1.0, abs(thr))) & ~inside
    near |= margin <= AMBIGUOUS_REL * (1.0 + f.shell_half_width)
    return keep, near


def _centre_chunk(args):
    f, depth, thr, a, b = args
    codes = np.arange(a, b, dtype=np.uint64)
    keep, near = _centre_decide(f, depth, thr, codes)
    return codes[keep], codes[near]


def centre_occupancy(f: Field, depth: int, prune_sigma: float = 0.01, chunk: int = 1 << 21, workers: int = 1):
    """Step (1)-(2): Morton codes (ascending) of the voxels whose centre
    density is >= prune_sigma, and the codes of the ambiguous voxels (either
    decision valid).  workers > 1 spreads the chunks of voxels over
    processes (the same computation per voxel)."""
    thr = math.log(prune_sigma) - f.log_base
    total = (1 << depth) ** 3
    jobs = [(f, depth, thr, a, min(total, a + chunk)) for a in range(0, total, chunk)]
    if workers > 1 and len(jobs) > 1:
        from concurrent.futures import ProcessPoolExecutor
        with ProcessPoolExecutor(workers) as ex:
            parts = list(ex.map(_centre_chunk, jobs))
    else:
        parts = [_centre_chunk(j) for j in jobs]
    return np.concatenate([p[0] for p in parts]), np.concatenate([p[1] for p in parts])


def average_samples(f: Field, depth: int, codes, n_samples: int = 256, seed: int = 0,
                    chunk_samples: int = 1 << 20):
    """Step (3): per voxel, the mean density and mean SH coefficients of
    n_samples uniform positions inside it.  Returns (sigma [n], sh [n, 3, K])."""
    codes = np.asarray(codes, dtype=np.uint64)
    n = 1 << depth
    h = 2.0 / n
    q = morton_decode(codes)
    sig = np.zeros(codes.size)
    sh = np.zeros((codes.size, 3, f.K))
    per = max(1, chunk_samples // n_samples)
    for a in range(0, codes.size, per):
        b = min(codes.size, a + per)
        u = unit_offsets(codes[a:b], n_samples, seed)            # [m, S, 3]
        x = -1.0 + (q[a:b, None, :] + u) * h
        x = x.reshape(-1, 3)
        sig[a:b] = density(f, x).reshape(b - a, n_samples).mean(1)
        sh[a:b] = sh_coefficients(f, x).reshape(b - a, n_samples, 3, f.K).mean(1)
    return sig, sh


def build_octree(depth: int, codes):
    """Step (4), bottom-up collapse: the nodes of level l are the distinct
    prefixes (code >> 3 (depth - l)) of the kept voxels; the root is level 0.
    Child table [n_nodes, 8] int32: > 0 node index, < 0 -(leaf + 1), 0
    empty; nodes breadth-first, Morton order within a level; leaf i is the
    i-th kept code in ascending order."""
    codes = np.unique(np.asarray(codes, dtype=np.uint64))
    levels = {depth: codes}
    for lvl in range(depth - 1, -1, -1):
        levels[lvl] = np.unique(levels[lvl + 1] >> np.uint64(3))
    levels[0] = np.zeros(1, np.uint64)
    base, acc = {}, 0
    for lvl in range(depth):
        base[lvl] = acc
        acc += levels[lvl].size
    child = np.zeros((acc, 8), np.int32)
    for lvl in range(depth):
        kids = levels[lvl + 1]
        if kids.size == 0:
            continue
        p = np.searchsorted(levels[lvl], kids >> np.uint64(3))       # parent's position in its level
        i = np.arange(kids.size, dtype=np.int64)
        val = base[lvl + 1] + i if lvl + 1 < depth else -(i + 1)
        child[base[lvl] + p, (kids & np.uint64(7)).astype(np.int64)] = val
    return child


def field_from_params(p: dict) -> Field:
    return Field(centres=np.asarray(p["centres"], np.float64), radii=np.asarray(p["radii"], np.float64),
                 amps=np.asarray(p["amps"], np.float64), emission=np.asarray(p["emission"], np.float64),
                 hi=np.asarray(p["hi"], np.float64), shells=np.asarray(p["shells"], np.float64).reshape(-1, 4),
                 shell_half_width=float(p["shell_half_width"]), log_base=float(p["log_base"]),
                 sigma_max=float(p["sigma_max"]), l_max=float(p["l_max"]), sh_degree=int(p["sh_degree"]))


def distill(f: Field, depth: int, prune_sigma: float = 0.01, n_samples: int = 256, seed: int = 0):
    """The whole extraction: (codes, ambiguous codes, child table, sigma, sh)."""
    codes, amb = centre_occupancy(f, depth, prune_sigma)
    sig, sh = average_samples(f, depth, codes, n_samples, seed)
    return codes, amb, build_octree(depth, codes), sig, sh
