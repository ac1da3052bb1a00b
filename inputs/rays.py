"""Seeded synthetic ray batches (input data only).

Every generator returns (origins, dirs) as contiguous float32 [n, 3] arrays.
Directions are normalised in float64 and then rounded to float32; the float32
arrays are the canonical inputs for both the oracle and the GPU library.
Rays point *into* the luminaire: d goes from the shading point toward the
proxy (the paper's emission direction is omega = -d/|d|).
"""
from __future__ import annotations

import math

import numpy as np


def _norm_f32(v: np.ndarray) -> np.ndarray:
    n = np.sqrt((v * v).sum(axis=1, keepdims=True))
    return np.ascontiguousarray((v / n).astype(np.float32))


def _uniform_sphere(rng, n):
    v = rng.normal(size=(n, 3))
    return v / np.sqrt((v * v).sum(axis=1, keepdims=True))


def sphere_to_cube(n: int, seed: int, radius: float = 3.0):
    """Origins uniform on the sphere |o| = radius, aimed at points uniform in
    the proxy cube [-1, 1]^3 (the small configuration)."""
    rng = np.random.default_rng(seed)
    o = _uniform_sphere(rng, n) * radius
    tgt = rng.uniform(-1.0, 1.0, size=(n, 3))
    o32 = np.ascontiguousarray(o.astype(np.float32))
    return o32, _norm_f32(tgt - o32.astype(np.float64))


def camera_eye(dist: float = 3.0) -> np.ndarray:
    th, ph = math.radians(60.0), math.radians(30.0)
    return dist * np.array([math.sin(th) * math.cos(ph), math.sin(th) * math.sin(ph), math.cos(th)])


def pinhole(width: int = 2048, height: int = 2048, fov_deg: float = 40.0,
            dist: float = 3.0, rows: slice | None = None):
    """Pinhole camera looking at the origin from a generic pose (no exactly
    axis-parallel rays); up +z, vertical field of view fov_deg, pixel centres.
    Ray order is row-major (j outer, i inner)."""
    eye = camera_eye(dist)
    fwd = -eye / np.linalg.norm(eye)
    right = np.cross(fwd, np.array([0.0, 0.0, 1.0]))
    right /= np.linalg.norm(right)
    up = np.cross(right, fwd)
    tan_h = math.tan(math.radians(fov_deg) / 2.0)
    aspect = width / height
    j0, j1 = (0, height) if rows is None else (rows.start, rows.stop)
    jj, ii = np.meshgrid(np.arange(j0, j1, dtype=np.float64),
                         np.arange(width, dtype=np.float64), indexing="ij")
    sx = (2.0 * (ii + 0.5) / width - 1.0) * tan_h * aspect
    sy = (1.0 - 2.0 * (jj + 0.5) / height) * tan_h
    d = fwd[None, :] + sx.reshape(-1, 1) * right[None, :] + sy.reshape(-1, 1) * up[None, :]
    o = np.broadcast_to(eye.astype(np.float32), d.shape)
    return np.ascontiguousarray(o), _norm_f32(d)


def room_to_proxy(n: int, seed: int, half=(5.0, 5.0, 1.5)):
    """Incoherent shading queries: origins uniform in the room box
    [-5,5]x[-5,5]x[-1.5,1.5] outside the proxy cube, aimed at points uniform
    on the cube's surface."""
    rng = np.random.default_rng(seed)
    hx = np.asarray(half, dtype=np.float64)
    o = np.empty((n, 3))
    filled = 0
    while filled < n:
        m = int((n - filled) * 1.1) + 16
        cand = rng.uniform(-1.0, 1.0, size=(m, 3)) * hx
        inside = np.all(np.abs(cand) <= 1.0, axis=1)
        cand = cand[~inside][: n - filled]
        o[filled: filled + len(cand)] = cand
        filled += len(cand)
    face = rng.integers(0, 6, size=n)
    uv = rng.uniform(-1.0, 1.0, size=(n, 2))
    tgt = np.empty((n, 3))
    ax = face % 3
    sgn = np.where(face < 3, 1.0, -1.0)
    for a in range(3):
        sel = ax == a
        others = [b for b in range(3) if b != a]
        tgt[sel, a] = sgn[sel]
        tgt[sel, others[0]] = uv[sel, 0]
        tgt[sel, others[1]] = uv[sel, 1]
    o32 = np.ascontiguousarray(o.astype(np.float32))
    return o32, _norm_f32(tgt - o32.astype(np.float64))


def adversarial(depth: int, seed: int, n: int = 512):
    """Degenerate rays for traversal tests: axis-parallel rays (also along
    cell faces and edges), rays through grid vertices and edges, rays lying in
    face planes, +-0 direction components, origins on the proxy faces and
    inside the proxy, rays that miss or graze the proxy, and very short and
    very long direction vectors."""
    rng = np.random.default_rng(seed)
    N = 1 << depth
    h = 2.0 / N
    plane = lambda k: -1.0 + k * h
    O, D = [], []

    def add(o, d):
        O.append(np.asarray(o, dtype=np.float64))
        D.append(np.asarray(d, dtype=np.float64))

    for _ in range(n // 8):
        # axis-parallel along a face/edge line or cell interior
        a = rng.integers(0, 3)
        s = rng.choice([-1.0, 1.0])
        o = np.zeros(3)
        for b in range(3):
            if b == a:
                o[b] = -3.0 * s
            else:
                o[b] = plane(rng.integers(0, N + 1)) if rng.random() < 0.7 else rng.uniform(-1.2, 1.2)
        d = np.zeros(3)
        d[a] = s
        if rng.random() < 0.3:
            d[(a + 1) % 3] = -0.0
        add(o, d)
        # through two grid vertices (diagonal-ish), exact integer steps
        p0 = np.array([plane(rng.integers(0, N + 1)) for _ in range(3)])
        step = rng.integers(-3, 4, size=3).astype(np.float64) * h
        if not np.any(step):
            step[0] = h
        add(p0 - 4.0 * step, step)
        # in a face plane, crossing edges
        a = rng.integers(0, 3)
        o = rng.uniform(-2.5, 2.5, size=3)
        o[a] = plane(rng.integers(0, N + 1))
        d = rng.normal(size=3)
        d[a] = 0.0
        add(o, d)
        # origin on a proxy face pointing inward / outward
        o = rng.uniform(-1.0, 1.0, size=3)
        a = rng.integers(0, 3)
        o[a] = rng.choice([-1.0, 1.0])
        add(o, rng.normal(size=3))
        # origin inside the proxy
        add(rng.uniform(-0.99, 0.99, size=3), rng.normal(size=3))
        # miss / graze: aimed at the cube's edges and corners from outside
        corner = rng.choice([-1.0, 1.0], size=3)
        if rng.random() < 0.5:
            corner[rng.integers(0, 3)] = plane(rng.integers(0, N + 1))
        o = corner + rng.normal(size=3) * 2.0
        add(o, corner - o)
        # tiny and huge direction vectors (power-of-two scaled)
        d = rng.normal(size=3)
        add(rng.normal(size=3) * 3.0, d * 2.0 ** rng.integers(-60, 60))
        # rays from a vertex along a diagonal
        p0 = np.array([plane(rng.integers(0, N + 1)) for _ in range(3)])
        d = rng.choice([-1.0, 1.0], size=3)
        add(p0 - 3.0 * d, d)
    o = np.ascontiguousarray(np.array(O, dtype=np.float32))
    d = np.ascontiguousarray(np.array(D, dtype=np.float32))
    return o, d


def floor_points(nx: int, ny: int, z: float = -1.5, half: float = 5.0):
    """Shading points on the floor of the room around the luminaire: an
    nx x ny grid of cell centres on [-half, half]^2 at height z, normal +z
    (row-major, x fastest)."""
    xs = (np.arange(nx, dtype=np.float64) + 0.5) / nx * 2.0 * half - half
    ys = (np.arange(ny, dtype=np.float64) + 0.5) / ny * 2.0 * half - half
    yy, xx = np.meshgrid(ys, xs, indexing="ij")
    p = np.stack([xx.ravel(), yy.ravel(), np.full(nx * ny, z)], axis=1).astype(np.float32)
    nrm = np.zeros_like(p)
    nrm[:, 2] = 1.0
    return np.ascontiguousarray(p), nrm


def scattered_points(n: int, seed: int, radius=(1.2, 6.0)):
    """Shading points outside the proxy box, at distances in `radius` from
    the origin in uniform directions, each with a normal toward the origin
    tilted by up to ~35 degrees (some samples then fall below the tangent
    plane)."""
    rng = np.random.default_rng(seed)
    p = _uniform_sphere(rng, n) * rng.uniform(radius[0], radius[1], size=(n, 1))
    out = np.abs(p).max(axis=1) <= 1.05             # keep every point outside the box
    p[out] *= 1.2 / np.abs(p[out]).max(axis=1, keepdims=True)
    nrm = -p / np.linalg.norm(p, axis=1, keepdims=True) + rng.normal(0, 0.35, size=(n, 3))
    return p.astype(np.float32), nrm.astype(np.float32)


def sample_numbers(n: int, samples: int, seed: int):
    """Uniform numbers in [0, 1) for the proxy samples, [n, samples, 3] float32."""
    rng = np.random.default_rng(seed)
    return rng.random((n, samples, 3), dtype=np.float32)


def probe_numbers(n_cells: int, probes: int, seed: int):
    """Uniform numbers in [0, 1) for the guide's probe rays, [n_cells,
    probes, 5] float32 (a point of the cell, a target in the box)."""
    rng = np.random.default_rng(seed)
    return rng.random((n_cells, probes, 5), dtype=np.float32)


def guide_weights(n_cells: int, seed: int, zero_fraction: float = 0.3):
    """Synthetic guide weights for the proxy's cells: exponential values with
    a share of exact zeros, float32."""
    rng = np.random.default_rng(seed)
    w = rng.exponential(1.0, n_cells).astype(np.float32)
    w[rng.random(n_cells) < zero_fraction] = 0.0
    return w
