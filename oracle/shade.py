"""FP64 oracle of the consumer side of the emission query (test
infrastructure only: tests/, the smoke check and the benchmark's CPU leg use
it; the GPU library never does).

Irradiance at a shading point x with normal n from the light that leaves the
luminaire's proxy box toward x.  The radiance leaving the proxy along a ray
is the luminaire's emission plus the scene light seen through it, weighted
by the ray's transparency (Sec. 3, Eq. 2): L_o = L_e + (1 - alpha) L_b,
where alpha is the opacity the query returns (Sec. 4.1, Eq. 5) and L_b the
radiance behind the luminaire (here one constant colour).  The proxy is
sampled uniformly over its surface (Sec. 6, Sampling): the box [-1,1]^3 has
six faces of area 4, so a sample picks face f = floor(6 u0) and the point
(2 u1 - 1, 2 u2 - 1) on it, with area density p_A = 1/24.  A sample on a
face that x does not see from the front, or below x's tangent plane,
contributes 0; otherwise its Monte Carlo term is

    L_o(x <- y) cos(theta_x) cos(theta_y) / (|y - x|^2 p_A),

and the estimate is the mean of the terms over a point's samples.  Every
direction toward the box meets exactly one front-facing face point, so the
estimate is unbiased for the irradiance (the integral of L_o cos(theta_x)
over the box's solid angle).  A Lambertian surface of albedo rho then
reflects rho / pi times it.

The sample ray is built in float32 with the operations the definition
lists (the query's inputs are float32): y as above, d = y - x per
component; the weight and the sum are FP64.
"""
from __future__ import annotations

import math

import numpy as np

from . import core

P_AREA = 1.0 / 24.0


def proxy_rays(points, normals, u):
    """Rays and weights of the samples.  points, normals: [n, 3]; u: [n, S, 3]
    in [0, 1).  Returns o, d (float32 [n S, 3]) and w (float64 [n S]); the
    direction of a zero-weight sample is zeroed (the query returns 0 for it)."""
    x = np.ascontiguousarray(points, np.float32).reshape(-1, 3)
    nrm = np.asarray(normals, np.float64).reshape(-1, 3)
    u = np.ascontiguousarray(u, np.float32)
    n, S = u.shape[0], u.shape[1]
    u = u.reshape(n * S, 3)
    f = np.clip((u[:, 0] * np.float32(6.0)).astype(np.int32), 0, 5)
    axis = f >> 1
    sgn = np.where(f & 1, np.float32(1.0), np.float32(-1.0)).astype(np.float32)
    a = u[:, 1] * np.float32(2.0) - np.float32(1.0)
    b = u[:, 2] * np.float32(2.0) - np.float32(1.0)
    y = np.empty((n * S, 3), np.float32)
    rows = np.arange(n * S)
    y[rows, axis] = sgn
    y[rows, (axis + 1) % 3] = a
    y[rows, (axis + 2) % 3] = b
    xs = np.repeat(x, S, axis=0)
    d = (y - xs).astype(np.float32)
    # weights in FP64 from the float32 geometry
    d64 = d.astype(np.float64)
    dist2 = np.einsum("ij,ij->i", d64, d64)
    dist = np.sqrt(dist2)
    ns = np.repeat(nrm, S, axis=0)
    nlen = np.linalg.norm(ns, axis=1)
    cos_x = np.einsum("ij,ij->i", ns, d64) / np.where(nlen * dist > 0, nlen * dist, 1.0)
    h = sgn.astype(np.float64) * xs.astype(np.float64)[rows, axis] - 1.0   # x in front of the face plane
    cos_y = h / np.where(dist > 0, dist, 1.0)
    ok = (h > 0) & (cos_x > 0) & (dist2 > 0) & (nlen > 0)
    w = np.where(ok, cos_x * cos_y / np.where(dist2 > 0, dist2, 1.0) / P_AREA, 0.0)
    d[~ok] = 0.0
    return xs, d, w


def proxy_irradiance(tree, points, normals, u, background=(0.0, 0.0, 0.0), model: int = core.LINEAR,
                     storage: str = "f32") -> dict:
    """Irradiance estimate per point (E [n, 3]) and the Monte Carlo terms
    (terms [n, S, 3]); terms_alt uses the query's alternative candidate
    where the oracle marks a ray threshold-ambiguous (alt_valid)."""
    u = np.asarray(u, np.float32)
    n, S = u.shape[0], u.shape[1]
    o, d, w = proxy_rays(points, normals, u)
    q = core.query(tree, o, d, model=model, storage=storage)
    B = np.asarray(background, np.float64)[None, :]
    lo = q["L"] + (1.0 - q["alpha"])[:, None] * B
    lo_alt = q["alt_L"] + (1.0 - q["alt_alpha"])[:, None] * B
    terms = (w[:, None] * lo).reshape(n, S, 3)
    terms_alt = (w[:, None] * lo_alt).reshape(n, S, 3)
    return {"E": terms.mean(axis=1), "terms": terms, "terms_alt": terms_alt,
            "alt_valid": q["alt_valid"].reshape(n, S).astype(bool), "w": w.reshape(n, S)}


# ---------------------------------------------------------------- guided sampling
# Importance sampling of the proxy according to the radiance field (the
# paper's stated future work, Sec. 6 "Sampling" and Sec. 7 "Limitations --
# Sampling"; the design below is this project's).  The proxy surface is cut
# into 6 G^2 cells (face f, then G x G cells on it along the face's next two
# axes in cyclic order).  The guide weight of a cell is the mean luminance
# (channel mean) of the emission the query returns for probe rays that start
# at uniform points of the cell and aim at uniform points inside the box.
# The cells have the probabilities
#     p_k = (1 - beta) w_k / sum_i w_i + beta / (6 G^2)
# (the defensive share beta keeps every cell reachable: the light behind
# the luminaire also passes where it emits nothing).  A shading point x only
# receives light through the faces it sees from the front (sgn x_axis > 1);
# the others contribute exactly zero, so a sample of x picks among the cells
# of those faces only: a face by its guide mass mixed with the irradiance
# integrand at its centre (guided_cell), a cell of it in proportion to p_k,
# and a uniform point in the cell.  The estimate is unbiased whenever every
# cell of a visible face has p_k > 0 (beta > 0 ensures it).
# With D > 1 direction bins the guide is directional: each probe also falls
# in one of D x D bins of its outward direction (the light it measures
# leaves the cell along -d) on the face's two tangent axes, a cell has one
# weight per bin, and each bin its own table; a shading point uses, on
# every face it sees, the bin of its own direction from the face's centre
# (face f's table is cdf[b_f(x)]).

def guide_cells(G):
    return 6 * G * G


def _cell_point(cell, ua, ub, G):
    """Face point of (cell, ua, ub) in float32 with the operations the
    definition lists; returns (y [m, 3] float32, face, axis, sign)."""
    cell = np.asarray(cell, np.int64)
    face = cell // (G * G)
    ca = (cell // G) % G
    cb = cell % G
    axis = face >> 1
    sgn = np.where(face & 1, np.float32(1.0), np.float32(-1.0)).astype(np.float32)
    step = np.float32(2.0 / G)
    a = (ca.astype(np.float32) + ua.astype(np.float32)) * step - np.float32(1.0)
    b = (cb.astype(np.float32) + ub.astype(np.float32)) * step - np.float32(1.0)
    y = np.empty((cell.size, 3), np.float32)
    rows = np.arange(cell.size)
    y[rows, axis] = sgn
    y[rows, (axis + 1) % 3] = a
    y[rows, (axis + 2) % 3] = b
    return y, face, axis, sgn


def guide_probe_rays(G, u_probe):
    """Probe rays of the guide: u_probe [6 G^2, R, 5] in [0, 1): a point of
    the cell (two numbers) and a target inside the box (three); the ray
    starts on the face and points at the target (float32, d = t - y)."""
    u = np.ascontiguousarray(u_probe, np.float32)
    n_cells, R = u.shape[0], u.shape[1]
    cell = np.repeat(np.arange(n_cells), R)
    uu = u.reshape(-1, 5)
    y, _, _, _ = _cell_point(cell, uu[:, 0], uu[:, 1], G)
    t = uu[:, 2:5] * np.float32(2.0) - np.float32(1.0)
    d = (t - y).astype(np.float32)
    return y, d


def direction_bin(v, l2, D):
    """Tangent bin 0..D-1 of a direction whose component on a tangent axis
    is v and whose squared length is l2: the number of thresholds
    theta_j = 2 j / D - 1 (j = 1..D-1) with v / sqrt(l2) >= theta_j, decided
    on squares (FP64) so that no square root enters the decision.  v and l2
    are FP64 arrays (or scalars)."""
    if isinstance(v, float) and isinstance(l2, float):   # one direction: plain floats, the same operations
        i = 0
        for j in range(1, D):
            th = (2.0 * j) / D - 1.0
            if th < 0.0:
                ok = v >= 0.0 or v * v <= (th * th) * l2
            elif th == 0.0:
                ok = v >= 0.0
            else:
                ok = v >= 0.0 and v * v >= (th * th) * l2
            i = j if ok else i
        return i
    v = np.asarray(v, np.float64)
    l2 = np.asarray(l2, np.float64)
    i = np.zeros(np.broadcast(v, l2).shape, np.int64)
    for j in range(1, D):
        th = (2.0 * j) / D - 1.0
        if th < 0.0:
            ok = (v >= 0.0) | (v * v <= (th * th) * l2)
        elif th == 0.0:
            ok = v >= 0.0
        else:
            ok = (v >= 0.0) & (v * v >= (th * th) * l2)
        i = np.where(ok, j, i)
    return i


def face_direction_bin(face, w, D):
    """Bin i1 D + i2 of an outward direction w [m, 3] (FP64 values) through
    face `face`: i1, i2 the tangent bins of its components on the face's
    next two axes (cyclic); the squared length summed in axis order."""
    w = np.asarray(w, np.float64).reshape(-1, 3)
    face = np.broadcast_to(np.asarray(face, np.int64), (w.shape[0],))
    a = face >> 1
    rows = np.arange(w.shape[0])
    l2 = w[:, 0] * w[:, 0] + w[:, 1] * w[:, 1] + w[:, 2] * w[:, 2]
    return direction_bin(w[rows, (a + 1) % 3], l2, D) * D + direction_bin(w[rows, (a + 2) % 3], l2, D)


def guide_weights(tree, G, u_probe, model: int = core.LINEAR, storage: str = "f32", D: int = 1):
    """Guide weights [6 G^2 * D^2], cell-major: the mean probe luminance of
    each cell (D = 1), or per direction bin of the probes' outward
    direction -d (FP64 sums in probe order; a bin no probe of the cell fell
    in takes the cell's mean over all its probes); and the oracle's query
    output on the probes (for candidate checks)."""
    o, d = guide_probe_rays(G, u_probe)
    q = core.query(tree, o, d, model=model, storage=storage)
    R = np.asarray(u_probe).shape[1]
    n = guide_cells(G)
    lum = q["L"].mean(1)
    if D == 1:
        return lum.reshape(-1, R).mean(1), q
    cell = np.repeat(np.arange(n), R)
    b = face_direction_bin(cell // (G * G), -d.astype(np.float64), D)
    s = np.zeros((n, D * D))
    c = np.zeros((n, D * D))
    np.add.at(s, (cell, b), lum)
    np.add.at(c, (cell, b), 1.0)
    tot = np.zeros(n)
    np.add.at(tot, cell, lum)
    w = np.where(c > 0, s / np.where(c > 0, c, 1.0), (tot / R)[:, None])
    return w.reshape(-1), q


def guide_cdf(weights, beta):
    """Cell probabilities and their cumulative sums in FP64, summed in cell
    order: W = w_0 + w_1 + ..., p_k = (1 - beta) (w_k / W) + beta / n (all
    1 / n when W = 0), cdf[0] = 0, cdf[k + 1] = cdf[k] + p_k.  A weight
    that is negative, NaN or infinite counts as 0."""
    w = [float(v) if (v > 0 and math.isfinite(v)) else 0.0 for v in np.asarray(weights, np.float32)]
    n = len(w)
    W = 0.0
    for v in w:
        W += v
    if W > 0.0:
        p = [(1.0 - beta) * (v / W) + beta / n for v in w]
    else:
        p = [1.0 / n] * n
    cdf = [0.0] * (n + 1)
    for k in range(n):
        cdf[k + 1] = cdf[k] + p[k]
    return np.array(p), np.array(cdf)


def guide_tables(weights, beta, D):
    """One table per direction bin: (p [D^2, n], cdf [D^2, n + 1]), bin b
    from the weights w[k D^2 + b] by guide_cdf."""
    w = np.asarray(weights, np.float32).reshape(-1, D * D)
    pc = [guide_cdf(w[:, b], beta) for b in range(D * D)]
    return np.array([x[0] for x in pc]), np.array([x[1] for x in pc])


def visible_faces(x):
    """[n, 6] bool: the faces x sees from the front (face f: axis f >> 1,
    side -1 for even f, +1 for odd; visible iff side * x_axis > 1)."""
    x = np.asarray(x, np.float32).reshape(-1, 3)
    out = np.zeros((x.shape[0], 6), bool)
    for f in range(6):
        sgn = np.float32(1.0) if f & 1 else np.float32(-1.0)
        out[:, f] = sgn * x[:, f >> 1] > np.float32(1.0)
    return out


FACE_MIX = 0.5   # share of the face choice weighted by the face-centre geometry


def face_geometry(x, n, f):
    """Geometry weight of face f for a point x with normal n, at the face's
    centre c (c_a = side, the other coordinates 0): max(0, n.(c - x)) (side
    x_a - 1) / |c - x|^4, the irradiance integrand cos(theta_x)
    cos(theta_y) / r^2 there up to the point's constant factor 1 / |n|.
    FP64 from the float32 inputs, each sum in axis order."""
    a, sgn = f >> 1, (1.0 if f & 1 else -1.0)
    xd = [float(v) for v in np.asarray(x, np.float32)]
    nd = [float(v) for v in np.asarray(n, np.float32)]
    d = [(sgn if b == a else 0.0) - xd[b] for b in range(3)]
    r2 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2]
    ndot = nd[0] * d[0] + nd[1] * d[1] + nd[2] * d[2]
    h = sgn * xd[a] - 1.0
    return (ndot * h) / (r2 * r2) if ndot > 0.0 else 0.0


def guided_cell(cdf, G, x, n, u0, D=1):
    """The cell a sample picks.  cdf [D^2, 6 G^2 + 1]: the tables of the
    direction bins (guide_tables).  The point sees faces vis (side
    x_axis > 1); on face f it uses table b_f, the bin of its direction
    x - c_f from the face's centre (face_direction_bin), with guide mass
    P_f = cdf[b_f][(f + 1) G^2] - cdf[b_f][f G^2]; P_vis is their sum over
    the visible faces, g_f = face_geometry and S = sum of P_f g_f.  Face f
    is chosen with probability
        Q_f = FACE_MIX P_f g_f / S + (1 - FACE_MIX) P_f / P_vis
    (P_f / P_vis when S = 0): t = u0 walks the visible faces in order, and
    in the face where t < Q_f (the last visible face takes any remainder)
    the cell is the largest k of the face with
    cdf[b_f][k] <= cdf[b_f][f G^2] + r P_f, r = t / Q_f (0 when Q_f = 0).
    Returns (cell, b_f, Q_f / P_f): the cell's area density is
    p[b_f][k] (Q_f / P_f) / A_cell.  Cell -1 when no face is visible or
    P_vis = 0."""
    gg = G * G
    cdf = np.asarray(cdf).reshape(D * D, -1)
    xs = np.asarray(x, np.float32)
    vis = visible_faces(xs)[0]
    xd = xs.astype(np.float64)
    bins = [0] * 6
    P = [0.0] * 6
    pv = 0.0
    gs = 0.0
    g = [0.0] * 6
    for f in range(6):
        if vis[f]:
            a, sgn = f >> 1, (1.0 if f & 1 else -1.0)
            w = [float(xd[k]) - (sgn if k == a else 0.0) for k in range(3)]
            l2 = w[0] * w[0] + w[1] * w[1] + w[2] * w[2]
            bins[f] = direction_bin(w[(a + 1) % 3], l2, D) * D + direction_bin(w[(a + 2) % 3], l2, D)
            c = cdf[bins[f]]
            P[f] = c[(f + 1) * gg] - c[f * gg]
            g[f] = face_geometry(xs, n, f)
            pv += P[f]
            gs += P[f] * g[f]
    if not pv > 0.0:
        return -1, 0, 0.0
    Q = [0.0] * 6
    for f in range(6):
        if vis[f]:
            Q[f] = FACE_MIX * (P[f] * g[f] / gs) + (1.0 - FACE_MIX) * (P[f] / pv) if gs > 0.0 else P[f] / pv
    t = float(np.float32(u0))
    last = max(f for f in range(6) if vis[f])
    for f in range(6):
        if not vis[f]:
            continue
        if t < Q[f] or f == last:
            c = cdf[bins[f]]
            r = t / Q[f] if Q[f] > 0.0 else 0.0
            target = c[f * gg] + r * P[f]
            lo, hi = f * gg, f * gg + gg - 1
            while lo < hi:
                mid = (lo + hi + 1) // 2
                if c[mid] <= target:
                    lo = mid
                else:
                    hi = mid - 1
            return lo, bins[f], (Q[f] / P[f] if P[f] > 0.0 else 0.0)
        t -= Q[f]
    return -1, 0, 0.0


def guided_proxy_rays(points, normals, u, weights, G, beta, D=1):
    """Rays and weights of guided samples: u [n, S, 3]: u0 picks the cell
    among the faces the point sees (guided_cell), u1, u2 the point in it.
    weights [6 G^2 D^2], cell-major.  The Monte Carlo weight is
    cos(theta_x) cos(theta_y) / (|y - x|^2 p_A) with
    p_A = p[b_f][k] (Q_f / P_f) / A_cell; zero below the horizon, and for a
    point that sees no face."""
    x = np.ascontiguousarray(points, np.float32).reshape(-1, 3)
    nrm32 = np.asarray(normals, np.float32).reshape(-1, 3)
    nrm = nrm32.astype(np.float64)
    u = np.ascontiguousarray(u, np.float32)
    n, S = u.shape[0], u.shape[1]
    u = u.reshape(n * S, 3)
    p, cdf = guide_tables(weights, beta, D)
    cell = np.empty(n * S, np.int64)
    cbin = np.zeros(n * S, np.int64)
    factor = np.zeros(n * S)
    for i in range(n):
        for j in range(S):
            cell[i * S + j], cbin[i * S + j], factor[i * S + j] = guided_cell(cdf, G, x[i], nrm32[i],
                                                                              u[i * S + j, 0], D)
    dead = cell < 0
    cell = np.where(dead, 0, cell)
    y, face, axis, sgn = _cell_point(cell, u[:, 1], u[:, 2], G)
    rows = np.arange(n * S)
    xs = np.repeat(x, S, axis=0)
    d = (y - xs).astype(np.float32)
    d64 = d.astype(np.float64)
    dist2 = np.einsum("ij,ij->i", d64, d64)
    dist = np.sqrt(dist2)
    ns = np.repeat(nrm, S, axis=0)
    nlen = np.linalg.norm(ns, axis=1)
    cos_x = np.einsum("ij,ij->i", ns, d64) / np.where(nlen * dist > 0, nlen * dist, 1.0)
    h = sgn.astype(np.float64) * xs.astype(np.float64)[rows, axis] - 1.0
    cos_y = h / np.where(dist > 0, dist, 1.0)
    area = (2.0 / G) ** 2
    pa = np.where(dead, 0.0, p[cbin, cell] * factor / area)
    ok = (h > 0) & (cos_x > 0) & (dist2 > 0) & (nlen > 0) & (pa > 0)
    w = np.where(ok, cos_x * cos_y / np.where(dist2 > 0, dist2, 1.0) / np.where(pa > 0, pa, 1.0), 0.0)
    d[~ok] = 0.0
    return xs, d, w, cell


def proxy_irradiance_guided(tree, points, normals, u, weights, G, beta, background=(0.0, 0.0, 0.0),
                            model: int = core.LINEAR, storage: str = "f32", D: int = 1) -> dict:
    """The guided estimate per point (E [n, 3]) and its terms, as
    proxy_irradiance does for uniform sampling."""
    u = np.asarray(u, np.float32)
    n, S = u.shape[0], u.shape[1]
    o, d, w, cell = guided_proxy_rays(points, normals, u, weights, G, beta, D)
    q = core.query(tree, o, d, model=model, storage=storage)
    B = np.asarray(background, np.float64)[None, :]
    lo = q["L"] + (1.0 - q["alpha"])[:, None] * B
    lo_alt = q["alt_L"] + (1.0 - q["alt_alpha"])[:, None] * B
    terms = (w[:, None] * lo).reshape(n, S, 3)
    terms_alt = (w[:, None] * lo_alt).reshape(n, S, 3)
    return {"E": terms.mean(axis=1), "terms": terms, "terms_alt": terms_alt,
            "alt_valid": q["alt_valid"].reshape(n, S).astype(bool), "w": w.reshape(n, S),
            "cell": cell.reshape(n, S)}
