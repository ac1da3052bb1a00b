"""Pins of the proxy-irradiance oracle (oracle/shade.py) against what the
geometry fixes: Lambert's closed form for the projected solid angle of a
polygon, the transparency blend of Sec. 3 Eq. 2 at its two extremes (an
empty luminaire passes the background, an opaque one hides it), and the
cases that must give exactly zero."""
import math

import numpy as np
import pytest

import inputs
from oracle import core, shade

Y00 = 0.28209479177387814   # real SH basis, l = 0


def _lambert(x, n, poly):
    """Projected solid angle of a planar polygon wholly above the tangent
    plane of (x, n): half the sum over edges of the edge's subtended angle
    times the normal's component along the edge's plane normal (Lambert's
    contour formula)."""
    n = np.asarray(n, np.float64) / np.linalg.norm(n)
    tot = 0.0
    for i in range(len(poly)):
        a = poly[i] - x
        b = poly[(i + 1) % len(poly)] - x
        a /= np.linalg.norm(a)
        b /= np.linalg.norm(b)
        g = np.cross(a, b)
        gl = np.linalg.norm(g)
        tot += math.atan2(gl, float(a @ b)) * float(n @ g) / gl
    return abs(tot) / 2.0


def _box_projected_solid_angle(x, n):
    x = np.asarray(x, np.float64)
    tot = 0.0
    for axis in range(3):
        for s in (-1.0, 1.0):
            if s * x[axis] <= 1.0:
                continue                      # the face is not seen from the front
            j, k = (axis + 1) % 3, (axis + 2) % 3
            poly = []
            for (p, q) in ((-1, -1), (1, -1), (1, 1), (-1, 1)):
                v = np.zeros(3)
                v[axis], v[j], v[k] = s, p, q
                poly.append(v)
            tot += _lambert(x, n, np.array(poly))
    return tot


# points whose tangent plane leaves every box vertex in front of it
POSES = [((0.3, -0.2, -3.0), (0.0, 0.1, 1.0)),
         ((2.5, 1.7, 0.4), (-1.0, -0.5, 0.1)),
         ((-4.0, 3.0, 2.0), (4.0, -3.0, -2.0))]


def _check_vertices_in_front(x, n):
    v = np.array([[a, b, c] for a in (-1, 1) for b in (-1, 1) for c in (-1, 1)], np.float64)
    assert np.all((v - np.asarray(x)) @ np.asarray(n, np.float64) > 0)


def test_lambert_formula_against_quadrature():
    # the closed form against a midpoint quadrature of cos cos / r^2 over the
    # bottom face seen from straight below, and its far-field limit A / r^2
    for z in (-2.0, -5.0, -400.0):
        D = -z - 1.0
        got = _box_projected_solid_angle(np.array([0.0, 0.0, z]), (0, 0, 1))
        N = 1000
        s = (np.arange(N) + 0.5) / N * 2.0 - 1.0
        X, Y = np.meshgrid(s, s)
        quad = float((D * D / (X ** 2 + Y ** 2 + D * D) ** 2).sum()) * (2.0 / N) ** 2
        assert got == pytest.approx(quad, rel=1e-6)
    assert got == pytest.approx(4.0 / 399.0 ** 2, rel=1e-4)


@pytest.mark.parametrize("pose", range(len(POSES)))
def test_empty_luminaire_passes_the_background(pose):
    x, n = POSES[pose]
    _check_vertices_in_front(x, n)
    S = 200_000
    u = inputs.rays.sample_numbers(1, S, 40 + pose)
    B = np.array([0.5, 1.25, 2.0])
    r = shade.proxy_irradiance(inputs.empty_tree(3), np.array([x], np.float32),
                               np.array([n], np.float32), u, background=B)
    ref = _box_projected_solid_angle(x, n)
    se = r["terms"][0].std(axis=0) / math.sqrt(S)
    assert np.all(np.abs(r["E"][0] - B * ref) < 5 * se + 1e-12), (r["E"][0], B * ref, se)


@pytest.mark.parametrize("pose", range(len(POSES)))
def test_opaque_luminaire_hides_the_background(pose):
    x, n = POSES[pose]
    c = np.array([[-1.0], [0.5], [2.0]])
    tree = inputs.uniform_tree(2, 1e6, c)
    phi = inputs.L_MAX / (1.0 + np.exp(-c[:, 0].astype(np.float32).astype(np.float64) * Y00))
    S = 100_000
    u = inputs.rays.sample_numbers(1, S, 50 + pose)
    r = shade.proxy_irradiance(tree, np.array([x], np.float32), np.array([n], np.float32), u,
                               background=(100.0, 100.0, 100.0))
    ref = _box_projected_solid_angle(x, n)
    se = r["terms"][0].std(axis=0) / math.sqrt(S)
    assert np.all(np.abs(r["E"][0] - phi * ref) < 5 * se + 1e-9), (r["E"][0], phi * ref, se)


def test_terms_of_a_blend():
    # a half-transparent sample: L_o = L_e + (1 - alpha) B, term = w L_o
    tree = inputs.uniform_tree(2, 0.25, np.array([[0.3]] * 3))
    x = np.array([[0.2, 0.1, -2.5]], np.float32)
    n = np.array([[0.0, 0.0, 1.0]], np.float32)
    u = inputs.rays.sample_numbers(1, 64, 7)
    B = np.array([3.0, 0.0, 1.0])
    r = shade.proxy_irradiance(tree, x, n, u, background=B)
    o, d, w = shade.proxy_rays(x, n, u)
    q = core.query(tree, o, d)
    assert np.all(q["alpha"][w > 0] < 0.9) and np.all(q["alpha"][w > 0] > 0.0)
    want = w[:, None] * (q["L"] + (1.0 - q["alpha"])[:, None] * B[None, :])
    assert np.allclose(r["terms"][0], want, rtol=1e-15, atol=0)
    assert np.allclose(r["E"][0], want.mean(axis=0), rtol=1e-15, atol=0)


def test_zero_cases():
    tree = inputs.uniform_tree(2, 5.0, np.array([[0.3]] * 3))
    u = inputs.rays.sample_numbers(3, 256, 9)
    pts = np.array([[0.2, 0.1, 0.3],        # inside the proxy: nothing seen from the front
                    [0.0, 0.0, -3.0],       # normal facing away from the box
                    [0.0, 0.0, -3.0]], np.float32)
    nrm = np.array([[0.0, 0.0, 1.0], [0.0, 0.0, -1.0], [0.0, 0.0, 0.0]], np.float32)
    r = shade.proxy_irradiance(tree, pts, nrm, u, background=(1.0, 1.0, 1.0))
    assert np.all(r["E"] == 0.0) and np.all(r["w"] == 0.0)


def test_only_front_faces_carry_weight():
    # from below the box only the bottom face (axis 2, sign -1: f = 4) is seen
    x = np.array([[0.1, -0.3, -2.0]], np.float32)
    n = np.array([[0.0, 0.0, 1.0]], np.float32)
    u = inputs.rays.sample_numbers(1, 4096, 11)
    _, _, w = shade.proxy_rays(x, n, u)
    face = np.minimum((u[0, :, 0] * np.float32(6.0)).astype(np.int32), 5)
    assert np.all(w[face != 4] == 0.0) and np.all(w[face == 4] > 0.0)
    assert abs(np.mean(face == 4) - 1 / 6) < 0.03


# ---------------------------------------------------------------- guided sampling
G = 8


def _random_guide(seed, zeros=0.3):
    rng = np.random.default_rng(seed)
    w = rng.exponential(1.0, shade.guide_cells(G)).astype(np.float32)
    w[rng.random(w.size) < zeros] = 0.0
    return w


def test_uniform_guide_is_area_uniform():
    """With equal cell weights the guided density is uniform over the faces
    the point sees: from below, only the bottom face (area 4), so every
    sample's weight is cos cos / r^2 times 4, and no sample is dead."""
    x = np.array([[0.4, -0.3, -2.7]], np.float32)
    n = np.array([[0.1, 0.2, 1.0]], np.float32)
    u = inputs.rays.sample_numbers(1, 4096, 21)
    for beta in (0.0, 0.3, 1.0):
        o, d, w, cell = shade.guided_proxy_rays(x, n, u, np.ones(shade.guide_cells(G), np.float32), G, beta)
        live = w > 0
        d64 = d[live].astype(np.float64)
        r2 = (d64 ** 2).sum(1)
        nn = n[0].astype(np.float64)
        cos_x = d64 @ (nn / np.linalg.norm(nn)) / np.sqrt(r2)
        cos_y = (-x[0, 2].astype(np.float64) - 1.0) / np.sqrt(r2)     # bottom face (z = -1)
        assert live.all()
        assert np.allclose(w[live] * r2 / (cos_x * cos_y), 4.0, rtol=1e-9)


def _face_choice(x, n, P, vis):
    """Face probabilities from their definition: half in proportion to the
    guide mass, half to the guide mass times cos cos / r^2 at the face
    centre (r^4 in the denominator: cos_y = h / r, cos_x = n.d / (|n| r),
    and the constant 1 / |n| cancels)."""
    x = x.astype(np.float64)
    n = n.astype(np.float64)
    centres = np.array([[-1, 0, 0], [1, 0, 0], [0, -1, 0], [0, 1, 0], [0, 0, -1], [0, 0, 1]], np.float64)
    d = centres - x
    h = np.abs(x[np.arange(6) >> 1]) - 1.0
    g = np.clip(d @ n, 0.0, None) * h / np.einsum("ij,ij->i", d, d) ** 2
    Pv = np.where(vis, P, 0.0)
    if (Pv * g).sum() == 0:
        return Pv / Pv.sum()
    return 0.5 * Pv * g / (Pv * g).sum() + 0.5 * Pv / Pv.sum()


def test_cell_frequencies_follow_the_guide():
    """Cells of the faces the point sees are picked with probability
    Q_f p_k / P_f: faces by the mix of guide mass and face-centre geometry,
    cells within a face by p_k = (1 - beta) w_k / W + beta / n.  Counts
    within 5 standard deviations, none on the other faces; with beta = 0 a
    cell of weight 0 is never picked."""
    w = _random_guide(3)
    S = 200_000
    u = inputs.rays.sample_numbers(1, S, 22)
    # points that see three faces: x > 1, y < -1, z < -1 (faces 1, 2, 4),
    # the second with a normal that turns away from face 4's centre
    for x, n in ((np.array([[2.5, -3.0, -1.7]], np.float32), np.array([[-1.0, 1.0, 1.0]], np.float32)),
                 (np.array([[1.3, -2.2, -1.4]], np.float32), np.array([[0.0, -1.0, 3.0]], np.float32))):
        vis = shade.visible_faces(x)[0]
        assert list(np.nonzero(vis)[0]) == [1, 2, 4]
        for beta in (0.0, 0.25):
            _, _, _, cell = shade.guided_proxy_rays(x, n, u, w, G, beta)
            p, cdf = shade.guide_cdf(w, beta)
            assert cdf[-1] == pytest.approx(1.0, abs=1e-12)
            P = p.reshape(6, G * G).sum(1)
            Q = _face_choice(x[0], n[0], P, vis)
            q = np.repeat(np.where(P > 0, Q / np.where(P > 0, P, 1), 0.0), G * G) * p
            on = np.repeat(vis, G * G)
            assert q.sum() == pytest.approx(1.0, abs=1e-12)
            cnt = np.bincount(cell, minlength=p.size)
            sd = np.sqrt(S * q * (1 - q))
            assert np.all(np.abs(cnt - S * q) <= 5 * sd + 1e-9)
            assert np.all(cnt[~on] == 0)
            if beta == 0.0:
                assert np.all(cnt[w == 0] == 0)


def test_face_choice_keeps_a_defensive_share():
    """A visible face whose centre lies behind the point's tangent plane
    has geometry weight 0 yet keeps half its guide-mass share."""
    x = np.array([1.3, -2.2, -1.4], np.float32)
    n = np.array([0.0, -1.0, 3.0], np.float32)
    assert shade.face_geometry(x, n, 4) == 0.0 and shade.face_geometry(x, n, 2) > 0.0
    w = np.ones(shade.guide_cells(G), np.float32)
    _, cdf = shade.guide_cdf(w, 0.0)
    # face 4 is the last visible face: u0 just below 1 lands in it
    cell, _, factor = shade.guided_cell(cdf, G, x, n, np.float32(0.9999))
    assert cell // (G * G) == 4
    # P_f = 1/6 on every face, P_vis = 1/2: Q_4 = 0.5 (1/6) / (1/2) = 1/6
    assert factor == pytest.approx((1.0 / 6.0) / (1.0 / 6.0), rel=1e-12)


@pytest.mark.parametrize("pose", range(len(POSES)))
def test_guided_estimate_is_unbiased(pose):
    """The guided estimator against Lambert's closed form: an opaque uniform
    luminaire (E = Phi times the projected solid angle) and an empty one
    passing the background (E = L_b times it), with a guide that favours
    some cells and ignores others (defensive share 0.2), within 5 standard
    errors."""
    x, n = POSES[pose]
    ref = _box_projected_solid_angle(x, n)
    w = _random_guide(10 + pose)
    S = 100_000
    u = inputs.rays.sample_numbers(1, S, 60 + pose)
    c = np.array([[-1.0], [0.5], [2.0]])
    tree = inputs.uniform_tree(2, 1e6, c)
    phi = inputs.L_MAX / (1.0 + np.exp(-c[:, 0].astype(np.float32).astype(np.float64) * Y00))
    r = shade.proxy_irradiance_guided(tree, np.array([x], np.float32), np.array([n], np.float32), u, w, G, 0.2)
    se = r["terms"][0].std(axis=0) / math.sqrt(S)
    assert np.all(np.abs(r["E"][0] - phi * ref) < 5 * se + 1e-9), (r["E"][0], phi * ref, se)
    B = np.array([0.5, 1.25, 2.0])
    r = shade.proxy_irradiance_guided(inputs.empty_tree(3), np.array([x], np.float32), np.array([n], np.float32),
                                      u, w, G, 0.2, background=B)
    se = r["terms"][0].std(axis=0) / math.sqrt(S)
    assert np.all(np.abs(r["E"][0] - B * ref) < 5 * se + 1e-12), (r["E"][0], B * ref, se)


def test_invalid_weights_count_as_zero():
    """Negative, NaN and infinite weights take no share of the guide: the
    table equals the one with those weights set to 0, and a guide of only
    such weights is the uniform one."""
    w = _random_guide(5)
    bad = w.copy()
    k = np.flatnonzero(w > 0)[:4]
    bad[k] = [-1.0, np.nan, np.inf, -np.inf]
    ref = w.copy()
    ref[k] = 0.0
    for beta in (0.0, 0.3):
        p, cdf = shade.guide_cdf(bad, beta)
        p0, cdf0 = shade.guide_cdf(ref, beta)
        assert np.array_equal(p, p0) and np.array_equal(cdf, cdf0)
    p, _ = shade.guide_cdf(np.full(shade.guide_cells(G), np.nan, np.float32), 0.0)
    assert np.allclose(p, 1.0 / p.size)


def _bin_by_normalising(v, l2, D):
    """The tangent bin from its definition with the square root taken."""
    return np.clip(np.floor((v / np.sqrt(l2) + 1.0) * 0.5 * D), 0, D - 1).astype(np.int64)


def test_direction_bins():
    """Bins decided on squares against bins of the normalised component,
    away from the thresholds; thresholds that a direction meets exactly
    (components 1, 2, 2: 1/3 of its length) count as passed."""
    rng = np.random.default_rng(7)
    w = rng.normal(size=(20000, 3)).astype(np.float32).astype(np.float64)
    l2 = (w * w).sum(1)
    for D in (2, 3, 4):
        c = w[:, 0] / np.sqrt(l2)
        th = 2.0 * np.arange(1, D) / D - 1.0
        away = np.min(np.abs(c[:, None] - th[None, :]), axis=1) > 1e-9
        got = shade.direction_bin(w[:, 0], l2, D)
        assert np.array_equal(got[away], _bin_by_normalising(w[away, 0], l2[away], D))
    assert shade.direction_bin(0.0, 1.0, 2) == 1
    # one direction (plain floats) and arrays take the same decisions
    for D in (2, 3, 4):
        got = shade.direction_bin(w[:500, 1], l2[:500], D)
        assert all(shade.direction_bin(float(a), float(b), D) == g for a, b, g in zip(w[:500, 1], l2[:500], got))
    assert shade.direction_bin(1.0, 9.0, 3) == 2 and shade.direction_bin(-1.0, 9.0, 3) == 1
    # face 4 (z = -1): tangent axes x then y; (3, 0, -4) / 5 has x component 0.6
    assert shade.face_direction_bin(4, np.array([[3.0, 0.0, -4.0]]), 4)[0] == 3 * 4 + 2


def _random_directional_guide(seed, D):
    rng = np.random.default_rng(seed)
    w = rng.exponential(1.0, shade.guide_cells(G) * D * D).astype(np.float32)
    w[rng.random(w.size) < 0.3] = 0.0
    return w


def test_directional_cell_frequencies():
    """With D x D direction bins, cells are picked with probability
    Q_f p[b_f][k] / P_f, b_f the bin of the point's direction from face f's
    centre (computed here with the square root), Q_f as in the
    direction-averaged case from the bins' face masses."""
    D = 2
    w = _random_directional_guide(13, D)
    S = 100_000
    u = inputs.rays.sample_numbers(1, S, 27)
    x = np.array([[2.5, -3.0, -1.7]], np.float32)
    n = np.array([[-1.0, 1.0, 1.0]], np.float32)
    vis = shade.visible_faces(x)[0]
    centres = np.array([[-1, 0, 0], [1, 0, 0], [0, -1, 0], [0, 1, 0], [0, 0, -1], [0, 0, 1]], np.float64)
    for beta in (0.0, 0.25):
        _, _, _, cell = shade.guided_proxy_rays(x, n, u, w, G, beta, D)
        p, cdf = shade.guide_tables(w, beta, D)
        gg = G * G
        P = np.zeros(6)
        pk = np.zeros(p.shape[1])
        for f in np.nonzero(vis)[0]:
            a = f >> 1
            dvec = x[0].astype(np.float64) - centres[f]
            l2 = (dvec * dvec).sum()
            b = _bin_by_normalising(dvec[(a + 1) % 3], l2, D) * D + _bin_by_normalising(dvec[(a + 2) % 3], l2, D)
            P[f] = p[b, f * gg:(f + 1) * gg].sum()
            pk[f * gg:(f + 1) * gg] = p[b, f * gg:(f + 1) * gg]
        Q = _face_choice(x[0], n[0], P, vis)
        q = np.repeat(np.where(P > 0, Q / np.where(P > 0, P, 1), 0.0), gg) * pk
        assert q.sum() == pytest.approx(1.0, abs=1e-12)
        cnt = np.bincount(cell, minlength=q.size)
        sd = np.sqrt(S * q * (1 - q))
        assert np.all(np.abs(cnt - S * q) <= 5 * sd + 1e-9)


@pytest.mark.parametrize("pose", range(len(POSES)))
def test_directional_guided_estimate_is_unbiased(pose):
    """The estimator with a 3 x 3 directional guide against Lambert's closed
    form for an opaque uniform luminaire, within 5 standard errors."""
    D = 3
    x, n = POSES[pose]
    ref = _box_projected_solid_angle(x, n)
    w = _random_directional_guide(30 + pose, D)
    S = 100_000
    u = inputs.rays.sample_numbers(1, S, 70 + pose)
    c = np.array([[-1.0], [0.5], [2.0]])
    tree = inputs.uniform_tree(2, 1e6, c)
    phi = inputs.L_MAX / (1.0 + np.exp(-c[:, 0].astype(np.float32).astype(np.float64) * Y00))
    r = shade.proxy_irradiance_guided(tree, np.array([x], np.float32), np.array([n], np.float32), u, w, G, 0.2,
                                      D=D)
    se = r["terms"][0].std(axis=0) / math.sqrt(S)
    assert np.all(np.abs(r["E"][0] - phi * ref) < 5 * se + 1e-9), (r["E"][0], phi * ref, se)


def test_directional_guide_of_an_opaque_uniform_luminaire():
    """Every probe of an opaque uniform luminaire sees Phi, so every
    (cell, direction bin) weight is Phi's luminance, including bins no
    probe fell in (they take the cell's mean)."""
    c = np.array([[-1.0], [0.5], [2.0]])
    tree = inputs.uniform_tree(2, 1e6, c)
    phi = inputs.L_MAX / (1.0 + np.exp(-c[:, 0].astype(np.float32).astype(np.float64) * Y00))
    u = inputs.rays.probe_numbers(shade.guide_cells(4), 8, 25)
    wts, _ = shade.guide_weights(tree, 4, u, D=3)
    assert wts.shape == (shade.guide_cells(4) * 9,)
    assert np.allclose(wts, phi.mean(), rtol=1e-9)


def test_guide_of_an_opaque_uniform_luminaire():
    """Every probe of an opaque uniform luminaire sees its emission Phi, so
    every cell's guide weight is Phi's luminance (channel mean)."""
    c = np.array([[-1.0], [0.5], [2.0]])
    tree = inputs.uniform_tree(2, 1e6, c)
    phi = inputs.L_MAX / (1.0 + np.exp(-c[:, 0].astype(np.float32).astype(np.float64) * Y00))
    u = inputs.rays.probe_numbers(shade.guide_cells(4), 8, 23)
    wts, _ = shade.guide_weights(tree, 4, u)
    assert np.allclose(wts, phi.mean(), rtol=1e-9)
    # and of an empty one: all zero, so the guided density falls back to uniform
    wts, _ = shade.guide_weights(inputs.empty_tree(3), 4, u)
    p, _ = shade.guide_cdf(wts, 0.0)
    assert np.all(wts == 0.0) and np.allclose(p, 1.0 / p.size)


def test_guide_probes_start_on_their_cell():
    u = inputs.rays.probe_numbers(shade.guide_cells(2), 3, 24)
    o, d = shade.guide_probe_rays(2, u)
    for c in range(shade.guide_cells(2)):
        face, ca, cb = c // 4, (c // 2) % 2, c % 2
        axis, sgn = face >> 1, (1.0 if face & 1 else -1.0)
        pts = o[3 * c: 3 * c + 3]
        assert np.all(pts[:, axis] == sgn)
        a, b = pts[:, (axis + 1) % 3], pts[:, (axis + 2) % 3]
        assert np.all((a >= -1 + ca) & (a <= ca)) and np.all((b >= -1 + cb) & (b <= cb))
        # the probes aim into the box
        assert np.all(d[3 * c: 3 * c + 3, axis] * sgn < 0)
