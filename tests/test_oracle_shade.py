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
