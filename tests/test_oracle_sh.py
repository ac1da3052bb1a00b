"""Pins for the oracle's spherical harmonics (Sec. 4.2, Eq. 6)."""
import math
import os

import numpy as np
import pytest
import scipy.special as sps

from oracle import core

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "real_sh_table.txt")


def _golden_rows():
    rows = []
    for line in open(GOLDEN):
        line = line.strip()
        if not line or line.startswith("#"):
            continue
        l, m, const, poly = line.split()
        rows.append((int(l), int(m), const, poly))
    return rows


def _unit_dirs(n, seed):
    v = np.random.default_rng(seed).normal(size=(n, 3))
    return v / np.linalg.norm(v, axis=1, keepdims=True)


def test_golden_cartesian_table():
    env = {"sqrt": math.sqrt, "pi": math.pi}
    for w in _unit_dirs(50, 1):
        Y = core.sh_eval(3, w)
        x, y, z = w
        for l, m, const, poly in _golden_rows():
            ref = eval(const, {"__builtins__": {}}, env) * eval(
                poly, {"__builtins__": {}}, {"x": x, "y": y, "z": z})
            assert Y[l * l + l + m] == pytest.approx(ref, rel=1e-12, abs=1e-14)


def test_against_scipy_complex_harmonics():
    # scipy's Y_l^m carries the Condon-Shortley phase (-1)^m; strip it
    for w in _unit_dirs(30, 2):
        th, ph = math.acos(max(-1.0, min(1.0, w[2]))), math.atan2(w[1], w[0])
        Y = core.sh_eval(4, w)
        for l in range(5):
            for m in range(-l, l + 1):
                c = sps.sph_harm_y(l, abs(m), th, ph)
                if m == 0:
                    ref = c.real
                elif m > 0:
                    ref = math.sqrt(2) * (-1) ** m * c.real
                else:
                    ref = math.sqrt(2) * (-1) ** m * c.imag
                assert Y[l * l + l + m] == pytest.approx(ref, rel=1e-11, abs=1e-13)


def test_orthonormality_by_quadrature():
    # Gauss-Legendre in cos(theta) x uniform phi is exact for these degrees
    deg = 4
    K = (deg + 1) ** 2
    xs, ws = np.polynomial.legendre.leggauss(12)
    nphi = 24
    G = np.zeros((K, K))
    for x, wq in zip(xs, ws):
        s = math.sqrt(1 - x * x)
        for j in range(nphi):
            ph = 2 * math.pi * j / nphi
            Y = core.sh_eval(deg, [s * math.cos(ph), s * math.sin(ph), x])
            G += wq * (2 * math.pi / nphi) * np.outer(Y, Y)
    assert np.abs(G - np.eye(K)).max() < 1e-12


def test_addition_theorem_and_parity():
    for w in _unit_dirs(40, 3):
        Y = core.sh_eval(4, w)
        Yn = core.sh_eval(4, -w)
        for l in range(5):
            band = Y[l * l: (l + 1) ** 2]
            assert (band ** 2).sum() == pytest.approx((2 * l + 1) / (4 * math.pi), rel=1e-12)
            assert np.allclose(Yn[l * l: (l + 1) ** 2], (-1) ** l * band, rtol=0, atol=1e-14)


def test_degree_zero_is_direction_independent():
    vals = {core.sh_eval(0, w)[0] for w in _unit_dirs(20, 4)}
    assert len(vals) == 1 and vals.pop() == pytest.approx(0.5 / math.sqrt(math.pi), rel=1e-15)
