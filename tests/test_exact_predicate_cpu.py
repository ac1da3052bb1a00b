"""The traversal's exact decision (march.h exact_cross_sign, built for the
host with ROCm's clang++): the sign of (Pa - oa) db - (Pb - ob) da for finite float32
operands, against rational arithmetic (fractions.Fraction) on random
operands over the whole float32 range, subnormals and zeros, exact ties
and ties moved by one unit in the last place."""
import os
import subprocess
from fractions import Fraction

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2207_05009_amd", "csrc")

PROGRAM = r"""
#include "march.h"
#include <cstdio>
#include <cstring>
int main() {
    unsigned b[6];
    while (std::scanf("%x %x %x %x %x %x", b, b + 1, b + 2, b + 3, b + 4, b + 5) == 6) {
        float f[6];
        std::memcpy(f, b, sizeof f);
        std::printf("%d\n", lq::exact_cross_sign(f[0], f[1], f[2], f[3], f[4], f[5]));
    }
    return 0;
}
"""


def _exact(v):
    Pa, oa, da, Pb, ob, db = (Fraction(float(x)) for x in v)
    s = (Pa - oa) * db - (Pb - ob) * da
    return (s > 0) - (s < 0)


def _finite_bits(rng, n, lo_exp=0, hi_exp=254):
    sign = rng.integers(0, 2, n, dtype=np.uint32) << 31
    e = rng.integers(lo_exp, hi_exp + 1, n, dtype=np.uint32) << 23
    m = rng.integers(0, 1 << 23, n, dtype=np.uint32)
    return (sign | e | m).view(np.float32)


def _cases():
    rng = np.random.default_rng(2022)
    out = []
    # random operands over the whole range (subnormals included), and over
    # narrow exponent windows where cancellation is likely
    out.append(_finite_bits(rng, 6 * 6000).reshape(-1, 6))
    for lo, hi in ((120, 134), (0, 3), (100, 160), (60, 70)):
        out.append(_finite_bits(rng, 6 * 3000, lo, hi).reshape(-1, 6))
    # planes and origins as in the query (|P| <= 1 on a grid, origins near
    # the box), directions of any size
    n = 6000
    P = (rng.integers(-512, 513, (n, 2)) / 512.0).astype(np.float32)
    o = rng.uniform(-3, 3, (n, 2)).astype(np.float32)
    d = _finite_bits(rng, 2 * n, 60, 190).reshape(n, 2)
    out.append(np.stack([P[:, 0], o[:, 0], d[:, 0], P[:, 1], o[:, 1], d[:, 1]], 1))
    # exact ties: (Pa - oa) db == (Pb - ob) da with small-integer operands
    # scaled by powers of two, then each operand moved by one ulp
    n = 3000
    k = rng.integers(-40, 41, (n, 4)).astype(np.float64)
    sc = np.ldexp(1.0, rng.integers(-60, 61, n))
    Pa, oa = k[:, 0] * sc, k[:, 1] * sc
    Pb = k[:, 2] * sc
    ra = Pa - oa
    da = rng.integers(1, 64, n) * np.ldexp(1.0, rng.integers(-70, 71, n))
    da *= np.where(rng.integers(0, 2, n) == 1, 1.0, -1.0)
    # Pb - ob = 2 (Pa - oa) and db = 2 da: (Pa - oa) db = (Pb - ob) da
    ob = Pb - ra * 2.0
    db = da * 2.0
    ties = np.stack([Pa, oa, da, Pb, ob, db], 1).astype(np.float32)
    ok = np.all(np.isfinite(ties), 1) & (ties[:, 2] != 0) & (ties[:, 5] != 0)
    ties = ties[ok]
    out.append(ties)
    for j in range(6):
        t = ties.copy()
        t[:, j] = np.nextafter(t[:, j], np.float32(np.inf))
        out.append(t)
        t = ties.copy()
        t[:, j] = np.nextafter(t[:, j], np.float32(-np.inf))
        out.append(t)
    # zeros and extremes
    ext = np.array([0.0, -0.0, 1.0, -1.0, 2.0 ** -149, -(2.0 ** -149), 2.0 ** -126, 3.4028235e38, -3.4028235e38,
                    2.0 ** 127, 1.5, 0.1], np.float32)
    idx = rng.integers(0, len(ext), (4000, 6))
    out.append(ext[idx])
    c = np.concatenate(out).astype(np.float32)
    c = c[np.all(np.isfinite(c), 1) & (c[:, 2] != 0) & (c[:, 5] != 0)]
    return c


def test_exact_cross_sign_against_rationals(tmp_path):
    cxx = "/opt/rocm/llvm/bin/clang++"        # the storage types need _Float16 on the host
    if not os.path.exists(cxx) or not os.path.isdir("/opt/rocm/include"):
        pytest.skip("needs ROCm's clang++ and headers")
    src = tmp_path / "pred.cpp"
    src.write_text(PROGRAM)
    exe = tmp_path / "pred"
    subprocess.run([cxx, "-std=c++17", "-O2", "-ffp-contract=off", "-D__HIP_PLATFORM_AMD__",
                    "-I/opt/rocm/include", f"-I{CSRC}", "-o", str(exe), str(src)], check=True)
    cases = _cases()
    text = "\n".join(" ".join(f"{x:08x}" for x in row) for row in cases.view(np.uint32))
    r = subprocess.run([str(exe)], input=text, capture_output=True, text=True, timeout=120, check=True)
    got = np.array([int(x) for x in r.stdout.split()])
    assert len(got) == len(cases)
    want = np.array([_exact(row) for row in cases])
    bad = np.nonzero(got != want)[0]
    assert bad.size == 0, [(cases[i].tolist(), int(got[i]), int(want[i])) for i in bad[:5]]
    # the ties and their one-ulp neighbours exercise every sign
    assert (want == 0).sum() > 1000 and (want > 0).sum() > 1000 and (want < 0).sum() > 1000
