"""Pins of the distillation oracle (oracle/distill.py; Sec. 5, "Creating the
plenoctree")."""
import math

import numpy as np
import pytest

import inputs
from inputs.trees import field_params
from oracle import distill as od


def test_philox_known_answers():
    """Philox4x32-10 against the known-answer vectors published with the
    generator (counter, key -> output)."""
    cases = [
        ((0, 0, 0, 0), (0, 0), (0x6627E8D5, 0xE169C58D, 0xBC57AC4C, 0x9B00DBD8)),
        ((0xFFFFFFFF,) * 4, (0xFFFFFFFF,) * 2, (0x408F276D, 0x41C83B0E, 0xA20BC7C6, 0x6D5451FD)),
        ((0x243F6A88, 0x85A308D3, 0x13198A2E, 0x03707344), (0xA4093822, 0x299F31D0),
         (0xD16CFE09, 0x94FDCCEB, 0x5001E420, 0x24126EA1)),
    ]
    for c, k, want in cases:
        got = od.philox4x32_10(*[np.array([v], np.uint64) for v in c], *k)
        assert tuple(int(g[0]) for g in got) == want


def test_offsets_are_uniform_and_distinct():
    codes = np.array([0, 1, 12345, (1 << 27) + 5], np.uint64)
    u = od.unit_offsets(codes, 4096, seed=99)
    assert u.shape == (4, 4096, 3) and u.min() >= 0.0 and u.max() < 1.0
    # 24-bit dyadic values
    assert np.all(u * 2.0 ** 24 == np.floor(u * 2.0 ** 24))
    m = u.reshape(-1, 3).mean(0)
    assert np.all(np.abs(m - 0.5) < 5 * math.sqrt(1 / 12 / u[:, :, 0].size))
    assert not np.array_equal(u[0], u[1]) and not np.array_equal(u, od.unit_offsets(codes, 4096, seed=98))


def _one_blob(deg=2, shells=()):
    K = (deg + 1) ** 2
    hi = np.arange(3 * (K - 1), dtype=np.float64).reshape(1, 3, K - 1) * 0.1 - 0.5
    return od.Field(centres=np.array([[0.1, -0.2, 0.05]]), radii=np.array([0.3]), amps=np.array([8.0]),
                    emission=np.array([[5.0, 50.0, 500.0]]), hi=hi, shells=np.array(shells).reshape(-1, 4),
                    shell_half_width=0.02, log_base=math.log(1e-3), sigma_max=50.0, l_max=2048.0,
                    sh_degree=deg)


def test_field_closed_forms():
    f = _one_blob()
    # density at the blob centre and one radius away along x
    x = np.array([[0.1, -0.2, 0.05], [0.4, -0.2, 0.05]])
    s = od.density(f, x)
    assert s[0] == pytest.approx(min(math.exp(math.log(1e-3) + 8.0), 50.0), rel=1e-14)
    assert s[1] == pytest.approx(math.exp(math.log(1e-3) + 8.0 * math.exp(-0.5)), rel=1e-14)
    # one blob: the weights are 1 everywhere, the SH are its own, and the DC
    # term reproduces its radiance through Eq. 6's sigmoid
    c = od.sh_coefficients(f, np.random.default_rng(0).uniform(-1, 1, (100, 3)))
    for ch, e in enumerate((5.0, 50.0, 500.0)):
        assert np.allclose(2048.0 / (1 + np.exp(-c[:, ch, 0] * od.Y00)), e, rtol=1e-12)
        assert np.allclose(c[:, ch, 1:], f.hi[0, ch], rtol=0, atol=1e-15)
    # a shell overrides the density
    g = _one_blob(shells=[(0.0, 0.0, 0.0, 0.5)])
    pts = np.array([[0.5, 0, 0], [0.515, 0, 0], [0.53, 0, 0]])
    assert list(od.density(g, pts)[:2]) == [50.0, 50.0] and od.density(g, pts)[2] < 50.0


def test_two_blob_weights_are_a_softmax():
    f = _one_blob()
    f.centres = np.array([[-0.3, 0, 0], [0.3, 0, 0]])
    f.radii = np.array([0.2, 0.4])
    f.amps = np.array([3.0, 4.0])
    f.emission = np.array([[1.0, 2.0, 3.0], [30.0, 20.0, 10.0]])
    f.hi = np.stack([f.hi[0], -f.hi[0]])
    x = np.array([[0.05, 0.1, -0.2]])
    g = np.array([math.exp(-((0.35) ** 2 + 0.01 + 0.04) / (2 * 0.04)),
                  math.exp(-((0.25) ** 2 + 0.01 + 0.04) / (2 * 0.16))])
    w = g / g.sum()
    E = w @ f.emission
    c = od.sh_coefficients(f, x)[0]
    assert np.allclose(2048.0 / (1 + np.exp(-c[:, 0] * od.Y00)), E, rtol=1e-12)
    assert np.allclose(c[:, 1:], w[0] * f.hi[0] + w[1] * f.hi[1], rtol=1e-12, atol=1e-15)
    assert od.log_density_sum(f, x)[0] == pytest.approx(3.0 * g[0] + 4.0 * g[1], rel=1e-14)


def test_sample_mean_matches_the_voxel_integral():
    """The 256-sample mean of a voxel estimates the mean of the field over
    that voxel: against 6-point Gauss-Legendre quadrature per axis, within 5
    standard errors (a sample placed in the wrong voxel or along the wrong
    axis fails this)."""
    f = _one_blob()
    depth = 3
    h = 2.0 / 8
    codes = od.morton_encode(np.array([3, 4, 1]), np.array([2, 3, 6]), np.array([4, 3, 2]))
    sig, sh = od.average_samples(f, depth, codes, n_samples=256, seed=5)
    gx, gw = np.polynomial.legendre.leggauss(6)
    q = od.morton_decode(codes)
    for i in range(len(codes)):
        lo = -1.0 + q[i] * h
        pts = np.stack(np.meshgrid(*[lo[a] + (gx + 1) * h / 2 for a in range(3)], indexing="ij"), -1).reshape(-1, 3)
        wts = np.einsum("i,j,k->ijk", gw, gw, gw).ravel() / 8.0
        exact = (od.density(f, pts) * wts).sum()
        u = od.unit_offsets(codes[i:i + 1], 256, 5)[0]
        vals = od.density(f, lo + u * h)
        se = vals.std() / math.sqrt(256)
        assert abs(sig[i] - exact) <= 5 * se + 1e-12 * exact, (i, sig[i], exact, se)
        assert sig[i] == pytest.approx(vals.mean(), rel=1e-13)


def test_centre_sampling_reproduces_the_generator():
    """Steps (1), (2) and (4) alone are what the input generator does with
    its own (separable, libm) evaluation: the same occupied voxels and the
    same child table, for blob-and-shell fields at depths 4 and 5."""
    for depth, shells, seed in ((4, 0, 1), (5, 2, 3)):
        spec = inputs.TreeSpec(depth=depth, n_blobs=8, n_shells=shells, sh_degree=2, seed=seed, occupancy=0.3)
        f = od.field_from_params(field_params(spec))
        codes, amb = od.centre_occupancy(f, depth)
        tree = inputs.make_tree(spec)
        gen = np.sort(inputs.morton3(tree.leaf_cells[:, 0], tree.leaf_cells[:, 1], tree.leaf_cells[:, 2]))
        diff = np.setxor1d(gen, codes)
        assert np.all(np.isin(diff, amb)), diff
        if diff.size == 0:
            assert np.array_equal(od.build_octree(depth, codes), tree.child)


def test_octree_build_reaches_every_leaf():
    """Walking the child table from the root by the octant bits of a kept
    code reaches leaf i for the i-th code, every node is reached once, and no
    other cell of the grid reaches a leaf."""
    rng = np.random.default_rng(4)
    depth = 4
    codes = np.unique(rng.integers(0, 8 ** depth, 300).astype(np.uint64))
    child = od.build_octree(depth, codes)
    seen = set()
    for code in range(8 ** depth):
        node = 0
        leaf = None
        for lvl in range(depth):
            c = child[node, (code >> (3 * (depth - 1 - lvl))) & 7]
            if c == 0:
                break
            if c < 0:
                assert lvl == depth - 1
                leaf = -c - 1
                break
            seen.add(int(c))
            node = c
        if leaf is None:
            assert code not in set(codes.tolist())
        else:
            assert codes[leaf] == code
    assert seen == set(range(1, child.shape[0]))
