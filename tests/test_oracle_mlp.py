"""Pins for the surrogate oracle (oracle/mlp.py)."""
import math

import numpy as np
import pytest

from oracle import mlp


def _batch(n, seed):
    rng = np.random.default_rng(seed)
    o = rng.normal(size=(n, 3))
    o = 3.0 * o / np.linalg.norm(o, axis=1, keepdims=True)
    d = rng.uniform(-0.8, 0.8, size=(n, 3)) - o
    target = np.exp(rng.uniform(-3, 4, size=(n, 3)))
    return o, d, target


def test_sphere_parameterisation():
    o, d, _ = _batch(200, 1)
    x6, hit = mlp.sphere_param(o, d)
    assert hit.all()
    e = x6[:, :3] * math.sqrt(3.0)
    dn = d / np.linalg.norm(d, axis=1, keepdims=True)
    assert np.allclose((e * e).sum(1), 3.0, rtol=1e-12)
    # e lies on the line and is the nearer of the two hits along d
    w = e - o
    cross = np.cross(w, dn)
    assert np.abs(cross).max() < 1e-12
    other = e + 2.0 * (-(e * dn).sum(1))[:, None] * dn     # reflect to the far hit
    assert np.all(((other - o) * dn).sum(1) > ((e - o) * dn).sum(1))
    assert np.allclose(x6[:, 3:], dn)
    # a line through the centre enters at -sqrt(3) d_hat; a line that misses
    x6, hit = mlp.sphere_param(np.array([[0, 0, 5.0], [5, 5, 5.0]]), np.array([[0, 0, -2.0], [1, 0, 0.0]]))
    assert hit[0] and not hit[1]
    assert np.allclose(x6[0, :3] * math.sqrt(3), [0, 0, math.sqrt(3)])
    assert np.all(x6[1] == 0)


def test_fourier_features_at_special_points():
    x6 = np.array([[0.0, 0.5, -0.5, 1.0, 0.25, -1.0]])
    F = mlp.features(x6)[0]
    assert F.shape == (128,) and F[126] == 0 and F[127] == 0
    for v, x in enumerate(x6[0]):
        b = v * 21
        assert F[b] == x
        for k in range(10):
            assert F[b + 1 + 2 * k] == pytest.approx(math.sin(2 ** k * math.pi * x), abs=1e-12)
            assert F[b + 2 + 2 * k] == pytest.approx(math.cos(2 ** k * math.pi * x), abs=1e-12)
    # x = 0: raw 0, every sine 0, every cosine 1
    assert np.all(F[1:21:2] == 0) and np.all(F[2:21:2] == 1)
    # x = 0.5: sin(pi/2) = 1, cos(pi/2) = 0, then sin(k pi) = 0, cos = +-1
    assert F[21 + 1] == pytest.approx(1.0) and abs(F[21 + 2]) < 1e-15
    assert F[21 + 4] == pytest.approx(-1.0)


def test_parameter_count():
    assert mlp.n_params() == 20931


def test_loss_by_hand():
    # one sample, zero weights: y = b5, so L_hat = exp(b5) - 0.01
    theta = np.zeros(mlp.n_params())
    theta[-3:] = np.log([1.01, 2.01, 4.01])
    F = np.zeros((1, 128))
    target = np.array([[2.0, 2.0, 2.0]])
    loss, _ = mlp.loss_and_grad(theta, F, target, np.array([True]))
    Lh = np.array([1.0, 2.0, 4.0])
    den = Lh.mean() + 0.01
    assert loss == pytest.approx(((Lh - 2.0) ** 2).sum() / den ** 2, rel=1e-12)
    # an inactive sample contributes nothing but still counts in the batch size
    loss2, _ = mlp.loss_and_grad(theta, np.zeros((2, 128)), np.vstack([target, target]),
                                 np.array([True, False]))
    assert loss2 == pytest.approx(loss / 2, rel=1e-12)


def test_gradient_matches_central_differences():
    rng = np.random.default_rng(3)
    theta = mlp.he_uniform(7) * 0.7
    theta[-3:] = 0.3
    o, d, target = _batch(6, 4)
    x6, hit = mlp.sphere_param(o, d)
    F = mlp.features(x6)
    _, g = mlp.loss_and_grad(theta, F, target, hit)
    # the luminance denominator is a constant of the gradient: hold it fixed
    y0, _ = mlp.forward(theta, F)
    den0 = (np.exp(y0) - mlp.EPS_OUT).mean(1) + mlp.LOSS_EPS

    def loss_fixed(th):
        y, _ = mlp.forward(th, F)
        diff = np.exp(y) - mlp.EPS_OUT - target
        return ((diff * diff).sum(1) / den0 ** 2 * hit).sum() / F.shape[0]

    def masks(th):
        _, (hs, zs, _, _) = mlp.forward(th, F)
        return [z > 0 for z in zs[:-1]]

    idx = rng.choice(mlp.n_params(), 300, replace=False)
    idx = np.concatenate([idx, np.arange(mlp.n_params() - 195, mlp.n_params())])
    h = 1e-5
    # cancellation noise of a central difference in FP64: ~ eps * |loss| / h
    noise = 8 * np.finfo(float).eps * max(1.0, abs(loss_fixed(theta))) / h
    checked = 0
    for i in idx:
        tp, tm = theta.copy(), theta.copy()
        tp[i] += h
        tm[i] -= h
        # a ReLU switching inside the stencil has no two-sided derivative
        if any((a != b).any() for a, b in zip(masks(tp), masks(tm))):
            continue
        checked += 1
        fd = (loss_fixed(tp) - loss_fixed(tm)) / (2 * h)
        assert g[i] == pytest.approx(fd, rel=1e-6, abs=noise), i
    assert checked > 400


def test_bfloat16_mirror_stays_within_rounding_error():
    """With every GEMM input rounded to bfloat16 (weights, activations and
    output gradients), the gradient stays within the rounding error of the
    exact one: 8 significant bits per operand, so a few per cent per element
    at most and a direction that barely moves."""
    theta = mlp.he_uniform(9) * 0.7
    theta[-3:] = 0.3
    o, d, target = _batch(512, 5)
    x6, hit = mlp.sphere_param(o, d)
    F = mlp.features(x6)
    _, g = mlp.loss_and_grad(theta, F, target, hit)
    _, gr = mlp.loss_and_grad(theta, F, target, hit, round_bf16=mlp.bf16)
    cos = g @ gr / (np.linalg.norm(g) * np.linalg.norm(gr))
    rel = np.linalg.norm(gr - g) / np.linalg.norm(g)
    assert cos > 0.99 and 1e-4 < rel < 0.1
    # rounding only a GEMM input that is already a bfloat16 value changes nothing
    assert np.array_equal(mlp.bf16(mlp.bf16(F)), mlp.bf16(F))


def test_adam_first_steps_closed_form():
    g = np.array([0.3, -2.0, 1e-3, -5e-5])
    theta = np.zeros(4)
    m = np.zeros(4)
    v = np.zeros(4)
    lr = 1e-3
    # bias-corrected moments of a constant gradient are g and g^2: each step
    # moves by lr * g / (|g| + eps), i.e. lr * sign(g) up to eps
    for step in (1, 2, 3):
        theta, m, v = mlp.adam_step(theta, g, m, v, step, lr)
        expect = -step * lr * g / (np.abs(g) + 1e-8)
        assert np.allclose(theta, expect, rtol=1e-12, atol=1e-18)


def test_learning_rate_schedule():
    assert mlp.lr_at(0, 20000) == pytest.approx(5e-4)
    assert mlp.lr_at(20000, 20000) == pytest.approx(5e-6)
    assert mlp.lr_at(10000, 20000) == pytest.approx(math.sqrt(5e-4 * 5e-6))


def test_route_against_box_chords():
    """The hybrid's routing rule against the box geometry: a ray routed to
    the network sees the whole chord its line cuts from the box (the slab
    interval of the line lies at t >= 0); a ray routed to zero sees none of
    it (the octree of a box full of emitting density returns exactly 0)."""
    import inputs
    from oracle import core
    rng = np.random.default_rng(5)
    n = 4000
    # origins around and inside the box and the sphere, toward the box or away
    o = rng.uniform(-3, 3, size=(n, 3))
    tgt = rng.uniform(-1.2, 1.2, size=(n, 3))
    d = (tgt - o) * np.where(rng.random(n) < 0.4, -1.0, 1.0)[:, None]
    o, d = o.astype(np.float32), d.astype(np.float32)
    r = mlp.route(o, d)
    assert set(np.unique(r)) == {mlp.ROUTE_NET, mlp.ROUTE_OCTREE, mlp.ROUTE_ZERO}
    od, dd = o.astype(np.float64), d.astype(np.float64)
    with np.errstate(divide="ignore", invalid="ignore"):
        t0, t1 = (-1 - od) / dd, (1 - od) / dd
    tin = np.nanmax(np.minimum(t0, t1), axis=1)
    tout = np.nanmin(np.maximum(t0, t1), axis=1)
    meets_line = tout > tin
    net = r == mlp.ROUTE_NET
    assert np.all(tin[net & meets_line] >= 0)
    assert np.all((np.linalg.norm(od, axis=1) ** 2 > 3) | (r == mlp.ROUTE_OCTREE) | (r == mlp.ROUTE_ZERO))
    full = inputs.uniform_tree(2, 0.5, np.zeros((3, 1)))
    q = core.query(full, o, d, opts=core.NO_STOP)
    zero = r == mlp.ROUTE_ZERO
    assert np.all(q["L"][zero] == 0) and np.all(q["alpha"][zero] == 0)
    # and rays routed to the network that meet the box see its whole chord
    chord = (tout - tin) * np.linalg.norm(dd, axis=1)
    sel = net & meets_line
    assert np.allclose(q["alpha"][sel], np.minimum(1.0, 0.5 * chord[sel]), rtol=1e-9, atol=1e-12)
