"""FP64 oracle of the learned surrogate (test infrastructure only).

The surrogate stands in for the octree march on incoherent shading queries:
a ray is reduced to the 5D light-field coordinates of Sec. 3 (Eq. 1) -- the
point where its line enters the sphere of radius sqrt(3) that bounds the
proxy box, and its unit direction -- encoded with NeRF-style Fourier features
(Sec. 4.2, "Network architecture": positional encoding of the inputs), and
mapped by a 4 x 64 ReLU MLP to log-radiance.

  x6      = (e / sqrt(3), d/|d|)  in [-1, 1]^6, e the near sphere hit of the line
  feat(v) = [v, sin(2^k pi v), cos(2^k pi v)]_{k=0..9}  -> 6 x 21 = 126, + 2 zeros
  h1..h4  = relu(W_l h + b_l),  W_1: 64 x 128, W_2..4: 64 x 64
  y       = W_5 h4 + b_5 (3 outputs),  L_hat = exp(y) - eps_out, eps_out = 1e-2

Loss: the HDR relative colour loss of Sec. 4.3 (Eq. 8) with lambda = 1,
epsilon = 0.01, the approximate luminance taken as the channel mean of the
prediction, treated as a constant in the gradient:
  l = sum_c (L_hat_c - L_c)^2 / (mean_c L_hat + 0.01)^2,   batch mean over B.
Optimiser: Adam (beta = 0.9, 0.999, eps = 1e-8) with the learning rate
decaying exponentially from 5e-4 to 5e-6 over the run (Sec. 4.4).

Parameters are one flat vector: for each layer W_l as [out][in] row-major,
then b_l [out].  Rays whose line misses the sphere have no surrogate value
(radiance 0) and contribute nothing to the loss.
"""
from __future__ import annotations

import math

import numpy as np

N_FREQ = 10
N_FEAT = 6 * (1 + 2 * N_FREQ)          # 126
FEAT_PAD = 128
HIDDEN = 64
LAYERS = [(FEAT_PAD, HIDDEN), (HIDDEN, HIDDEN), (HIDDEN, HIDDEN), (HIDDEN, HIDDEN), (HIDDEN, 3)]
EPS_OUT = 1e-2
LOSS_EPS = 1e-2
R2 = 3.0                               # squared radius of the bounding sphere of [-1,1]^3


def n_params() -> int:
    return sum(i * o + o for i, o in LAYERS)


def unpack(theta):
    """Flat vector -> [(W [out, in], b [out]), ...] (views)."""
    out, p = [], 0
    for i, o in LAYERS:
        W = theta[p: p + i * o].reshape(o, i)
        p += i * o
        b = theta[p: p + o]
        p += o
        out.append((W, b))
    return out


def sphere_param(o, d):
    """Near intersection of the line o + t d with |x|^2 = 3 (t may be
    negative: only the line matters for a ray starting outside the proxy).
    Returns (x6 [n, 6], hit [n] bool)."""
    o = np.asarray(o, dtype=np.float64)
    d = np.asarray(d, dtype=np.float64)
    dn = d / np.linalg.norm(d, axis=1, keepdims=True)
    b = (o * dn).sum(1)
    c = (o * o).sum(1) - R2
    disc = b * b - c
    hit = disc > 0.0
    t = -b - np.sqrt(np.where(hit, disc, 0.0))
    e = o + t[:, None] * dn
    x6 = np.concatenate([e / math.sqrt(R2), dn], axis=1)
    x6[~hit] = 0.0
    return x6, hit


ROUTE_NET, ROUTE_OCTREE, ROUTE_ZERO = 0, 1, 2


def route(o, d):
    """Which path answers a ray of the hybrid query.  The network models the
    radiance of a whole line (the proxy chord the line crosses); a ray sees
    that whole chord only when the bounding sphere, and so the box inside it,
    lies wholly ahead of its origin.  ROUTE_ZERO: the line misses the sphere
    or the sphere lies wholly behind (radiance 0); ROUTE_OCTREE: the origin
    is inside the sphere; ROUTE_NET: the sphere lies ahead (then both
    crossing parameters, whose product is |o|^2 - 3 > 0, are positive)."""
    o = np.asarray(o, dtype=np.float64)
    d = np.asarray(d, dtype=np.float64)
    _, hit = sphere_param(o, d)
    c = (o * o).sum(1) - R2
    ahead = (o * d).sum(1) < 0.0
    out = np.full(o.shape[0], ROUTE_ZERO, np.int32)
    out[hit & (c > 0) & ahead] = ROUTE_NET
    out[hit & ~(c > 0)] = ROUTE_OCTREE
    return out


def features(x6):
    x6 = np.asarray(x6, dtype=np.float64)
    n = x6.shape[0]
    F = np.zeros((n, FEAT_PAD))
    for v in range(6):
        x = x6[:, v]
        base = v * (1 + 2 * N_FREQ)
        F[:, base] = x
        for k in range(N_FREQ):
            F[:, base + 1 + 2 * k] = np.sin((2.0 ** k) * math.pi * x)
            F[:, base + 2 + 2 * k] = np.cos((2.0 ** k) * math.pi * x)
    return F


def forward(theta, F, round_bf16=None):
    """Returns (y [n, 3], cache).  round_bf16, if given, is applied to every
    GEMM input (weights and activations; in loss_and_grad also the output
    gradients) to mirror a bfloat16 kernel."""
    r = round_bf16 if round_bf16 is not None else (lambda a: a)
    layers = unpack(theta)
    h = r(F)
    hs, zs = [h], []
    for li, (W, b) in enumerate(layers):
        z = h @ r(W).T + b
        zs.append(z)
        if li < len(layers) - 1:
            h = r(np.maximum(z, 0.0))
            hs.append(h)
    return zs[-1], (hs, zs, layers, r)


def predict(theta, o, d, round_bf16=None):
    x6, hit = sphere_param(o, d)
    y, _ = forward(theta, features(x6), round_bf16)
    L = np.maximum(np.exp(y) - EPS_OUT, 0.0)
    L[~hit] = 0.0
    return L, hit


def loss_and_grad(theta, F, target, active, round_bf16=None):
    """Batch-mean loss and its gradient w.r.t. theta (flat)."""
    y, (hs, zs, layers, r) = forward(theta, F, round_bf16)
    B = F.shape[0]
    ey = np.exp(y)
    Lh = ey - EPS_OUT
    den = Lh.mean(1) + LOSS_EPS                        # treated as a constant
    diff = Lh - target
    per = (diff * diff).sum(1) / (den * den)
    per = np.where(active, per, 0.0)
    loss = per.sum() / B
    dy = np.where(active[:, None], 2.0 * diff * ey / (den * den)[:, None], 0.0) / B
    grads = []
    # the backward GEMM inputs (output gradients) are rounded like the forward
    # ones when round_bf16 is given
    g = r(dy)
    for li in range(len(layers) - 1, -1, -1):
        W, b = layers[li]
        h_in = hs[li]
        gW = g.T @ h_in
        gb = g.sum(0)
        grads.append((gW, gb))
        if li > 0:
            g = r((g @ r(W)) * (zs[li - 1] > 0.0))
    grads.reverse()
    flat = np.concatenate([np.concatenate([gW.ravel(), gb]) for gW, gb in grads])
    return loss, flat


def lr_at(step, steps, lr0=5e-4, lr1=5e-6):
    """Exponential decay from lr0 (step 0) to lr1 (step = steps)."""
    return lr0 * (lr1 / lr0) ** (step / steps)


def adam_step(theta, grad, m, v, step, lr, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update (Kingma & Ba); step counts from 1."""
    m = b1 * m + (1 - b1) * grad
    v = b2 * v + (1 - b2) * grad * grad
    mh = m / (1 - b1 ** step)
    vh = v / (1 - b2 ** step)
    theta = theta - lr * mh / (np.sqrt(vh) + eps)
    return theta, m, v


def he_uniform(seed):
    rng = np.random.default_rng(seed)
    parts = []
    for i, o in LAYERS:
        lim = math.sqrt(6.0 / i)
        parts.append(rng.uniform(-lim, lim, size=i * o))
        parts.append(np.zeros(o))
    return np.concatenate(parts)


def bf16(a):
    """Round to bfloat16 (nearest even), returned as float64."""
    from .core import to_bf16_rne
    return to_bf16_rne(np.asarray(a, dtype=np.float32)).astype(np.float64)
