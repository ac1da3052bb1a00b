"""A batch of more than 2^31 / 3 rays (its coordinate arrays hold more than
2^31 floats, so every ray's offsets need 64-bit arithmetic): 2^20 seeded
room rays repeated 720 times on the device.  Every copy must return the
bits of the first copy, and the first copy is checked against the oracle
on a sample."""
import sys

import numpy as np
import pytest

import inputs
from oracle import core
from tests import parity

pytestmark = pytest.mark.gpu

BASE = 1 << 20
COPIES = 720          # 754,974,720 rays: 2.26e9 floats per coordinate array


def _say(msg):
    print(f"[gpu] {msg}", flush=True)
    sys.stdout.flush()


def test_batch_beyond_32_bit_offsets(c1_tree):
    import torch
    import paper_2207_05009_amd as lq
    lq.lib()
    o, d = inputs.rays.room_to_proxy(BASE, 77)
    n = BASE * COPIES
    assert 3 * n > 2 ** 31
    _say(f"{n} rays ({COPIES} copies of {BASE}), {3 * n * 4 * 2 / 2 ** 30:.1f} GiB of inputs")
    O = torch.from_numpy(o).cuda().repeat(COPIES, 1)
    D = torch.from_numpy(d).cuda().repeat(COPIES, 1)
    oct_ = lq.Octree(c1_tree, "f16")
    rgb, alpha = oct_.query(O, D)
    torch.cuda.synchronize()
    del O, D
    base_rgb, base_alpha = rgb[:BASE].clone(), alpha[:BASE].clone()
    for k in range(1, COPIES):
        assert torch.equal(rgb[k * BASE:(k + 1) * BASE], base_rgb), k
        assert torch.equal(alpha[k * BASE:(k + 1) * BASE], base_alpha), k
    _say("every copy equals the first")
    idx = np.sort(np.random.default_rng(78).choice(BASE, 4000, replace=False))
    P = core.PreparedTree(c1_tree, "f16")
    oi, di = o[idx], d[idx]
    orc = core.query(c1_tree, oi, di, model=core.LINEAR, prepared=P)

    def cands(k):
        return core.candidates(None, oi[k], di[k], model=core.LINEAR, prepared=P)

    rep = parity.match_plain(base_rgb[idx].cpu().numpy(), base_alpha[idx].cpu().numpy(), orc, c1_tree.l_max,
                             cand_fn=cands)
    _say(f"first copy against the oracle: {rep}")
    assert rep["n_bad"] == 0, rep
