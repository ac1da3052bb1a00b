"""The emission query from a plain C program (tests/c_caller/query_file.c):
no torch in the process, the system HIP runtime, device buffers that the
caller allocates.  Its radiance and alpha match the oracle (Sec. 4.1,
Eqs. 3-5; Sec. 6.2), and inside the program the allocation-free entry point
returns the same bits and host pointers are refused."""
import subprocess
import sys

import numpy as np
import pytest

import inputs
from inputs import treefile
from oracle import core
from tests import c_caller, parity

pytestmark = pytest.mark.gpu


def _say(msg):
    print(f"[gpu] {msg}", flush=True)
    sys.stdout.flush()


@pytest.mark.parametrize("storage,code", [("f32", 0), ("f16", 1)])
def test_query_from_c(tmp_path, storage, code):
    exe = c_caller.program()
    tree = inputs.random_tree(6, 0.35, seed=81)
    path = tmp_path / "tree.lqot"
    treefile.save(tree, str(path))
    o1, d1 = inputs.rays.sphere_to_cube(20_000, 82)
    o2, d2 = inputs.rays.room_to_proxy(20_001, 83)     # ragged total: 40,001 rays
    o = np.concatenate([o1, o2]).astype(np.float32)
    d = np.concatenate([d1, d2]).astype(np.float32)
    n = len(o)
    rays = tmp_path / "rays.bin"
    np.concatenate([o.astype("<f4").ravel(), d.astype("<f4").ravel()]).tofile(rays)
    out = tmp_path / "out.bin"
    _say(f"C caller: {storage}, depth-6 tree, {n} rays")
    r = subprocess.run([exe, str(path), str(code), str(rays), str(n), str(out)], capture_output=True, text=True,
                       timeout=300)
    print(r.stdout[-2000:], r.stderr[-2000:], flush=True)
    assert r.returncode == 0
    raw = np.fromfile(out, dtype="<f4")
    assert raw.size == 4 * n
    rgb, alpha = raw[:3 * n].reshape(n, 3), raw[3 * n:]
    P = core.PreparedTree(tree, storage)
    orc = core.query(tree, o, d, model=core.LINEAR, prepared=P)

    def cands(k):
        return core.candidates(None, o[k], d[k], model=core.LINEAR, prepared=P)

    rep = parity.match_plain(rgb, alpha, orc, tree.l_max, cand_fn=cands)
    _say(f"against the oracle: {rep}")
    assert rep["n_bad"] == 0, rep
    assert (alpha > 0).sum() > n // 4          # the rays do cross the luminaire
