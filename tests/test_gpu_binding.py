"""The Python binding in a fresh process that uploads a tree before it
touches torch: the binding loads torch's HIP runtime first, so the library
and torch share one runtime, and the query still matches the oracle."""
import os
import subprocess
import sys

import numpy as np
import pytest

import inputs
from tests import parity

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

SCRIPT = r"""
import sys
import numpy as np
sys.path.insert(0, sys.argv[1])
import inputs
from paper_2207_05009_amd import lumiq
tree = inputs.random_tree(4, 0.4, seed=71)
oct_ = lumiq.Octree(tree, "f32")          # the first HIP call of the process
print("[child] tree uploaded", flush=True)
import torch
o, d = inputs.rays.sphere_to_cube(4096, 72)
out = oct_.trace(torch.from_numpy(o).cuda(), torch.from_numpy(d).cuda(), model="linear", max_ids=64)
torch.cuda.synchronize()
np.savez(sys.argv[2], **{k: v.cpu().numpy() for k, v in out.items()})
print("[child] done", flush=True)
"""


def test_tree_upload_before_torch(tmp_path):
    out = tmp_path / "trace.npz"
    print("[gpu] child process: tree upload before import torch", flush=True)
    r = subprocess.run([sys.executable, "-c", SCRIPT, ROOT, str(out)], capture_output=True, text=True,
                       timeout=300, cwd=ROOT)
    print(r.stdout[-2000:], r.stderr[-2000:], flush=True)
    assert r.returncode == 0
    g = dict(np.load(out))
    tree = inputs.random_tree(4, 0.4, seed=71)
    o, d = inputs.rays.sphere_to_cube(4096, 72)
    orc = parity.oracle_for(tree, o, d, 0, 0, max_ids=64)
    rep = parity.compare(g, orc, tree.l_max)
    assert rep["ok"], rep
