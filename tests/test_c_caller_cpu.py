"""The plain C caller of the library (tests/c_caller/query_file.c) builds
with gcc against include/lumiq.h alone, links liblumiq.so, and reports the
library's errors that need no GPU: a malformed tree file is LQ_ERR_FORMAT
before any device work."""
import os
import subprocess

import numpy as np

import inputs
from inputs import treefile
from tests import c_caller


def test_c_caller_builds_and_reports_a_malformed_file(tmp_path):
    exe = c_caller.build()
    r = subprocess.run([exe], capture_output=True, text=True, timeout=60)
    assert r.returncode == 1 and "usage" in r.stderr
    tree = inputs.random_tree(3, 0.4, seed=5)
    good = tmp_path / "t.lqot"
    treefile.save(tree, str(good))
    bad = tmp_path / "bad.lqot"
    bad.write_bytes(b"XXXX" + good.read_bytes()[4:])
    o, d = inputs.rays.sphere_to_cube(16, 3)
    rays = tmp_path / "rays.bin"
    np.concatenate([o.astype("<f4").ravel(), d.astype("<f4").ravel()]).tofile(rays)
    r = subprocess.run([exe, str(bad), "0", str(rays), "16", str(tmp_path / "out.bin")], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2, (r.stdout, r.stderr)
    assert "status -2" in r.stderr          # LQ_ERR_FORMAT
    r = subprocess.run([exe, str(good), "0", str(tmp_path / "missing.bin"), "16", str(tmp_path / "out.bin")],
                       capture_output=True, text=True, timeout=60)
    assert r.returncode == 1
    assert not os.path.exists(tmp_path / "out.bin")
