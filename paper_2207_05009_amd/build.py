"""Build liblumiq.so (gfx950) in-tree with hipcc: every translation unit is
compiled in parallel to an object, then the objects are linked."""
from __future__ import annotations

import os
import subprocess
import sys
import tempfile
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "liblumiq.so")
SOURCES = ["api.hip", "proxy_shade.hip", "octree_query.hip", "octree_query_f32.hip", "octree_query_f16.hip",
           "octree_query_bf16.hip", "mlp.hip", "distill.hip"]

HIPCC_FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC",
    # compositing and the error-free transformations rely on unfused
    # arithmetic; fused multiply-adds are written explicitly
    "-ffp-contract=off",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function",
]


def sources():
    return [os.path.join(CSRC, s) for s in SOURCES]


def _hipcc():
    return os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")


def build(verbose: bool = False, jobs: int | None = None) -> str:
    jobs = jobs or min(len(SOURCES), max(1, min(16, os.cpu_count() or 1)))
    with tempfile.TemporaryDirectory(prefix="lumiq_build_") as tmp:
        objs = [os.path.join(tmp, os.path.basename(s) + ".o") for s in sources()]

        def compile_one(pair):
            src, obj = pair
            cmd = [_hipcc(), *HIPCC_FLAGS, "-c", "-o", obj, src]
            if verbose:
                print(" ".join(cmd), flush=True)
            r = subprocess.run(cmd, capture_output=True, text=True)
            return src, r.returncode, r.stdout + r.stderr

        with ThreadPoolExecutor(jobs) as ex:
            results = list(ex.map(compile_one, zip(sources(), objs)))
        failed = False
        for src, rc, out in results:
            lines = [ln for ln in out.splitlines() if "packed-fp32-ops" not in ln]
            if rc != 0 or (verbose and lines):
                print("\n".join(lines), file=sys.stderr)
            failed = failed or rc != 0
        if failed:
            raise RuntimeError("hipcc failed")
        tmp_lib = LIB + ".tmp"
        cmd = [_hipcc(), "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp_lib, *objs]
        if verbose:
            print(" ".join(cmd), flush=True)
        subprocess.check_call(cmd)
        os.replace(tmp_lib, LIB)
    return LIB


if __name__ == "__main__":
    build(verbose="-v" in sys.argv)
    sys.exit(0)
