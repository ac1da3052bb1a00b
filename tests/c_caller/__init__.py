"""A plain C caller of the library (query_file.c) and its build step."""
from __future__ import annotations

import os
import shutil
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
SOURCE = os.path.join(HERE, "query_file.c")
PROGRAM = os.path.join(HERE, "query_file")
PKG = os.path.join(ROOT, "paper_2207_05009_amd")


def build(verbose: bool = False) -> str:
    """Compile query_file.c with gcc (C11) against include/lumiq.h, linking
    liblumiq.so and the system HIP runtime; the library is found next to
    the package at run time ($ORIGIN-relative path)."""
    if not os.path.exists(os.path.join(PKG, "liblumiq.so")):
        from paper_2207_05009_amd import build as lqbuild
        lqbuild.build()
    gcc = shutil.which("gcc")
    if gcc is None:
        raise RuntimeError("gcc not found")
    tmp = PROGRAM + ".tmp"
    cmd = [gcc, "-std=c11", "-O2", "-Wall", "-Wextra", "-Werror", "-D__HIP_PLATFORM_AMD__",
           "-I/opt/rocm/include", f"-I{os.path.join(ROOT, 'include')}", "-o", tmp, SOURCE,
           f"-L{PKG}", "-llumiq", "-L/opt/rocm/lib", "-lamdhip64",
           "-Wl,-rpath,$ORIGIN/../../paper_2207_05009_amd", "-Wl,-rpath,/opt/rocm/lib"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, PROGRAM)
    return PROGRAM


def program() -> str:
    """The built program (built first if missing)."""
    return PROGRAM if os.path.exists(PROGRAM) else build()
