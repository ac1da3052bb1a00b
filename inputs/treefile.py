"""Binary plenoctree file (little-endian), read by the GPU library's loader.

    offset  size  field
    0       4     magic  b"LQOT"
    4       4     u32    version (= 1)
    8       4     i32    max depth D (1..10)
    12      4     i32    SH degree (0..4)
    16      4     i32    n_nodes
    20      4     i32    n_leaves
    24      4     f32    L_max
    28      4     f32    sigma_min
    32      4     f32    alpha_max
    36      4     u32    reserved (0)
    40      ...   i32    child[n_nodes][8]
            ...   f32    sigma[n_leaves]
            ...   f32    sh[n_leaves][3][(deg+1)^2]
"""
from __future__ import annotations

import struct

import numpy as np

from .trees import Tree

MAGIC = b"LQOT"
VERSION = 1
HEADER = struct.Struct("<4sIiiiifffI")


def save(tree: Tree, path: str) -> None:
    with open(path, "wb") as f:
        f.write(HEADER.pack(MAGIC, VERSION, tree.depth, tree.sh_degree, tree.n_nodes,
                            tree.n_leaves, tree.l_max, tree.sigma_min, tree.alpha_max, 0))
        f.write(np.ascontiguousarray(tree.child, dtype="<i4").tobytes())
        f.write(np.ascontiguousarray(tree.sigma, dtype="<f4").tobytes())
        f.write(np.ascontiguousarray(tree.sh, dtype="<f4").tobytes())


def load(path: str) -> Tree:
    with open(path, "rb") as f:
        raw = f.read(HEADER.size)
        magic, ver, depth, deg, nn, nl, lmax, smin, amax, _ = HEADER.unpack(raw)
        if magic != MAGIC or ver != VERSION:
            raise ValueError("not a plenoctree file")
        K = (deg + 1) ** 2
        child = np.frombuffer(f.read(nn * 32), dtype="<i4").reshape(nn, 8).copy()
        sigma = np.frombuffer(f.read(nl * 4), dtype="<f4").copy()
        sh = np.frombuffer(f.read(nl * 12 * K), dtype="<f4").reshape(nl, 3, K).copy()
    t = Tree(depth=depth, sh_degree=deg, l_max=lmax, child=child, sigma=sigma, sh=sh,
             leaf_cells=np.zeros((nl, 3), np.int32), sigma_min=smin, alpha_max=amax)
    return t
