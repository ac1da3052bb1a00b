"""Python driver for the FP64 CPU oracle (test infrastructure only).

Only tests/, the smoke check and the benchmark's CPU-baseline leg use this
module; the GPU library never imports it.  It

  * builds and loads lq_oracle.c (gcc, OpenMP);
  * dequantises a tree to the stored precision it is queried at (round to
    nearest even from float32 to float16 / bfloat16, then back to float64
    exactly), written here independently of the GPU library's converter;
  * runs the FP64 octree march over a batch, and re-runs every ray whose
    FP64 decisions were within the filter in exact rational arithmetic
    (oracle/exact.py).
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
import threading

import numpy as np

from . import exact

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "lq_oracle.c")
LIB = os.path.join(HERE, "liblq_oracle.so")

NEED_EXACT, AMBIGUOUS, MISS, BADRAY = 1, 2, 4, 8
NO_STOP, NO_SKIP = 1, 4
LINEAR, EXP = 0, 1
ETA = 1e-4

_lock = threading.Lock()
_lib = None


def build(force: bool = False) -> str:
    if force or not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
        tmp = LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-D_GNU_SOURCE", "-fopenmp", "-fPIC",
                               "-shared", "-Wall", "-o", tmp, SRC, "-lm"])
        os.replace(tmp, LIB)
    return LIB


class _Tree(C.Structure):
    _fields_ = [("depth", C.c_int32), ("sh_degree", C.c_int32), ("n_nodes", C.c_int32),
                ("n_leaves", C.c_int32), ("l_max", C.c_double), ("sigma_min", C.c_double),
                ("alpha_max", C.c_double), ("eta", C.c_double),
                ("child", C.c_void_p), ("sigma", C.c_void_p), ("sh", C.c_void_p)]


def lib():
    global _lib
    with _lock:
        if _lib is None:
            build()
            L = C.CDLL(LIB)
            L.orc_query.restype = C.c_int
            L.orc_query.argtypes = [C.POINTER(_Tree), C.c_void_p, C.c_void_p, C.c_int64, C.c_int,
                                    C.c_uint32] + [C.c_void_p] * 15 + [C.c_int32, C.c_int]
            L.orc_candidates.restype = C.c_int
            L.orc_candidates.argtypes = [C.POINTER(_Tree), C.c_void_p, C.c_void_p, C.c_int64, C.c_int,
                                         C.c_uint32, C.c_int] + [C.c_void_p] * 8 + [C.c_int]
            L.orc_sh_eval.restype = None
            L.orc_sh_eval.argtypes = [C.c_int, C.c_void_p, C.c_void_p]
            L.orc_max_threads.restype = C.c_int
            _lib = L
    return _lib


# ---------------------------------------------------------------- storage
def to_bf16_rne(x: np.ndarray) -> np.ndarray:
    """float32 -> bfloat16 (round to nearest, ties to even), returned as the
    exactly representable float32 values."""
    u = np.ascontiguousarray(x, dtype=np.float32).view(np.uint32).astype(np.uint64)
    lsb = (u >> np.uint64(16)) & np.uint64(1)
    r = ((u + np.uint64(0x7FFF) + lsb) >> np.uint64(16)) << np.uint64(16)
    out = (r & np.uint64(0xFFFFFFFF)).astype(np.uint32).view(np.float32)
    nan = np.isnan(x)
    if np.any(nan):
        out = out.copy()
        out[nan] = np.nan
    return out


def dequantize(x: np.ndarray, storage: str) -> np.ndarray:
    x = np.asarray(x, dtype=np.float32)
    if storage == "f32":
        return x.astype(np.float64)
    if storage == "f16":
        return x.astype(np.float16).astype(np.float64)
    if storage == "bf16":
        return to_bf16_rne(x).astype(np.float64)
    raise ValueError(storage)


# ---------------------------------------------------------------- SH
def sh_eval(deg: int, w) -> np.ndarray:
    """Real orthonormal SH (no Condon-Shortley phase) at unit direction w."""
    w = np.ascontiguousarray(np.asarray(w, dtype=np.float64).reshape(3))
    Y = np.zeros(25, dtype=np.float64)
    lib().orc_sh_eval(int(deg), w.ctypes.data, Y.ctypes.data)
    return Y[: (deg + 1) ** 2].copy()


# ---------------------------------------------------------------- pruning
def pruned_tree(tree, storage: str = "f32"):
    """The tree without the data leaves that the sigma_min skip never
    composites (Sec. 6.2: stored density below sigma_min, compared at the
    stored precision) and without the internal nodes left with no child.
    Leaf indices (and so the density and SH arrays) are unchanged; the root
    stays node 0.  Marching it with the skip off visits exactly the
    composited leaves of the original tree, over the same segments."""
    import dataclasses
    child = np.asarray(tree.child, dtype=np.int64)
    keep = dequantize(tree.sigma, storage) >= float(np.float32(tree.sigma_min))
    levels = [np.array([0])]
    while True:
        kids = child[levels[-1]]
        nxt = kids[kids > 0]
        if nxt.size == 0:
            break
        levels.append(nxt)
    alive = np.zeros(child.shape[0], bool)
    for nodes in reversed(levels):
        kids = child[nodes]
        sub = np.zeros(kids.shape, bool)
        sub[kids > 0] = alive[kids[kids > 0]]
        sub[kids < 0] = keep[-kids[kids < 0] - 1]
        alive[nodes] = sub.any(1)
    order = np.concatenate(levels)
    order = order[(order == 0) | alive[order]]
    new_index = np.zeros(child.shape[0], np.int64)
    new_index[order] = np.arange(order.size)
    kids = child[order]
    out = np.zeros(kids.shape, np.int32)
    node_kept = (kids > 0) & alive[np.maximum(kids, 0)]
    out[node_kept] = new_index[kids[node_kept]]
    leaf_kept = kids < 0
    leaf_kept[leaf_kept] = keep[-kids[leaf_kept] - 1]
    out[leaf_kept] = kids[leaf_kept]
    return dataclasses.replace(tree, child=out)


# ---------------------------------------------------------------- query
def _ptr(a):
    return None if a is None else a.ctypes.data


class PreparedTree:
    """A tree's arrays at one storage precision, promoted to float64."""

    def __init__(self, tree, storage: str = "f32"):
        self.tree = tree
        self.storage = storage
        self.child = np.ascontiguousarray(tree.child, dtype=np.int32)
        self.sigma = np.ascontiguousarray(dequantize(tree.sigma, storage))
        self.sh = np.ascontiguousarray(dequantize(tree.sh, storage))
        self.c = _Tree(tree.depth, tree.sh_degree, self.child.shape[0], self.sigma.shape[0],
                       float(tree.l_max), float(np.float32(tree.sigma_min)),
                       float(np.float32(tree.alpha_max)), ETA,
                       self.child.ctypes.data, self.sigma.ctypes.data, self.sh.ctypes.data)


def query(tree, o, d, model: int = LINEAR, opts: int = 0, storage: str = "f32",
          max_ids: int = 0, n_threads: int = 0, exact_fallback: bool = True,
          prepared: PreparedTree | None = None, force_exact: bool = False) -> dict:
    """Run the oracle over a batch of rays.  Returns a dict of numpy arrays:
    L [n,3], alpha, count, hash, term_idx, n_comp, n_nodes, flags, the
    alternative candidate for threshold-ambiguous rays (alt_*), optional
    leaf_ids [n, max_ids], and n_exact (rays re-run exactly)."""
    P = prepared if prepared is not None else PreparedTree(tree, storage)
    o = np.ascontiguousarray(o, dtype=np.float32).reshape(-1, 3)
    d = np.ascontiguousarray(d, dtype=np.float32).reshape(-1, 3)
    n = o.shape[0]
    out = {
        "L": np.zeros((n, 3)), "alpha": np.zeros(n), "count": np.zeros(n, np.int32),
        "hash": np.zeros(n, np.uint64), "term_idx": np.zeros(n, np.int32),
        "n_comp": np.zeros(n, np.int32), "n_nodes": np.zeros(n, np.int32),
        "flags": np.zeros(n, np.uint32),
        "alt_L": np.zeros((n, 3)), "alt_alpha": np.zeros(n), "alt_count": np.zeros(n, np.int32),
        "alt_hash": np.zeros(n, np.uint64), "alt_term": np.zeros(n, np.int32),
        "alt_valid": np.zeros(n, np.uint8),
    }
    ids = np.zeros((n, max_ids), np.uint32) if max_ids > 0 else None
    lib().orc_query(C.byref(P.c), o.ctypes.data, d.ctypes.data, n, int(model), int(opts),
                    _ptr(out["L"]), _ptr(out["alpha"]), _ptr(out["count"]), _ptr(out["hash"]),
                    _ptr(out["term_idx"]), _ptr(out["n_comp"]), _ptr(out["n_nodes"]),
                    _ptr(out["flags"]), _ptr(out["alt_L"]), _ptr(out["alt_alpha"]),
                    _ptr(out["alt_count"]), _ptr(out["alt_hash"]), _ptr(out["alt_term"]),
                    _ptr(out["alt_valid"]), _ptr(ids), int(max_ids), int(n_threads))
    if ids is not None:
        out["leaf_ids"] = ids
    flagged = np.nonzero(out["flags"] & NEED_EXACT)[0]
    if force_exact:       # test hook: re-run every ray in exact arithmetic
        flagged = np.arange(n)
    out["n_exact"] = int(flagged.size)
    if exact_fallback:
        for i in flagged.tolist():
            _exact_ray(P, o[i], d[i], model, opts, out, i, ids, max_ids)
    return out


def candidates(tree, o, d, model: int = LINEAR, opts: int = 0, storage: str = "f32",
               max_cand: int = 8, prepared: PreparedTree | None = None, force_exact: bool = False) -> dict:
    """Every valid outcome of each ray's alpha_max stop (Sec. 6.2, reading
    R3 for rays with several stop tests within eta of the threshold: each of
    those may go either way, so the march may stop at any of them or
    continue through all of them; the other tests keep their decision).
    Candidate 0 continues at every ambiguous test; candidate c >= 1 stops at
    the c-th ambiguous test.  Returns arrays [n, max_cand]: L [n, max_cand,
    3], alpha, count, hash, term_idx, n_comp, n_nodes and valid (unused
    slots 0).  Rays whose FP64 decisions were within the filter are re-run
    exactly, as in query()."""
    P = prepared if prepared is not None else PreparedTree(tree, storage)
    o = np.ascontiguousarray(o, dtype=np.float32).reshape(-1, 3)
    d = np.ascontiguousarray(d, dtype=np.float32).reshape(-1, 3)
    n, m = o.shape[0], int(max_cand)
    out = {"L": np.zeros((n, m, 3)), "alpha": np.zeros((n, m)), "count": np.zeros((n, m), np.int32),
           "hash": np.zeros((n, m), np.uint64), "term_idx": np.zeros((n, m), np.int32),
           "n_comp": np.zeros((n, m), np.int32), "n_nodes": np.zeros((n, m), np.int32),
           "valid": np.zeros((n, m), np.uint8)}
    lib().orc_candidates(C.byref(P.c), o.ctypes.data, d.ctypes.data, n, int(model), int(opts), m,
                         _ptr(out["L"]), _ptr(out["alpha"]), _ptr(out["count"]), _ptr(out["hash"]),
                         _ptr(out["term_idx"]), _ptr(out["n_comp"]), _ptr(out["n_nodes"]),
                         _ptr(out["valid"]), 0)
    # rays the FP64 march could not decide: the exact path
    flags = query(None, o, d, model=model, opts=opts, prepared=P, exact_fallback=False)["flags"]
    redo = np.arange(n) if force_exact else np.nonzero(flags & NEED_EXACT)[0]
    for i in redo.tolist():
        tr = P.tree
        segs, visited, ordinals = exact.march_octree(tr, o[i], d[i], with_ordinals=True)
        df = np.asarray(d[i], dtype=np.float64)
        dl = np.sqrt((df * df).sum())
        Y = sh_eval(tr.sh_degree, -df / dl) if dl > 0 else np.zeros(25)
        kw = dict(no_stop=bool(opts & NO_STOP), no_skip=bool(opts & NO_SKIP), sigma=P.sigma, sh=P.sh)
        first = exact.composite(tr, segs, d[i], Y, model, force_stop=exact.FORCE_CONTINUE, **kw)
        forces = [exact.FORCE_CONTINUE] + first["amb_tests"][: m - 1]
        out["valid"][i] = 0
        for c, f in enumerate(forces):
            r = exact.composite(tr, segs, d[i], Y, model, force_stop=f, **kw)
            out["L"][i, c] = r["L"]
            out["alpha"][i, c] = r["alpha"]
            out["count"][i, c] = r["count"]
            out["hash"][i, c] = r["hash"]
            out["term_idx"][i, c] = r["term_idx"]
            out["n_comp"][i, c] = r["n_comp"]
            out["n_nodes"][i, c] = ordinals[r["term_idx"]] if r["term_idx"] >= 0 else visited
            out["valid"][i, c] = 1
    return out


def _exact_ray(P, o, d, model, opts, out, i, ids, max_ids):
    tree = P.tree
    segs, visited, ordinals = exact.march_octree(tree, o, d, with_ordinals=True)
    flags = int(out["flags"][i]) & ~(NEED_EXACT | AMBIGUOUS | MISS)
    if not segs and not _hits(tree, o, d):
        flags |= MISS
    df = np.asarray(d, dtype=np.float64)
    dl = np.sqrt((df * df).sum())
    Y = sh_eval(tree.sh_degree, -df / dl) if dl > 0 else np.zeros(25)
    kw = dict(no_stop=bool(opts & NO_STOP), no_skip=bool(opts & NO_SKIP), sigma=P.sigma, sh=P.sh)
    r = exact.composite(tree, segs, d, Y, model, **kw)
    out["L"][i] = r["L"]
    out["alpha"][i] = r["alpha"]
    out["count"][i] = r["count"]
    out["hash"][i] = r["hash"]
    out["term_idx"][i] = r["term_idx"]
    out["n_comp"][i] = r["n_comp"]
    # nodes visited up to the stop leaf (or to the far box hit)
    out["n_nodes"][i] = ordinals[r["term_idx"]] if r["term_idx"] >= 0 else visited
    out["alt_valid"][i] = 0
    if r["first_amb_test"] >= 0:
        flags |= AMBIGUOUS
        a = exact.composite(tree, segs, d, Y, model, flip_test=r["first_amb_test"], **kw)
        out["alt_L"][i] = a["L"]
        out["alt_alpha"][i] = a["alpha"]
        out["alt_count"][i] = a["count"]
        out["alt_hash"][i] = a["hash"]
        out["alt_term"][i] = a["term_idx"]
        out["alt_valid"][i] = 1
    out["flags"][i] = flags
    if ids is not None:
        ids[i] = 0
        m = min(max_ids, len(r["ids"]))
        ids[i, :m] = r["ids"][:m]


def _hits(tree, o, d) -> bool:
    return exact._Ray(o, d, tree.depth).clip() is not None


def max_threads() -> int:
    return int(lib().orc_max_threads())
