"""Helpers comparing the GPU library with the oracle (imported by GPU tests).

Radiance error per ray and channel (relative, floored at 1e-6 L_max):
    |L - L_ref| / max(|L_ref|, 1e-6 L_max).
A ray whose alpha_max stop test came within eta = 1e-4 of the threshold in
the oracle has two valid outcomes (stop there, or continue); the GPU must
match one of them, bit-exactly in its leaf records.
"""
from __future__ import annotations

import numpy as np

from oracle import core

RTOL = 1e-4          # float32 compositing vs the FP64 oracle
FLOOR = 1e-6         # x L_max


def rel_err(L, ref, l_max):
    return np.abs(L - ref) / np.maximum(np.abs(ref), FLOOR * l_max)


def compare(gpu: dict, orc: dict, l_max: float, rtol: float = RTOL, ids: bool = True) -> dict:
    """gpu: numpy dict from Octree.trace (count, hash, term_idx, rgb, alpha,
    optional leaf_ids); orc: oracle.core.query output.  Returns a report;
    report['ok'] is True when every ray matches one oracle candidate."""
    n = len(orc["count"])
    g_hash = gpu["hash"].astype(np.int64).view(np.uint64)
    o_hash = orc["hash"].astype(np.uint64)
    canon = ((gpu["count"].astype(np.int64) == orc["count"]) & (g_hash == o_hash)
             & (gpu["term_idx"] == orc["term_idx"]))
    alt = (orc["alt_valid"].astype(bool)
           & (gpu["count"].astype(np.int64) == orc["alt_count"])
           & (g_hash == orc["alt_hash"].astype(np.uint64))
           & (gpu["term_idx"] == orc["alt_term"]))
    use_alt = ~canon & alt
    ref_L = np.where(use_alt[:, None], orc["alt_L"], orc["L"])
    ref_a = np.where(use_alt, orc["alt_alpha"], orc["alpha"])
    err = rel_err(gpu["rgb"].astype(np.float64), ref_L, l_max)
    aerr = np.abs(gpu["alpha"].astype(np.float64) - ref_a)
    seq_ok = canon | alt
    id_ok = np.ones(n, bool)
    if ids and "leaf_ids" in gpu and "leaf_ids" in orc:
        m = min(gpu["leaf_ids"].shape[1], orc["leaf_ids"].shape[1])
        cnt = np.minimum(orc["count"], m)
        mask = np.arange(m)[None, :] < cnt[:, None]
        same = (gpu["leaf_ids"][:, :m].astype(np.uint32) == orc["leaf_ids"][:, :m]) | ~mask
        id_ok = same.all(1) | use_alt
    steps_ok = np.ones(n, bool)
    if "n_steps" in gpu:
        steps_ok = (gpu["n_steps"].astype(np.int64) == orc["n_nodes"]) | use_alt
    bad = ~seq_ok | ~id_ok | ~steps_ok | (err.max(1) > rtol) | (aerr > rtol)
    return {
        "n": n, "ok": not bad.any(), "n_bad": int(bad.sum()), "bad_idx": np.nonzero(bad)[0][:20],
        "n_seq_mismatch": int((~seq_ok).sum()), "n_id_mismatch": int((~id_ok).sum()),
        "n_steps_mismatch": int((~steps_ok).sum()),
        "n_alt": int(use_alt.sum()), "n_ambiguous": int(orc["alt_valid"].sum()),
        "max_rel": float(err.max()) if n else 0.0,
        "p99_rel": float(np.quantile(err.max(1), 0.99)) if n else 0.0,
        "max_alpha_err": float(aerr.max()) if n else 0.0,
        "rel_l2": float(np.linalg.norm(gpu["rgb"] - ref_L) / max(np.linalg.norm(ref_L), 1e-300)),
        "n_exact": orc.get("n_exact", 0),
    }


def to_numpy(d: dict) -> dict:
    return {k: v.cpu().numpy() for k, v in d.items()}


def oracle_for(tree, o, d, model, flags_gpu: int, storage="f32", max_ids=0):
    opts = 0
    if flags_gpu & 1:
        opts |= core.NO_STOP
    if flags_gpu & 4:
        opts |= core.NO_SKIP
    return core.query(tree, o, d, model=model, opts=opts, storage=storage, max_ids=max_ids)
