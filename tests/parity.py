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


def match_candidates(gpu: dict, cand: dict, l_max: float, rtol: float = RTOL, records: bool = True):
    """Per ray, True when the GPU output equals one valid outcome of
    oracle.core.candidates (every outcome of a ray with several stop tests
    within eta of alpha_max): radiance and alpha within rtol, and with
    records the count, hash, stop index (and node count) bit-exact."""
    n, m = cand["valid"].shape
    ok = np.zeros(n, bool)
    g = np.asarray(gpu["rgb"], np.float64)
    for c in range(m):
        good = cand["valid"][:, c].astype(bool)
        good &= rel_err(g, cand["L"][:, c], l_max).max(1) <= rtol
        if gpu.get("alpha") is not None:
            good &= np.abs(np.asarray(gpu["alpha"], np.float64) - cand["alpha"][:, c]) <= rtol
        if records:
            g_hash = np.asarray(gpu["hash"]).astype(np.int64).view(np.uint64)
            good &= (np.asarray(gpu["count"]).astype(np.int64) == cand["count"][:, c])
            good &= g_hash == cand["hash"][:, c].astype(np.uint64)
            good &= np.asarray(gpu["term_idx"]) == cand["term_idx"][:, c]
            if "n_steps" in gpu:
                good &= np.asarray(gpu["n_steps"]).astype(np.int64) == cand["n_nodes"][:, c]
        ok |= good
    return ok


def compare(gpu: dict, orc: dict, l_max: float, rtol: float = RTOL, ids: bool = True,
            cand_fn=None) -> dict:
    """gpu: numpy dict from Octree.trace (count, hash, term_idx, rgb, alpha,
    optional leaf_ids); orc: oracle.core.query output.  Returns a report;
    report['ok'] is True when every ray matches one oracle candidate.  A ray
    with more than one stop test within eta of the threshold may match
    neither the canonical outcome nor the single alternative; given
    cand_fn(indices) -> oracle.core.candidates of those rays, such rays are
    checked against every valid outcome (counted in n_multi)."""
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
    n_multi = 0
    redo = np.nonzero(bad & ((orc["flags"] & 2) != 0))[0]
    if cand_fn is not None and redo.size:
        sub = {k: np.asarray(gpu[k])[redo] for k in ("rgb", "alpha", "count", "hash", "term_idx", "n_steps")
               if k in gpu}
        ok = match_candidates(sub, cand_fn(redo), l_max, rtol, records=True)
        bad[redo[ok]] = False
        seq_ok[redo[ok]] = True
        steps_ok[redo[ok]] = True
        err[redo[ok]] = 0.0        # within rtol of the candidate they match
        aerr[redo[ok]] = 0.0
        n_multi = int(ok.sum())
    return {
        "n": n, "ok": not bad.any(), "n_bad": int(bad.sum()), "bad_idx": np.nonzero(bad)[0][:20],
        "n_seq_mismatch": int((~seq_ok).sum()), "n_id_mismatch": int((~id_ok).sum()),
        "n_steps_mismatch": int((~steps_ok).sum()),
        "n_alt": int(use_alt.sum()), "n_multi": n_multi, "n_ambiguous": int(orc["alt_valid"].sum()),
        "max_rel": float(err.max()) if n else 0.0,
        "p99_rel": float(np.quantile(err.max(1), 0.99)) if n else 0.0,
        "max_alpha_err": float(aerr.max()) if n else 0.0,
        "rel_l2": float(np.linalg.norm(gpu["rgb"] - ref_L) / max(np.linalg.norm(ref_L), 1e-300)),
        "n_exact": orc.get("n_exact", 0),
    }


def match_plain(rgb, alpha, orc: dict, l_max: float, cand_fn=None) -> dict:
    """Radiance and alpha of a kernel without records (the production
    query) against the oracle: each ray against the candidate it is closest
    to (ambiguous rays have two; with cand_fn, as in compare, every valid
    outcome of the rays that match neither)."""
    g = np.asarray(rgb, np.float64)
    amb = orc["alt_valid"].astype(bool)
    e_main = rel_err(g, orc["L"], l_max).max(1)
    e_alt = rel_err(g, orc["alt_L"], l_max).max(1)
    use_alt = amb & (e_alt < e_main)
    err = np.where(use_alt, e_alt, e_main)
    ref_a = np.where(use_alt, orc["alt_alpha"], orc["alpha"])
    aerr = np.abs(np.asarray(alpha, np.float64) - ref_a) if alpha is not None else np.zeros_like(err)
    bad = (err > RTOL) | (aerr > RTOL)
    n_multi = 0
    redo = np.nonzero(bad & ((orc["flags"] & 2) != 0))[0]
    if cand_fn is not None and redo.size:
        sub = {"rgb": g[redo], "alpha": None if alpha is None else np.asarray(alpha)[redo]}
        ok = match_candidates(sub, cand_fn(redo), l_max, RTOL, records=False)
        bad[redo[ok]] = False
        err[redo[ok]] = 0.0
        aerr[redo[ok]] = 0.0
        n_multi = int(ok.sum())
    return {"n": len(err), "max_rel": float(err.max()) if len(err) else 0.0,
            "max_alpha_err": float(aerr.max()) if len(err) else 0.0,
            "n_bad": int(bad.sum()), "n_alt": int(use_alt.sum()), "n_multi": n_multi}


class Tally:
    """Sums parity reports over the chunks of a large batch."""

    def __init__(self):
        self.r = {"n": 0, "n_bad": 0, "n_seq_mismatch": 0, "n_steps_mismatch": 0, "n_alt": 0,
                  "n_multi": 0, "n_ambiguous": 0, "n_exact": 0, "max_rel": 0.0, "max_alpha_err": 0.0}
        self.bad_examples = []

    def add(self, rep: dict, offset: int = 0):
        for k in ("n", "n_bad", "n_seq_mismatch", "n_steps_mismatch", "n_alt", "n_multi", "n_ambiguous",
                  "n_exact"):
            self.r[k] += int(rep.get(k, 0))
        for k in ("max_rel", "max_alpha_err"):
            self.r[k] = max(self.r[k], float(rep.get(k, 0.0)))
        if "bad_idx" in rep and len(self.bad_examples) < 20:
            self.bad_examples += [int(i) + offset for i in rep["bad_idx"][:20 - len(self.bad_examples)]]

    @property
    def ok(self) -> bool:
        return self.r["n_bad"] == 0 and self.r["n"] > 0

    def __repr__(self):
        return repr({**self.r, "bad_examples": self.bad_examples})


def to_numpy(d: dict) -> dict:
    return {k: v.cpu().numpy() for k, v in d.items()}


def oracle_for(tree, o, d, model, flags_gpu: int, storage="f32", max_ids=0):
    opts = 0
    if flags_gpu & 1:
        opts |= core.NO_STOP
    if flags_gpu & 4:
        opts |= core.NO_SKIP
    return core.query(tree, o, d, model=model, opts=opts, storage=storage, max_ids=max_ids)
