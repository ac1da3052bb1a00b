"""Every ray of the full-size batches against the oracle (through the C ABI).

The depth-9 luminaire (6.2M data leaves, SH degree 2) is queried with the
4,194,304 camera rays and the 16,777,216 incoherent room rays in float32,
float16 and bfloat16 storage, in the launches the benchmark times.  For
every ray:

  * the validation trace over the full table: leaf count, ordered hash of
    the Morton ids, stop index and number of octree nodes visited equal to
    the oracle's (Sec. 5; Sec. 6.2 heuristics), radiance and alpha within
    1e-4 (Sec. 4.1, Eqs. 3-5);
  * the trace over the sigma_min-pruned table that the production query
    marches, against the oracle on the same pruned tree with the skip off:
    the same records, bit for bit;
  * the production query (camera batches through the camera-batch entry
    point): radiance and alpha within 1e-4 of the oracle.

A ray whose alpha_max test lands within 1e-4 of the threshold has more than
one valid outcome (stop there or continue; with several such tests, stop at
any of them or continue through all); it must match one of them.  For the 16-bit storages the
error against the float32 tree (the storage error) is stated.

The uneven multi-luminaire batch (16 trees of depth 6-10, SH degree 3,
float16) is checked the same way on every ray of its one persistent launch,
with the records of the three depth-10 trees.
"""
import sys
import time

import numpy as np
import pytest

import inputs
from oracle import core
from tests import parity

pytestmark = pytest.mark.gpu

CHUNK = 1 << 21
_F32_L = {}          # oracle radiance on the float32 tree, per workload


def _say(msg):
    print(f"[gpu] {msg}", flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def lq():
    import torch
    import paper_2207_05009_amd as lq
    assert torch.cuda.is_available()
    lq.lib()
    return lq


@pytest.fixture(scope="module")
def full_rays():
    return {"camera": inputs.rays.pinhole(2048, 2048), "room": inputs.rays.room_to_proxy(1 << 24, 20)}


def _dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


@pytest.mark.parametrize("storage", ["f32", "f16", "bf16"])
@pytest.mark.parametrize("workload", ["camera", "room"])
def test_every_ray_full_size(lq, c1_tree, full_rays, workload, storage):
    import torch
    o, d = full_rays[workload]
    n = len(o)
    lmax = c1_tree.l_max
    _say(f"every ray: {workload} batch, {n} rays, depth-9 tree in {storage}")
    t0 = time.perf_counter()
    oct_ = lq.Octree(c1_tree, storage)
    O, D = _dev(o), _dev(d)
    tr = parity.to_numpy(oct_.trace(O, D, model="linear"))
    trp = parity.to_numpy(oct_.trace(O, D, model="linear", flags=lq.LQ_TRACE_PRUNED))
    if workload == "camera":
        rgb, alpha = oct_.query_image(O, D, 2048, 2048, model="linear")
    else:
        rgb, alpha = oct_.query(O, D, model="linear")
    torch.cuda.synchronize()
    rgb, alpha = rgb.cpu().numpy(), alpha.cpu().numpy()
    oct_.free()
    del O, D
    # the trace of the pruned table computes what the production kernel does
    same = (trp["rgb"] == rgb).all(1) & (trp["alpha"] == alpha)
    assert float(same.mean()) > 0.9999, float(same.mean())
    assert parity.rel_err(trp["rgb"].astype(np.float64), rgb.astype(np.float64), lmax).max() < 1e-6
    _say(f"GPU launches done in {time.perf_counter() - t0:.1f} s")

    P = core.PreparedTree(c1_tree, storage)
    PP = core.PreparedTree(core.pruned_tree(c1_tree, storage), storage)
    full, pruned, plain = parity.Tally(), parity.Tally(), parity.Tally()
    L32 = _F32_L.setdefault(workload, np.zeros((n, 3))) if storage == "f32" else _F32_L.get(workload)
    for s in range(0, n, CHUNK):
        sl = slice(s, min(n, s + CHUNK))
        oc, dc = o[sl], d[sl]
        orc = core.query(c1_tree, oc, dc, model=core.LINEAR, prepared=P)

        def cands(idx):
            return core.candidates(None, oc[idx], dc[idx], model=core.LINEAR, prepared=P)

        def cands_pruned(idx):
            return core.candidates(None, oc[idx], dc[idx], model=core.LINEAR, opts=core.NO_SKIP, prepared=PP)

        full.add(parity.compare({k: v[sl] for k, v in tr.items()}, orc, lmax, ids=False, cand_fn=cands), s)
        plain.add(parity.match_plain(rgb[sl], alpha[sl], orc, lmax, cand_fn=cands), s)
        if storage == "f32":
            L32[sl] = orc["L"]
        del orc
        orcp = core.query(None, oc, dc, model=core.LINEAR, opts=core.NO_SKIP, prepared=PP)
        pruned.add(parity.compare({k: v[sl] for k, v in trp.items()}, orcp, lmax, ids=False,
                                  cand_fn=cands_pruned), s)
        del orcp
    _say(f"{workload} {storage} full-table trace: {full}")
    _say(f"{workload} {storage} pruned-table trace: {pruned}")
    _say(f"{workload} {storage} production query: {plain}")
    _say(f"oracle passes done in {time.perf_counter() - t0:.1f} s")
    if storage != "f32" and L32 is not None:
        e = parity.rel_err(rgb.astype(np.float64), L32, lmax).max(1)
        rl2 = float(np.linalg.norm(rgb - L32) / np.linalg.norm(L32))
        _say(f"{workload} {storage} storage error vs the float32 tree (every ray): median "
             f"{np.median(e):.2e} p99 {np.quantile(e, 0.99):.2e} max {e.max():.2e} rel-L2 {rl2:.2e}")
    assert full.ok, full
    assert pruned.ok, pruned
    assert plain.ok, plain


def test_uneven_batch_every_ray(lq):
    """The uneven multi-luminaire batch in its one persistent launch: every
    ray's radiance and alpha against the oracle on its tree (float16
    storage, SH degree 3), and the leaf records of the three depth-10 trees
    (1024^3 cells, about 2.5e7 leaves each) from the trace kernel."""
    import torch
    from inputs import uneven
    t0 = time.perf_counter()
    trees = uneven.trees(progress=_say)
    o, d, offs = uneven.batch_rays()
    _say(f"uneven batch: {len(trees)} trees, {len(o)} rays, ready in {time.perf_counter() - t0:.0f} s")
    octs = [lq.Octree(t, "f16") for t in trees]
    O, D = _dev(o), _dev(d)
    rgb, alpha = lq.query_multi(octs, offs, O, D, model="linear")
    torch.cuda.synchronize()
    rgb, alpha = rgb.cpu().numpy(), alpha.cpu().numpy()
    traces = {}
    for k, t in enumerate(trees):
        if t.depth == 10:
            sl = slice(int(offs[k]), int(offs[k + 1]))
            traces[k] = parity.to_numpy(octs[k].trace(O[sl], D[sl], model="linear"))
    torch.cuda.synchronize()
    for oc in octs:
        oc.free()
    del O, D
    plain, records = parity.Tally(), parity.Tally()
    for k, t in enumerate(trees):
        sl = slice(int(offs[k]), int(offs[k + 1]))
        P = core.PreparedTree(t, "f16")
        ok_, dk_ = o[sl], d[sl]
        orc = core.query(t, ok_, dk_, model=core.LINEAR, prepared=P)

        def cands(idx):
            return core.candidates(None, ok_[idx], dk_[idx], model=core.LINEAR, prepared=P)

        rep = parity.match_plain(rgb[sl], alpha[sl], orc, t.l_max, cand_fn=cands)
        plain.add(rep, int(offs[k]))
        if k in traces:
            r = parity.compare(traces[k], orc, t.l_max, ids=False, cand_fn=cands)
            records.add(r, int(offs[k]))
            _say(f"tree {k} (depth 10, {t.n_leaves} leaves, {sl.stop - sl.start} rays): records {r['n_bad']} bad, "
                 f"{r['n_ambiguous']} ambiguous, max rel {r['max_rel']:.2e}")
        del orc, P
    _say(f"uneven batch, one launch: {plain}")
    _say(f"uneven batch, depth-10 records: {records}")
    assert len(traces) == 3
    assert plain.ok, plain
    assert records.ok, records
