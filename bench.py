#!/usr/bin/env python3
"""Throughput of the luminaire emission query on one MI355X.

Workload (one step = one launch of the whole query over the batch, inputs
resident in HBM): the depth-9 synthetic luminaire plenoctree (512^3 cells,
~6.2M data leaves, SH degree 2, float32 storage, 16 density blobs + 4 thin
shells) and the 4,194,304 rays of a 2048x2048 pinhole camera at distance 3
with a 40 degree field of view; linear transmittance, sigma_min = 0.1,
alpha_max = 0.9.

Prints one JSON line (rays/s) with the dominant kernel's roofline fraction
(algorithmic bytes per launch / measured launch time vs 8 TB/s; the bytes
are counted on the table the timed kernel marches) and the CPU oracle's
throughput on a bounded sample of the same rays.  Extra variants
(float16/bfloat16 storage, exponential transmittance, incoherent room
queries, the learned surrogate with octree fallback, the consumer side, the
uneven 16-luminaire batch) are reported under "variants".

The CPU leg is the only part that runs the oracle: it times it, and it
compares the GPU outputs of every variant, on a seeded sample of its rays,
with it (the "error" records), and states the bias of the render
heuristics (sigma_min skip and alpha_max stop) on the camera and room rays.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "rays/s: octree radiance query FP32 vs FP16 vs MLP surrogate at ≤1% rel err"
HBM_PEAK_GBS = 8000.0
ALU_PEAK_TFLOPS = 78.6      # vector FMA without packed float32 (= the FP64 rate)
PROFILE_DIR = os.path.join(ROOT, "profiles")
CSRC = os.path.join(ROOT, "paper_2207_05009_amd", "csrc")


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def kernel_sources_hash():
    """Hash of the sources the query kernel is built from."""
    h = hashlib.sha1()
    for name in ("octree_kernels.h", "octree_query_f32.hip", "march.h", "lq_internal.h"):
        with open(os.path.join(CSRC, name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:12]


def time_launches(fn, steps, warmup):
    import torch
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    start = torch.cuda.Event(enable_timing=True)
    end = torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    start.record()
    for _ in range(steps):
        fn()
    end.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    return start.elapsed_time(end) / steps, wall


def alg_bytes(trace, K, elem_bytes):
    """Bytes the method must move per launch, counted on the table the
    production query marches (a trace with LQ_TRACE_PRUNED: only the leaves
    it composites, the nodes of that table it visits): rays in (24 B), RGB +
    alpha out (16 B), per composited leaf its density and 3K SH coefficients,
    one 4-byte child slot per octree node visited."""
    n = trace["count"].numel()
    comp = int(trace["n_comp"].sum())
    steps = int(trace["n_steps"].sum())
    return 40 * n + comp * (1 + 3 * K) * elem_bytes + steps * 4, {
        "rays": n, "mean_composited": comp / n, "mean_nodes": steps / n}


def alg_bytes_full_table(trace, K, elem_bytes):
    """The same formula on the full table (the validation trace): a density
    per data leaf visited, including those below sigma_min that the
    production query never reads, and the nodes of the full table."""
    n = trace["count"].numel()
    occ = int(trace["count"].sum())
    comp = int(trace["n_comp"].sum())
    steps = int(trace["n_steps"].sum())
    return 40 * n + occ * elem_bytes + comp * 3 * K * elem_bytes + steps * 4, {
        "rays": n, "mean_leaves": occ / n, "mean_composited": comp / n, "mean_nodes": steps / n}


def variant_record(lumiq, oc, o, d, model, K, elem_bytes, vms, traffic_tag=None):
    """rays/s of a timed query launch and its algorithmic bytes against the
    HBM peak (per-ray counts from a trace of the pruned table over the same
    rays), plus the measured HBM bytes per launch where a counter summary
    exists."""
    n = o.shape[0]
    nbytes, counts = alg_bytes(oc.trace(o, d, model=model, flags=lumiq.LQ_TRACE_PRUNED), K, elem_bytes)
    achieved = nbytes / (vms * 1e-3) / 1e9
    rec = {"rays_per_s": n / (vms * 1e-3), "ms_per_step": vms, "alg_bytes_per_launch": nbytes,
           "achieved_gbs": round(achieved, 1), "roofline_frac": round(achieved / HBM_PEAK_GBS, 4),
           "per_ray": counts}
    if traffic_tag:
        rec["traffic"] = traffic_from_profiles(traffic_tag)
    return rec


def traffic_from_profiles(kernel_tag):
    """HBM bytes per launch from the committed rocprofv3 counter summary
    (lines "key: value"), if it was taken on the current kernel sources
    (else None)."""
    p = os.path.join(PROFILE_DIR, f"traffic_{kernel_tag}.txt")
    if not os.path.exists(p):
        return None
    try:
        kv = {}
        for line in open(p):
            if ":" in line and not line.startswith("#"):
                k, v = line.split(":", 1)
                kv[k.strip()] = v.strip()
        if kv.get("kernel_src_sha1") != kernel_sources_hash():
            return None
        return float(kv["hbm_bytes_per_launch"])
    except Exception:
        return None


def host_info():
    """The host the CPU leg runs on: logical CPUs, the CPUs this process may
    run on (affinity and cgroup quota), OMP_NUM_THREADS and the CPU model."""
    info = {"nproc": os.cpu_count(), "omp_num_threads": os.environ.get("OMP_NUM_THREADS")}
    try:
        info["affinity"] = len(os.sched_getaffinity(0))
    except Exception:
        info["affinity"] = os.cpu_count()
    info["cgroup_cpu_quota"] = None
    try:
        q, per = open("/sys/fs/cgroup/cpu.max").read().split()[:2]
        if q != "max":
            info["cgroup_cpu_quota"] = float(q) / float(per)
    except Exception:
        pass
    info["cpu_model"] = None
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                info["cpu_model"] = line.split(":", 1)[1].strip()
                break
    except Exception:
        pass
    usable = info["affinity"] or 1
    if info["cgroup_cpu_quota"]:
        usable = min(usable, max(1, int(info["cgroup_cpu_quota"])))
    info["usable_cores"] = usable
    return info


def cpu_baseline(tree, o, d, budget_s):
    """The FP64 oracle on every core this process may use, on a seeded
    sample of the rays, chunk by chunk until the time budget is spent; then
    the same oracle on one thread for a fifth of the budget."""
    import numpy as np
    from oracle import core
    host = host_info()
    threads = host["usable_cores"]
    P = core.PreparedTree(tree, "f32")
    rng = np.random.default_rng(123)
    order = rng.permutation(len(o))

    def run(n_threads, budget, chunk):
        done, t_total = 0, 0.0
        while done < len(o) and t_total < budget:
            idx = np.sort(order[done: done + chunk])
            t0 = time.perf_counter()
            core.query(tree, o[idx], d[idx], model=core.LINEAR, prepared=P, n_threads=n_threads)
            t_total += time.perf_counter() - t0
            done += len(idx)
        return done, t_total

    done, t_total = run(threads, budget_s, 131072)
    done1, t1 = run(1, budget_s / 5.0, 8192)
    # the surrogate's FP64 oracle (numpy forward pass) on room rays, for context
    import inputs
    from oracle import mlp as omlp
    ro, rd = inputs.rays.room_to_proxy(65536, 21)
    theta = omlp.he_uniform(31)
    t0 = time.perf_counter()
    omlp.predict(theta, ro, rd)
    t_mlp = time.perf_counter() - t0
    return {"value": done / t_total, "unit": "rays/s", "cores": threads, "kind": "oracle",
            "sample": f"{done} of the {len(o)} camera rays (seeded random subset), FP64 oracle "
                      f"with its OpenMP loop over rays on {threads} threads, {t_total:.1f} s",
            "host": host,
            "one_thread": {"value": done1 / t1, "unit": "rays/s", "sample": f"{done1} rays, {t1:.1f} s"},
            "surrogate_oracle": {"value": len(ro) / t_mlp, "unit": "rays/s",
                                 "sample": f"{len(ro)} room rays, numpy FP64 forward, {t_mlp:.2f} s"}}


ERROR_SAMPLE = 20000


def sample_index(n, seed):
    import numpy as np
    m = min(n, ERROR_SAMPLE)
    return np.sort(np.random.default_rng(seed).choice(n, m, replace=False))


def keep_sample(samples, name, rgb, alpha, idx, **meta):
    """Keep the GPU outputs of a variant on a seeded sample of its rays for
    the CPU leg's error records."""
    import torch
    it = torch.from_numpy(idx).to(rgb.device)
    samples[name] = {"idx": idx, "rgb": rgb[it].cpu().numpy(),
                     "alpha": None if alpha is None else alpha[it].cpu().numpy(), **meta}


def error_records(samples, trees, rays):
    """Error of every sampled variant against the FP64 oracle (each ray
    against the nearer of its candidates when its alpha_max test is within
    1e-4 of the threshold), on the tree as stored; for float16 / bfloat16
    storage also the storage error against the float32 tree; for the
    surrogate against the oracle on the float32 tree.  Per ray and channel
    the error is |L - L_ref| / max(|L_ref|, 1e-6 L_max)."""
    import numpy as np
    from oracle import core
    out, cache = {}, {}

    def oracle(tree_key, storage, model, ray_key, idx):
        key = (tree_key, storage, model, ray_key)
        if key not in cache:
            o, d = rays[ray_key]
            cache[key] = core.query(trees[tree_key], o[idx], d[idx], model=model, storage=storage)
        return cache[key]

    def stats(rgb, alpha, orc, lmax):
        g = np.asarray(rgb, np.float64)
        fl = 1e-6 * lmax
        e_main = (np.abs(g - orc["L"]) / np.maximum(np.abs(orc["L"]), fl)).max(1)
        e_alt = (np.abs(g - orc["alt_L"]) / np.maximum(np.abs(orc["alt_L"]), fl)).max(1)
        alt = orc["alt_valid"].astype(bool) & (e_alt < e_main)
        err = np.where(alt, e_alt, e_main)
        ref = np.where(alt[:, None], orc["alt_L"], orc["L"])
        rec = {"rays": int(len(err)), "max_rel": float(err.max()), "p99_rel": float(np.quantile(err, 0.99)),
               "median_rel": float(np.median(err)),
               "rel_l2": float(np.linalg.norm(g - ref) / max(np.linalg.norm(ref), 1e-300)),
               "n_ambiguous": int(orc["alt_valid"].sum())}
        if alpha is not None:
            ra = np.where(alt, orc["alt_alpha"], orc["alpha"])
            rec["max_alpha_err"] = float(np.abs(np.asarray(alpha, np.float64) - ra).max())
        return rec

    for name, smp in samples.items():
        idx, kind = smp["idx"], smp.get("kind", "octree")
        if kind == "floor":
            out[name] = floor_error(trees["c1"], smp)
            continue
        if kind == "distill":
            out[name] = distill_error(smp)
            continue
        if kind == "uneven":
            recs = []
            tk = smp["tree_of"]
            for k in np.unique(tk):
                sel = tk == k
                o, d = rays["uneven"]
                orc = core.query(trees[("uneven", int(k))], o[idx[sel]], d[idx[sel]], model=core.LINEAR,
                                 storage="f16")
                recs.append((sel, orc))
            L = np.zeros((len(idx), 3))
            A = np.zeros(len(idx))
            merged = {"L": L, "alt_L": np.zeros_like(L), "alpha": A, "alt_alpha": np.zeros_like(A),
                      "alt_valid": np.zeros(len(idx), np.uint8)}
            for sel, orc in recs:
                for key in merged:
                    merged[key][sel] = orc[key]
            rec = stats(smp["rgb"], smp["alpha"], merged, 2048.0)
            rec["vs"] = "FP64 oracle on each luminaire's float16 tree"
            out[name] = rec
            continue
        model = core.EXP if smp.get("model") == "exp" else core.LINEAR
        tree_key, storage, ray_key = smp["tree"], smp.get("storage", "f32"), smp["rays"]
        lmax = trees[tree_key].l_max
        if kind == "surrogate":
            ref = oracle(tree_key, "f32", core.LINEAR, ray_key, idx)
            g = np.asarray(smp["rgb"], np.float64)
            err = (np.abs(g - ref["L"]) / np.maximum(np.abs(ref["L"]), 1e-6 * lmax)).max(1)
            out[name] = {"rays": int(len(g)), "vs": "FP64 oracle on the float32 tree",
                         "rel_l2": float(np.linalg.norm(g - ref["L"]) / np.linalg.norm(ref["L"])),
                         "p99_rel": float(np.quantile(err, 0.99)), "median_rel": float(np.median(err))}
            continue
        rec = stats(smp["rgb"], smp["alpha"], oracle(tree_key, storage, model, ray_key, idx), lmax)
        rec["vs"] = f"FP64 oracle on the tree as stored ({storage})"
        if storage != "f32":
            ref = oracle(tree_key, "f32", model, ray_key, idx)
            g = np.asarray(smp["rgb"], np.float64)
            e = (np.abs(g - ref["L"]) / np.maximum(np.abs(ref["L"]), 1e-6 * lmax)).max(1)
            rec["storage_error_vs_f32_tree"] = {
                "max_rel": float(e.max()), "p99_rel": float(np.quantile(e, 0.99)),
                "median_rel": float(np.median(e)),
                "rel_l2": float(np.linalg.norm(g - ref["L"]) / np.linalg.norm(ref["L"]))}
        out[name] = rec
    return out


def floor_error(tree, smp):
    """Irradiance of a seeded sample of floor points against the oracle on
    the same points and sample numbers (uniform or guided by the GPU's guide
    weights): per point, the largest channel error relative to max(|E_ref|,
    the point's mean sample weight x 1e-6 L_max); a point with a
    threshold-ambiguous sample ray is compared with the nearer of its two
    sums (main and alternative candidates)."""
    import numpy as np
    from oracle import shade
    if "guide" in smp:
        orc = shade.proxy_irradiance_guided(tree, smp["pts"], smp["nrm"], smp["u"], smp["guide"], smp["G"],
                                            smp["beta"], background=smp["bg"], D=smp["D"])
    else:
        orc = shade.proxy_irradiance(tree, smp["pts"], smp["nrm"], smp["u"], background=smp["bg"])
    g = np.asarray(smp["E"], np.float64)
    alt_E = orc["terms_alt"].mean(axis=1)
    fl = orc["w"].mean(axis=1)[:, None] * 1e-6 * tree.l_max + 1e-30
    e_main = (np.abs(g - orc["E"]) / np.maximum(np.abs(orc["E"]), fl)).max(1)
    e_alt = (np.abs(g - alt_E) / np.maximum(np.abs(alt_E), fl)).max(1)
    amb = orc["alt_valid"].any(axis=1)
    err = np.where(amb, np.minimum(e_main, e_alt), e_main)
    return {"points": int(len(g)), "samples_per_point": int(smp["u"].shape[1]), "max_rel": float(err.max()),
            "p99_rel": float(np.quantile(err, 0.99)), "median_rel": float(np.median(err)),
            "n_ambiguous_points": int(amb.sum()),
            "vs": "FP64 oracle (sample rays, query, blend, per-point mean) on the same points and numbers"}


def distill_error(smp):
    """Means of a seeded sample of distilled voxels against the oracle's
    256-sample means of the same voxels: relative errors with floors 1e-3
    (density) and 1e-2 (SH coefficients)."""
    import numpy as np
    from oracle import distill as od
    f = od.field_from_params(smp["params"])
    sig, sh = od.average_samples(f, smp["depth"], smp["codes"], 256, smp["seed"])
    es = np.abs(smp["sigma"].astype(np.float64) - sig) / np.maximum(np.abs(sig), 1e-3)
    eh = np.abs(smp["sh"].astype(np.float64).reshape(sh.shape) - sh) / np.maximum(np.abs(sh), 1e-2)
    return {"voxels": int(len(sig)), "density_max_rel": float(es.max()), "sh_max_rel": float(eh.max()),
            "sh_median_rel": float(np.median(eh)), "vs": "FP64 oracle means of the same voxels"}


def heuristic_bias(tree, rays):
    """Bias of the render heuristics (Sec. 6.2: sigma_min skip, alpha_max
    stop) on a seeded sample of each ray set: the oracle with them (L)
    against the oracle without them (L*, the exact integral of the
    piecewise-constant field)."""
    import numpy as np
    from oracle import core
    out = {}
    for key, (o, d) in rays.items():
        idx = sample_index(len(o), 17)
        L = core.query(tree, o[idx], d[idx], model=core.LINEAR)
        F = core.query(tree, o[idx], d[idx], model=core.LINEAR, opts=core.NO_SKIP | core.NO_STOP)
        fl = 1e-6 * tree.l_max
        e = (np.abs(L["L"] - F["L"]) / np.maximum(np.abs(F["L"]), fl)).max(1)
        out[key] = {"rays": int(len(idx)),
                    "rel_l2": float(np.linalg.norm(L["L"] - F["L"]) / np.linalg.norm(F["L"])),
                    "median_rel": float(np.median(e)), "p99_rel": float(np.quantile(e, 0.99)),
                    "max_rel": float(e.max()),
                    "mean_alpha": float(L["alpha"].mean()), "mean_alpha_exact": float(F["alpha"].mean()),
                    "mean_composited": float(L["n_comp"].mean()), "mean_composited_exact": float(F["n_comp"].mean())}
    return out


def surrogate_variant(args, lumiq, tree, oct32, qo, qd, qref_buf, samples=None, sample_idx=None):
    """Learned surrogate: trained on (ray, radiance) pairs that the float32
    octree renders for incoherent room rays, trust map from held-out pairs
    at 1% relative error (30,000,000 held-out rays), then inference with
    octree fallback on the 16,777,216 room rays."""
    import torch
    import inputs
    t0 = time.perf_counter()
    o, d = inputs.rays.room_to_proxy(args.surrogate_pairs, 30)
    ho, hd = inputs.rays.room_to_proxy(30_000_000, 32)
    o, d, ho, hd = [torch.from_numpy(x).cuda() for x in (o, d, ho, hd)]
    rgb, _ = oct32.query(o, d)
    hrgb, _ = oct32.query(ho, hd)
    qref, _ = oct32.query(qo, qd)
    torch.cuda.synchronize()
    log(f"surrogate data: {time.perf_counter() - t0:.1f} s")
    sur = lumiq.Surrogate(seed=31)
    lr0 = 5e-3
    t0 = time.perf_counter()
    losses = sur.train(o, d, rgb, steps=args.surrogate_steps, total_steps=args.surrogate_steps,
                       batch=65536, lr0=lr0, lr1=lr0 / 100)
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t0
    sur.build_trust(ho, hd, hrgb, max_rel_err=0.01)
    del o, d, rgb, ho, hd, hrgb
    n = qo.shape[0]
    out = torch.empty_like(qref)
    ms_fwd, _ = time_launches(lambda: sur.forward(qo, qd, rgb=out), 10, 2)
    pred = out.clone()
    used = torch.empty((n,), dtype=torch.uint8, device="cuda")

    def hybrid():
        lumiq.check(lumiq._mlp_lib().lq_mlp_infer(sur.handle, oct32.handle, lumiq._ptr(qo),
                                                  lumiq._ptr(qd), n, lumiq._ptr(out),
                                                  lumiq._ptr(used), lumiq._stream(None)))

    ms_hyb, _ = time_launches(hybrid, 10, 2)
    ms_oct, _ = time_launches(lambda: oct32.query(qo, qd, rgb=qref_buf), 10, 2)
    torch.cuda.synchronize()

    def rel_l2(a, b):
        return float(torch.linalg.norm((a - b).double()) / torch.linalg.norm(b.double()))

    if samples is not None:
        keep_sample(samples, "surrogate_only", pred, None, sample_idx, kind="surrogate", tree="c1", rays="room")
        keep_sample(samples, "surrogate_with_fallback", out, None, sample_idx, kind="surrogate", tree="c1",
                    rays="room")
    res = {
        "train_steps": args.surrogate_steps, "train_pairs": args.surrogate_pairs, "batch": 65536,
        "lr": [lr0, lr0 / 100], "train_s": round(t_train, 2),
        "loss_first": float(losses[:20].mean()), "loss_last": float(losses[-200:].mean()),
        "surrogate_only": {"rays_per_s": n / (ms_fwd * 1e-3), "ms": ms_fwd,
                           "rel_l2_vs_octree_f32": rel_l2(pred, qref)},
        "surrogate_with_fallback": {"rays_per_s": n / (ms_hyb * 1e-3), "ms": ms_hyb,
                                    "rel_l2_vs_octree_f32": rel_l2(out, qref),
                                    "fallback_fraction": float(used.float().mean())},
        "octree_f32_same_rays": {"rays_per_s": n / (ms_oct * 1e-3), "ms": ms_oct},
        "flop_per_ray": 41344,
        "mfma_frac_surrogate_only": 41344 * n / (ms_fwd * 1e-3) / 2.5e15,
    }
    log(f"surrogate: {res}")
    return res


UNEVEN_SURROGATE_STEPS = 5000


def sh_sweep_variant(lumiq, o, d, steps):
    """Cost of the SH degree and of the transmittance model: the depth-9
    luminaire's geometry with SH degree 0..4 (one degree-4 tree, lower
    degrees by keeping its first (l+1)^2 coefficients, so every degree sees
    the same leaves), camera rays, float32 and float16 storage."""
    import dataclasses
    import inputs
    t0 = time.perf_counter()
    full = inputs.cached_tree(dataclasses.replace(inputs.C1_TREE, sh_degree=4))
    log(f"SH sweep: degree-4 tree ready in {time.perf_counter() - t0:.1f} s")
    out = {}
    for deg in range(5):
        K = (deg + 1) ** 2
        tree = dataclasses.replace(full, sh_degree=deg, sh=full.sh[:, :, :K].copy())
        for storage in ("f32", "f16"):
            oc = lumiq.Octree(tree, storage)
            rec = {}
            for model in ("linear", "exp"):
                ms, _ = time_launches(lambda: oc.query_image(o, d, 2048, 2048, model=model), steps, 2)
                rec[f"{model}_ms"] = ms
            rec["linear_speedup_over_exp"] = rec["exp_ms"] / rec["linear_ms"]
            out[f"deg{deg}_{storage}"] = rec
            log(f"SH sweep: degree {deg} {storage}: linear {rec['linear_ms']:.3f} ms, exp {rec['exp_ms']:.3f} ms")
            oc.free()
    return out


SHADE_SAMPLE = 300   # floor points (and distilled voxels) the CPU leg checks


def floor_variant(inputs, oct32, steps, samples=None):
    """The consumer side: irradiance from the luminaire's proxy (emission plus
    background through it) on a 1024 x 1024 floor grid 0.5 below the proxy,
    16 uniform proxy samples per point, one call per step (sample rays, the
    query over them, the per-point blend and sum)."""
    import numpy as np
    import torch
    pts, nrm = inputs.rays.floor_points(1024, 1024)
    u = inputs.rays.sample_numbers(len(pts), 16, 5)
    P, N, U = (torch.from_numpy(a).cuda() for a in (pts, nrm, u))
    E = torch.empty((len(pts), 3), device="cuda")
    ms, _ = time_launches(lambda: oct32.proxy_irradiance(P, N, U, background=(0.05, 0.05, 0.08), irradiance=E),
                          steps, 2)
    n_rays = len(pts) * 16
    if samples is not None:
        idx = np.sort(np.random.default_rng(41).choice(len(pts), SHADE_SAMPLE, replace=False))
        samples["floor_irradiance"] = {"kind": "floor", "idx": idx, "E": E.cpu().numpy()[idx],
                                       "pts": pts[idx], "nrm": nrm[idx], "u": u[idx], "bg": (0.05, 0.05, 0.08)}
    rec = {"points": len(pts), "samples_per_point": 16, "ms": ms, "points_per_s": len(pts) / (ms * 1e-3),
           "sample_rays_per_s": n_rays / (ms * 1e-3)}
    log(f"floor irradiance: {ms:.3f} ms for {n_rays} sample rays")
    return rec


QUALITY_POINTS, QUALITY_SAMPLES = 4096, 4096
GUIDE_DIRS = 2   # direction bins per tangent axis of the benchmarked guide (2 x 2 per cell)
GUIDE_PROBES = 256   # probe rays per cell of the benchmarked guide


def guided_variant(inputs, oct32, steps, samples=None):
    """Radiance-field-guided proxy sampling on the floor grid: the
    direction-binned guide (16 x 16 cells per face, 2 x 2 direction bins,
    256 probe rays per cell, one lq_proxy_guide call) and the guided
    irradiance call (1,048,576 points x 16 samples, the floor workload of
    the uniform variant), timed; then the estimator's quality on 4,096
    random points of the floor at 4,096 samples each: the variance of one
    sample's luminance term (the error of an n-sample estimate is this over
    n, all estimators being unbiased), mean and median over the points, for
    the uniform estimator over the whole proxy, for the guided one with
    defensive share 1 (uniform cells, the face chosen by the geometry mix
    among the faces the point sees), with the direction-averaged guide and
    share 0.5, and with the direction-binned guide and share 0.5 (the timed
    configuration); and the mean z-score of the last against the uniform
    means (near 0 when both estimate the same integral)."""
    import numpy as np
    import torch
    G, R, Q, D = 16, GUIDE_PROBES, QUALITY_SAMPLES, GUIDE_DIRS
    up = torch.from_numpy(inputs.rays.probe_numbers(6 * G * G, R, 90)).cuda()
    w = torch.empty((6 * G * G * D * D,), device="cuda")
    ms_guide, _ = time_launches(lambda: oct32.proxy_guide(G, up, weights=w, dir_res=D), steps, 1)
    w1 = oct32.proxy_guide(G, up)
    pts, nrm = inputs.rays.floor_points(1024, 1024)
    u = inputs.rays.sample_numbers(len(pts), 16, 5)
    P, N, U = (torch.from_numpy(a).cuda() for a in (pts, nrm, u))
    E = torch.empty((len(pts), 3), device="cuda")
    bg = (0.05, 0.05, 0.08)
    ms, _ = time_launches(lambda: oct32.proxy_irradiance_guided(P, N, U, w, G, defensive=0.5, background=bg,
                                                                irradiance=E, dir_res=D), steps, 2)
    if samples is not None:
        idx = np.sort(np.random.default_rng(42).choice(len(pts), SHADE_SAMPLE, replace=False))
        samples["floor_irradiance_guided"] = {"kind": "floor", "idx": idx, "E": E.cpu().numpy()[idx],
                                              "pts": pts[idx], "nrm": nrm[idx], "u": u[idx], "bg": bg,
                                              "guide": w.cpu().numpy(), "G": G, "beta": 0.5, "D": D}
    # quality: 4,096 seeded random floor points, 4,096 samples each (the
    # per-point variance of a heavy-tailed term needs many samples; mean and
    # median over the points)
    sub = np.sort(np.random.default_rng(44).choice(len(pts), QUALITY_POINTS, replace=False))
    Ps, Ns = P[sub].contiguous(), N[sub].contiguous()
    Uq = torch.from_numpy(inputs.rays.sample_numbers(len(sub), Q, 91)).cuda()

    def term_stats(t):
        lum = t.double().mean(-1)
        return lum.mean(1).cpu().numpy(), lum.var(1).cpu().numpy()

    mu, vu = term_stats(oct32.proxy_irradiance(Ps, Ns, Uq, background=bg, want_terms=True)[1])
    _, v1 = term_stats(oct32.proxy_irradiance_guided(Ps, Ns, Uq, w1, G, defensive=1.0, background=bg,
                                                     want_terms=True)[1])
    _, va = term_stats(oct32.proxy_irradiance_guided(Ps, Ns, Uq, w1, G, defensive=0.5, background=bg,
                                                     want_terms=True)[1])
    mh, vh = term_stats(oct32.proxy_irradiance_guided(Ps, Ns, Uq, w, G, defensive=0.5, background=bg,
                                                      want_terms=True, dir_res=D)[1])
    torch.cuda.synchronize()
    z = (mh - mu) / np.maximum(np.sqrt((vu + vh) / Q), 1e-30)
    stats = lambda v: {"mean": float(v.mean()), "median": float(np.median(v))}
    rec = {"grid": G, "direction_bins": f"{D} x {D}", "probes_per_cell": R, "guide_ms": ms_guide,
           "points": len(pts), "samples_per_point": 16, "ms": ms, "points_per_s": len(pts) / (ms * 1e-3),
           "defensive": 0.5,
           "term_variance": {"uniform_whole_proxy": stats(vu), "geometry_only_defensive_1": stats(v1),
                             "direction_averaged_guide_0.5": stats(va), "directional_guide_0.5": stats(vh)},
           "variance_ratio_uniform_over_guided": float(vu.mean() / vh.mean()) if vh.mean() > 0 else None,
           "median_point_variance_ratio_uniform_over_guided": float(np.median(vu / np.maximum(vh, 1e-300))),
           "variance_ratio_direction_averaged_over_directional": float(va.mean() / vh.mean())
           if vh.mean() > 0 else None,
           "mean_z_guided_vs_uniform": float(z.mean()),
           "quality_sample": f"{len(sub)} random floor points x {Q} samples"}
    log(f"guided floor irradiance: guide {ms_guide:.3f} ms, call {ms:.3f} ms; term variance (mean / median over "
        f"points) uniform {vu.mean():.4g} / {np.median(vu):.4g}, geometry only {v1.mean():.4g} / "
        f"{np.median(v1):.4g}, direction-averaged guide {va.mean():.4g} / {np.median(va):.4g}, "
        f"directional guide {vh.mean():.4g} / {np.median(vh):.4g}; mean z {z.mean():.3f}")
    return rec


DISTILL_SAMPLES = 256


def distill_variant(lumiq, steps, samples=None):
    """Plenoctree distillation (Sec. 5): the continuous field behind the
    depth-9 luminaire (16 blobs + 4 shells, SH degree 2) distilled at 512^3
    with 256 samples per kept voxel, one lq_distill_leaves call per step
    (centre test, compaction, sampling and averaging; the call reads the
    kept count back to size the launch).  The sampling kernel is bound by
    its arithmetic: per sample 24 + 23 n_blobs operations (an FMA counts 2,
    a transcendental 1; 9 of each blob's 23 in FP64, the rest float32).
    Its time is the call's minus that of a counting call (the centre test
    and scan alone); the peak is the chip's vector FMA rate without packed
    float32 math, which is also its FP64 rate: 256 CUs x 4 SIMDs x 16 lanes
    x 2 FLOP x 2.4 GHz = 78.6 TFLOP/s."""
    import torch
    import inputs
    from inputs.trees import field_params
    p = field_params(inputs.C1_TREE)
    codes, sig, sh = lumiq.distill_leaves(p, 9, 0.01, DISTILL_SAMPLES, 2022)
    n = codes.shape[0]
    desc, keep = lumiq.field_desc(p)
    cnt = lumiq.C.c_int64()
    L = lumiq.lib()

    def call():
        lumiq.check(L.lq_distill_leaves(lumiq.C.byref(desc), 9, 0.01, DISTILL_SAMPLES, 2022, 0, n,
                                        lumiq._ptr(codes), lumiq._ptr(sig), lumiq._ptr(sh), lumiq.C.byref(cnt),
                                        lumiq._stream(None)))

    def count():
        lumiq.check(L.lq_distill_leaves(lumiq.C.byref(desc), 9, 0.01, DISTILL_SAMPLES, 2022, 0, 0, None, None,
                                        None, lumiq.C.byref(cnt), lumiq._stream(None)))

    ms, _ = time_launches(call, steps, 2)
    ms_count, _ = time_launches(count, steps, 2)
    if samples is not None:
        import numpy as np
        idx = np.sort(np.random.default_rng(43).choice(n, SHADE_SAMPLE, replace=False))
        samples["distillation"] = {"kind": "distill", "idx": idx, "params": p, "depth": 9, "seed": 2022,
                                   "codes": codes.cpu().numpy().view(np.uint32)[idx].astype(np.uint64),
                                   "sigma": sig.cpu().numpy()[idx], "sh": sh.cpu().numpy()[idx]}
    ms_sample = ms - ms_count
    nb = len(p["radii"])
    flop = n * DISTILL_SAMPLES * (24 + 23 * nb)
    # what the call writes: the centre-test bits of every voxel, then per kept
    # voxel its code, density and 3 x 9 SH coefficients (float32)
    wbytes = (1 << 27) // 8 + n * (4 + 4 + 3 * 9 * 4)
    t0 = time.perf_counter()
    tree = lumiq.octree_from_leaves(9, 2, codes, sig, sh, l_max=p["l_max"])
    torch.cuda.synchronize()
    t_tree = time.perf_counter() - t0
    info = tree.info()
    tree.free()
    rec = {"depth": 9, "voxels": 1 << 27, "kept": int(n), "samples_per_voxel": DISTILL_SAMPLES, "ms": ms,
           "ms_centre_test_and_scan": ms_count, "ms_sampling": ms_sample,
           "samples_per_s": n * DISTILL_SAMPLES / (ms * 1e-3),
           "roofline": {"bound": "alu", "achieved": round(flop / (ms_sample * 1e-3) / 1e12, 2),
                        "peak": ALU_PEAK_TFLOPS, "unit": "TFLOP/s",
                        "frac": round(flop / (ms_sample * 1e-3) / (ALU_PEAK_TFLOPS * 1e12), 4),
                        "flop_per_sample": 24 + 23 * nb},
           "hbm_bytes_written": wbytes, "hbm_write_frac": round(wbytes / (ms * 1e-3) / (HBM_PEAK_GBS * 1e9), 5),
           "octree_build_and_load_s": round(t_tree, 3), "n_nodes": info["n_nodes"]}
    log(f"distillation: {ms:.3f} ms for {n} voxels x {DISTILL_SAMPLES} samples "
        f"(centre test and scan {ms_count:.3f} ms)")
    del keep
    return rec


def uneven_variant(lumiq, samples=None, trees_out=None, rays_out=None):
    """The uneven multi-luminaire batch (16 trees of depth 6 to 10, SH degree
    3, float16, log-uniform ray counts): one persistent launch over all rays
    against one launch per luminaire; load balance = sum of the isolated
    launch times / the one launch's time."""
    import torch
    import inputs
    from inputs import uneven
    t0 = time.perf_counter()
    trees = uneven.trees(progress=log)
    o, d, offs = uneven.batch_rays()
    log(f"uneven batch: {len(trees)} trees ready in {time.perf_counter() - t0:.0f} s, {len(o)} rays")
    octs = [lumiq.Octree(t, "f16") for t in trees]
    ot, dt = torch.from_numpy(o).cuda(), torch.from_numpy(d).cuda()
    n = len(o)
    rgb = torch.empty((n, 3), device="cuda")
    alpha = torch.empty((n,), device="cuda")
    ms_one, _ = time_launches(lambda: lumiq.query_multi(octs, offs, ot, dt, rgb=rgb, alpha=alpha), 10, 3)
    if samples is not None:
        import numpy as np
        idx = sample_index(n, 29)
        keep_sample(samples, "uneven_batch", rgb, alpha, idx, kind="uneven",
                    tree_of=np.searchsorted(offs, idx, side="right") - 1)
        for k, t in enumerate(trees):
            trees_out[("uneven", k)] = t
        rays_out["uneven"] = (o, d)
    iso = []
    for k, oc in enumerate(octs):
        a, b = int(offs[k]), int(offs[k + 1])
        ok, dk, rk, ak = ot[a:b], dt[a:b], rgb[a:b], alpha[a:b]
        ms_k, _ = time_launches(lambda: oc.query(ok, dk, rgb=rk, alpha=ak), 10, 2)
        iso.append(ms_k)
    res = {
        "trees": [{"depth": t.depth, "leaves": int(t.n_leaves), "rays": int(offs[k + 1] - offs[k]),
                   "ms_isolated": round(iso[k], 4)} for k, t in enumerate(trees)],
        "rays": n, "storage": "f16", "sh_degree": 3,
        "ms_one_launch": ms_one, "rays_per_s": n / (ms_one * 1e-3),
        "ms_sum_isolated": sum(iso), "load_balance": sum(iso) / ms_one,
    }
    log(f"uneven batch: one launch {ms_one:.3f} ms, isolated sum {sum(iso):.3f} ms")

    # per-luminaire surrogates (the training recipe of the single luminaire
    # with fewer steps) on the luminaires with at least 2^20 rays, compared
    # with the octree on the same rays
    surr = []
    for k, oc in enumerate(octs):
        a, b = int(offs[k]), int(offs[k + 1])
        if b - a < (1 << 20):
            continue
        to_, td_ = inputs.rays.room_to_proxy(8_000_000, 100 + k)
        ho_, hd_ = inputs.rays.room_to_proxy(24_000_000, 200 + k)
        to_, td_, ho_, hd_ = [torch.from_numpy(x).cuda() for x in (to_, td_, ho_, hd_)]
        trgb, _ = oc.query(to_, td_)
        hrgb, _ = oc.query(ho_, hd_)
        sur = lumiq.Surrogate(seed=31 + k)
        t0 = time.perf_counter()
        sur.train(to_, td_, trgb, steps=UNEVEN_SURROGATE_STEPS, total_steps=UNEVEN_SURROGATE_STEPS,
                  batch=65536, lr0=5e-3, lr1=5e-5)
        torch.cuda.synchronize()
        t_train = time.perf_counter() - t0
        sur.build_trust(ho_, hd_, hrgb, max_rel_err=0.01)
        del to_, td_, trgb, ho_, hd_, hrgb
        ok, dk, nk = ot[a:b], dt[a:b], b - a
        ref = torch.empty((nk, 3), device="cuda")
        out = torch.empty((nk, 3), device="cuda")
        used = torch.empty((nk,), dtype=torch.uint8, device="cuda")
        ms_oct, _ = time_launches(lambda: oc.query(ok, dk, rgb=ref), 10, 2)

        def hybrid():
            lumiq.check(lumiq._mlp_lib().lq_mlp_infer(sur.handle, oc.handle, lumiq._ptr(ok), lumiq._ptr(dk), nk,
                                                      lumiq._ptr(out), lumiq._ptr(used), lumiq._stream(None)))

        ms_h, _ = time_launches(hybrid, 10, 2)
        rel = float(torch.linalg.norm((out - ref).double()) / torch.linalg.norm(ref.double()))
        surr.append({"tree": k, "depth": trees[k].depth, "rays": nk, "train_s": round(t_train, 2),
                     "octree_ms": ms_oct, "hybrid_ms": ms_h, "speedup": ms_oct / ms_h,
                     "rel_l2_vs_octree": rel, "fallback_fraction": float(used.float().mean())})
        log(f"uneven batch: luminaire {k} surrogate {surr[-1]}")
        sur.free()
    res["surrogates"] = {"train_steps": UNEVEN_SURROGATE_STEPS, "train_pairs": 8_000_000,
                         "heldout_pairs": 24_000_000, "per_luminaire": surr}
    for oc in octs:
        oc.free()
    return res


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--cpu-budget", type=float, default=12.0)
    ap.add_argument("--no-variants", action="store_true")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--surrogate-steps", type=int, default=20000,
                    help="optimiser steps of the surrogate (0: skip the surrogate variant)")
    ap.add_argument("--surrogate-pairs", type=int, default=50_000_000)
    ap.add_argument("--sh-sweep", action="store_true",
                    help="also time SH degrees 0..4 x linear/exponential on the depth-9 geometry "
                         "(generates a degree-4 tree: a minute of CPU)")
    ap.add_argument("--no-uneven", action="store_true",
                    help="skip the uneven 16-luminaire batch (it generates three depth-10 trees: a minute "
                         "or more of CPU)")
    ap.add_argument("--copy-probe", action="store_true",
                    help="also run a plain 1 GiB device copy (calibrates HBM byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU: the query shards by rays with no exchange, and this "
              "build runs on a single MI355X (--gpus must be 1)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import inputs
    from paper_2207_05009_amd import lumiq

    if not os.path.exists(lumiq.LIB_PATH):
        import __graft_entry__
        __graft_entry__.build()
    assert torch.cuda.is_available(), "bench.py needs a GPU"

    log("generating the depth-9 tree")
    tree = inputs.cached_tree(inputs.C1_TREE)
    o_np, d_np = inputs.rays.pinhole(2048, 2048)
    n = len(o_np)
    o = torch.from_numpy(o_np).cuda()
    d = torch.from_numpy(d_np).cuda()
    rgb = torch.empty((n, 3), device="cuda")
    alpha = torch.empty((n,), device="cuda")

    oct32 = lumiq.Octree(tree, "f32")
    log(f"tree uploaded: {oct32.info()}")

    # the camera batch goes through the camera-batch entry point (rays taken
    # up in 8x8 pixel tiles; results bit-identical to the batch-order query)
    def step():
        oct32.query_image(o, d, 2048, 2048, model="linear", rgb=rgb, alpha=alpha)

    ms, wall = time_launches(step, args.steps, args.warmup)
    value = n / (ms * 1e-3)
    log(f"f32 linear: {ms:.3f} ms/step, {value / 1e6:.1f} Mrays/s (wall {wall:.3f} s)")

    if args.copy_probe:
        src = torch.ones(1 << 28, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        log("copy probe: 1 GiB read + 1 GiB written")
        del src, dst

    samples = {}
    keep_sample(samples, "headline", rgb, alpha, sample_index(n, 11), tree="c1", rays="camera")
    trp = oct32.trace(o, d, model="linear", flags=lumiq.LQ_TRACE_PRUNED)
    tr = oct32.trace(o, d, model="linear")
    torch.cuda.synchronize()
    nbytes, counts = alg_bytes(trp, tree.K, 4)
    full_bytes, full_counts = alg_bytes_full_table(tr, tree.K, 4)
    del trp, tr
    achieved = nbytes / (ms * 1e-3) / 1e9
    traffic = traffic_from_profiles("query_f32_camera")
    roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
                "alg_bytes_per_launch": nbytes, "per_ray": counts,
                "full_table": {"alg_bytes_per_launch": full_bytes, "per_ray": full_counts,
                               "frac": round(full_bytes / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
                               "note": "counts of the validation trace over the full table (densities of "
                                       "leaves below sigma_min and nodes the timed kernel never visits)"},
                "kernel": "k_query_plain<F32, SH deg 2, sigma_min-pruned table, linear, 8x8 pixel tiles>",
                "kernel_sources": kernel_sources_hash()}

    variants = {}
    trees = {"c1": tree}
    rays = {"camera": (o_np, d_np)}
    if not args.no_variants:
        for storage in ("f16", "bf16"):
            oc = lumiq.Octree(tree, storage)
            vms, _ = time_launches(lambda: oc.query_image(o, d, 2048, 2048, model="linear", rgb=rgb, alpha=alpha),
                                   max(5, args.steps // 2), 2)
            keep_sample(samples, f"camera_{storage}_linear", rgb, alpha, sample_index(n, 11), tree="c1",
                        rays="camera", storage=storage)
            variants[f"camera_{storage}_linear"] = variant_record(lumiq, oc, o, d, "linear", tree.K, 2, vms)
            log(f"{storage}: {vms:.3f} ms/step")
            oc.free()
        vms, _ = time_launches(lambda: oct32.query_image(o, d, 2048, 2048, model="exp", rgb=rgb, alpha=alpha),
                               max(5, args.steps // 2), 2)
        keep_sample(samples, "camera_f32_exp", rgb, alpha, sample_index(n, 11), tree="c1", rays="camera",
                    model="exp")
        variants["camera_f32_exp"] = variant_record(lumiq, oct32, o, d, "exp", tree.K, 4, vms)
        # the same camera batch through the batch-order entry point (row by row)
        vms, _ = time_launches(lambda: oct32.query(o, d, model="linear", rgb=rgb, alpha=alpha),
                               max(5, args.steps // 2), 2)
        keep_sample(samples, "camera_f32_linear_row_order", rgb, alpha, sample_index(n, 11), tree="c1",
                    rays="camera")
        variants["camera_f32_linear_row_order"] = variant_record(lumiq, oct32, o, d, "linear", tree.K, 4, vms)
        log(f"f32 linear, row order: {vms:.3f} ms/step")
        # incoherent shading queries from a room around the luminaire
        ro, rd = inputs.rays.room_to_proxy(1 << 24, 20)
        rays["room"] = (ro, rd)
        ridx = sample_index(len(ro), 13)
        ro_t, rd_t = torch.from_numpy(ro).cuda(), torch.from_numpy(rd).cuda()
        rrgb = torch.empty((1 << 24, 3), device="cuda")
        ralpha = torch.empty((1 << 24,), device="cuda")
        for storage in ("f32", "f16", "bf16"):
            oc = oct32 if storage == "f32" else lumiq.Octree(tree, storage)
            vms, _ = time_launches(lambda: oc.query(ro_t, rd_t, model="linear", rgb=rrgb, alpha=ralpha),
                                   max(3, args.steps // 4), 1)
            keep_sample(samples, f"room16M_{storage}_linear", rrgb, ralpha, ridx, tree="c1", rays="room",
                        storage=storage)
            variants[f"room16M_{storage}_linear"] = variant_record(
                lumiq, oc, ro_t, rd_t, "linear", tree.K, 4 if storage == "f32" else 2, vms,
                traffic_tag=f"query_{storage}_room")
            log(f"room {storage}: {vms:.3f} ms/step")
            if storage != "f32":
                oc.free()
        if args.surrogate_steps > 0:
            variants["surrogate"] = surrogate_variant(args, lumiq, tree, oct32, ro_t, rd_t, rrgb,
                                                      samples=samples, sample_idx=ridx)
        del ro_t, rd_t, rrgb, ralpha

    if not args.no_variants:
        variants["floor_irradiance"] = floor_variant(inputs, oct32, max(5, args.steps // 4), samples=samples)
        variants["floor_irradiance_guided"] = guided_variant(inputs, oct32, max(5, args.steps // 4),
                                                             samples=samples)
        variants["distillation"] = distill_variant(lumiq, 5, samples=samples)

    if args.sh_sweep:
        variants["sh_sweep_camera"] = sh_sweep_variant(lumiq, o, d, max(5, args.steps // 2))

    if not args.no_variants and not args.no_uneven:
        variants["uneven_batch"] = uneven_variant(lumiq, samples=samples, trees_out=trees, rays_out=rays)

    cpu = None
    error = None
    if not args.no_cpu:
        log("timing the CPU oracle")
        cpu = cpu_baseline(tree, o_np, d_np, args.cpu_budget)
        log(f"cpu oracle: {cpu['value']:.0f} rays/s on {cpu['cores']} threads")
        t0 = time.perf_counter()
        errs = error_records(samples, trees, rays)
        error = errs.pop("headline")
        for name, rec in errs.items():
            if name in ("surrogate_only", "surrogate_with_fallback"):
                variants["surrogate"][name]["error"] = rec
            else:
                variants[name]["error"] = rec
        cpu["heuristic_bias"] = heuristic_bias(tree, {k: rays[k] for k in ("camera", "room") if k in rays})
        log(f"error records and heuristic bias: {time.perf_counter() - t0:.1f} s")

    out = {
        "metric": METRIC, "value": round(value, 1), "unit": "rays/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms, 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "depth-9 synthetic luminaire plenoctree (512^3, SH degree 2, "
                               "float32) x 2048x2048 pinhole camera rays (one image, row-major), "
                               "linear transmittance",
                   "rays": n, "n_leaves": tree.n_leaves, "n_nodes": tree.n_nodes,
                   "sh_degree": tree.sh_degree, "storage": "f32", "transmittance": "linear",
                   "sigma_min": 0.1, "alpha_max": 0.9},
        "error": error, "roofline": roofline, "cpu_baseline": cpu, "variants": variants,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
