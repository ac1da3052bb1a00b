"""GPU parity of the proxy-irradiance entry point (the consumer side: the
Eq. 2 blend and uniform proxy sampling) against the oracle, through the C ABI."""
import sys

import numpy as np
import pytest

import inputs
from oracle import shade
from tests import parity

pytestmark = pytest.mark.gpu


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


def _dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def _check(tree, pts, nrm, u, B, model, terms_g, E_g, idx=None, orc=None):
    """Per-sample terms (if given) and per-point estimates against the oracle;
    a threshold-ambiguous sample may match either oracle candidate."""
    m = 0 if model == "linear" else 1
    if orc is None:
        orc = shade.proxy_irradiance(tree, pts, nrm, u, background=B, model=m)
    Bc = np.abs(np.asarray(B, np.float64))[None, None, :]
    floor = orc["w"][:, :, None] * (parity.FLOOR * tree.l_max + Bc)
    t_ref = orc["terms"]
    if terms_g is not None:
        e_main = np.abs(terms_g - orc["terms"]) / np.maximum(np.abs(orc["terms"]), floor + 1e-30)
        e_alt = np.abs(terms_g - orc["terms_alt"]) / np.maximum(np.abs(orc["terms_alt"]), floor + 1e-30)
        use_alt = orc["alt_valid"][:, :, None] & (e_alt < e_main)
        err = np.where(use_alt, e_alt, e_main)
        _say(f"terms: max rel {err.max():.2e}, {int(orc['alt_valid'].sum())} ambiguous samples")
        assert err.max() <= parity.RTOL, err.max()
        assert np.all(terms_g[orc["w"] == 0] == 0)
        t_ref = np.where(use_alt, orc["terms_alt"], orc["terms"])
    else:
        assert not orc["alt_valid"].any()
    E_ref = t_ref.mean(axis=1)
    e = np.abs(E_g - E_ref) / np.maximum(np.abs(E_ref), floor.mean(axis=1) + 1e-30)
    _say(f"irradiance: max rel {e.max():.2e} over {len(E_ref)} points")
    assert e.max() <= parity.RTOL, e.max()


def _trees(c0_tree):
    return {"c0": c0_tree, "empty": inputs.empty_tree(3),
            "opaque": inputs.uniform_tree(2, 1e6, np.array([[-1.0], [0.5], [2.0]]))}


@pytest.mark.parametrize("which", ["c0", "empty", "opaque"])
@pytest.mark.parametrize("model", ["linear", "exp"])
def test_proxy_irradiance_parity(lq, c0_tree, which, model):
    import torch
    tree = _trees(c0_tree)[which]
    pts, nrm = inputs.rays.scattered_points(400, 21)
    u = inputs.rays.sample_numbers(400, 64, 22)
    B = (0.2, 0.5, 1.0)
    _say(f"proxy irradiance {which} {model}: 400 points x 64 samples")
    oct_ = lq.Octree(tree, "f32")
    E, terms = oct_.proxy_irradiance(_dev(pts), _dev(nrm), _dev(u), background=B, model=model,
                                     want_terms=True)
    torch.cuda.synchronize()
    _check(tree, pts, nrm, u, B, model, terms.cpu().numpy().astype(np.float64),
           E.cpu().numpy().astype(np.float64))
    # deterministic: a second call gives the same bits, with or without the terms
    E2, _ = oct_.proxy_irradiance(_dev(pts), _dev(nrm), _dev(u), background=B, model=model)
    torch.cuda.synchronize()
    assert torch.equal(E, E2)


def test_proxy_irradiance_edge_cases(lq, c0_tree):
    import torch
    oct_ = lq.Octree(c0_tree, "f32")
    _say("proxy irradiance edge cases")
    # no points
    z = torch.empty((0, 3), device="cuda")
    E, _ = oct_.proxy_irradiance(z, z, torch.empty((0, 4, 3), device="cuda"))
    assert E.shape == (0, 3)
    # one sample per point, a ragged count of points; a point inside the proxy
    # and one facing away receive exactly 0; no background (black)
    pts, nrm = inputs.rays.scattered_points(333, 31)
    pts[0] = (0.2, -0.1, 0.3)
    pts[1], nrm[1] = (0.0, 0.0, -3.0), (0.0, 0.0, -1.0)
    u = inputs.rays.sample_numbers(333, 1, 32)
    E, terms = oct_.proxy_irradiance(_dev(pts), _dev(nrm), _dev(u), want_terms=True)
    torch.cuda.synchronize()
    E = E.cpu().numpy().astype(np.float64)
    assert np.all(E[:2] == 0)
    _check(c0_tree, pts, nrm, u, (0.0, 0.0, 0.0), "linear", terms.cpu().numpy().astype(np.float64), E)


@pytest.mark.parametrize("n,S", [(3, 5000), (100, 37), (1000, 2), (5, 2048)])
def test_proxy_irradiance_sample_counts(lq, c0_tree, n, S):
    """Sample counts that split a point over several reduction chunks, that
    do not divide the chunk, and that pack many points per chunk."""
    import torch
    pts, nrm = inputs.rays.scattered_points(n, 60 + S)
    u = inputs.rays.sample_numbers(n, S, 61 + S)
    B = (1.0, 0.0, 0.5)
    _say(f"proxy irradiance: {n} points x {S} samples")
    oct_ = lq.Octree(c0_tree, "f32")
    E, terms = oct_.proxy_irradiance(_dev(pts), _dev(nrm), _dev(u), background=B, want_terms=True)
    torch.cuda.synchronize()
    _check(c0_tree, pts, nrm, u, B, "linear", terms.cpu().numpy().astype(np.float64),
           E.cpu().numpy().astype(np.float64))


def test_proxy_irradiance_rejects_bad_arguments(lq, c0_tree):
    import ctypes as C
    import torch
    L = lq.lib()
    oct_ = lq.Octree(c0_tree, "f32")
    p = torch.zeros((8, 3), device="cuda")
    u = torch.zeros((8, 2, 3), device="cuda")
    out = torch.zeros((8, 3), device="cuda")
    host = np.zeros((8, 3), np.float32)
    ptr = lambda t: C.c_void_p(t.data_ptr())
    assert L.lq_proxy_irradiance(oct_.handle, ptr(p), ptr(p), 8, ptr(u), 0, None, 0, ptr(out), None, None) == -1
    assert L.lq_proxy_irradiance(oct_.handle, ptr(p), ptr(p), 8, ptr(u), 2, None, 5, ptr(out), None, None) == -1
    assert L.lq_proxy_irradiance(oct_.handle, C.c_void_p(host.ctypes.data), ptr(p), 8, ptr(u), 2, None, 0,
                                 ptr(out), None, None) == -1
    assert b"device pointer" in L.lq_last_error()
    assert L.lq_proxy_irradiance(oct_.handle, ptr(p), ptr(p), 8, ptr(u), 65536, None, 0, ptr(out), None,
                                 None) == -1
    assert b"smaller" in L.lq_last_error()          # u holds 2 samples per point


def test_full_size_floor_sampled_parity(lq, c1_tree):
    """The benchmarked configuration: the depth-9 tree lighting a 1024 x 1024
    floor grid with 16 proxy samples per point, in one call; a seeded sample
    of points is checked against the oracle."""
    import torch
    pts, nrm = inputs.rays.floor_points(1024, 1024)
    u = inputs.rays.sample_numbers(len(pts), 16, 5)
    B = (0.05, 0.05, 0.08)
    _say(f"full-size floor: {len(pts)} points x 16 samples")
    oct_ = lq.Octree(c1_tree, "f32")
    E, _ = oct_.proxy_irradiance(_dev(pts), _dev(nrm), _dev(u), background=B)
    torch.cuda.synchronize()
    E = E.cpu().numpy().astype(np.float64)
    oct_.free()
    idx = np.sort(np.random.default_rng(3).choice(len(pts), 2000, replace=False))
    orc = shade.proxy_irradiance(c1_tree, pts[idx], nrm[idx], u[idx], background=B)
    amb = orc["alt_valid"].any(axis=1)
    Bc = np.abs(np.asarray(B))[None, :]
    floor = orc["w"].mean(axis=1)[:, None] * (parity.FLOOR * c1_tree.l_max + Bc)
    e = np.abs(E[idx] - orc["E"]) / np.maximum(np.abs(orc["E"]), floor + 1e-30)
    _say(f"floor: max rel {e[~amb].max():.2e} over {int((~amb).sum())} points ({int(amb.sum())} with an ambiguous sample)")
    assert e[~amb].max() <= parity.RTOL
    assert np.all(np.isfinite(E)) and np.all(E >= 0)


# ------------------------------------------------------------ guided sampling
def test_guide_weights_parity(lq, c0_tree):
    """Guide weights (mean probe luminance per proxy cell) against the
    oracle's: 1e-4 relative (floor 1e-3 of the largest weight), plus, for a
    cell with threshold-ambiguous probes, the luminance gap of their
    candidates over the probe count."""
    import torch
    G, R = 8, 16
    u = inputs.rays.probe_numbers(shade.guide_cells(G), R, 70)
    oct_ = lq.Octree(c0_tree, "f32")
    for model, m in (("linear", 0), ("exp", 1)):
        w = oct_.proxy_guide(G, _dev(u), model=model)
        torch.cuda.synchronize()
        w = w.cpu().numpy().astype(np.float64)
        ref, q = shade.guide_weights(c0_tree, G, u, model=m)
        slack = (np.abs(q["alt_L"].mean(1) - q["L"].mean(1)) * q["alt_valid"]).reshape(-1, R).sum(1) / R
        err = np.abs(w - ref) - slack
        tol = 1e-4 * np.maximum(np.abs(ref), 1e-3 * ref.max())
        _say(f"guide {model}: {shade.guide_cells(G)} cells, max |dw| / tol {(err / tol).max():.3f}, "
             f"{int(q['alt_valid'].sum())} ambiguous probes")
        assert np.all(err <= tol)
        assert (w > 0).mean() > 0.5


def _directional_slack(q, G, R, D, u):
    """Per (cell, bin) allowance for threshold-ambiguous probes: the gap of
    their candidates' luminance over the bin's probe count (a bin no probe
    fell in: the cell's gap over R)."""
    n = shade.guide_cells(G)
    _, d = shade.guide_probe_rays(G, u)
    cell = np.repeat(np.arange(n), R)
    b = shade.face_direction_bin(cell // (G * G), -d.astype(np.float64), D)
    gap = np.abs(q["alt_L"].mean(1) - q["L"].mean(1)) * q["alt_valid"]
    s = np.zeros((n, D * D))
    c = np.zeros((n, D * D))
    np.add.at(s, (cell, b), gap)
    np.add.at(c, (cell, b), 1.0)
    tot = np.zeros(n)
    np.add.at(tot, cell, gap)
    return np.where(c > 0, s / np.where(c > 0, c, 1.0), (tot / R)[:, None]).reshape(-1)


@pytest.mark.parametrize("D", [2, 3, 4])
def test_directional_guide_weights_parity(lq, c0_tree, D):
    """Direction-binned guide weights against the oracle's: every probe in
    the same bin on both sides, then 1e-4 relative per (cell, bin)."""
    import torch
    G, R = 6, 48
    u = inputs.rays.probe_numbers(shade.guide_cells(G), R, 71 + D)
    oct_ = lq.Octree(c0_tree, "f32")
    w = oct_.proxy_guide(G, _dev(u), dir_res=D)
    torch.cuda.synchronize()
    w = w.cpu().numpy().astype(np.float64)
    ref, q = shade.guide_weights(c0_tree, G, u, D=D)
    assert w.shape == ref.shape == (shade.guide_cells(G) * D * D,)
    err = np.abs(w - ref) - _directional_slack(q, G, R, D, u)
    tol = 1e-4 * np.maximum(np.abs(ref), 1e-3 * ref.max())
    _say(f"directional guide D={D}: max |dw| / tol {(err / tol).max():.3f}")
    assert np.all(err <= tol)


@pytest.mark.parametrize("D", [2, 3, 4])
@pytest.mark.parametrize("beta", [0.0, 0.25])
def test_directional_guided_irradiance_parity(lq, c0_tree, D, beta):
    """The guided estimator with a direction-binned guide against the
    oracle, sample by sample (bins, cells and weights) and point by point."""
    import torch
    G = 8
    pts, nrm = inputs.rays.scattered_points(300, 33)
    u = inputs.rays.sample_numbers(300, 48, 34)
    w = inputs.rays.guide_weights(shade.guide_cells(G) * D * D, 35 + D)
    B = (0.2, 0.5, 1.0)
    _say(f"directional guided proxy irradiance, D={D}, beta {beta}")
    oct_ = lq.Octree(c0_tree, "f32")
    E, terms = oct_.proxy_irradiance_guided(_dev(pts), _dev(nrm), _dev(u), _dev(w), G, defensive=beta,
                                            background=B, want_terms=True, dir_res=D)
    torch.cuda.synchronize()
    orc = shade.proxy_irradiance_guided(c0_tree, pts, nrm, u, w, G, beta, background=B, D=D)
    _check(c0_tree, pts, nrm, u, B, "linear", terms.cpu().numpy().astype(np.float64),
           E.cpu().numpy().astype(np.float64), orc=orc)


def test_directional_guide_rejects_bad_resolution(lq, c0_tree):
    import torch
    oct_ = lq.Octree(c0_tree, "f32")
    u = _dev(inputs.rays.probe_numbers(shade.guide_cells(2), 4, 36))
    for D in (0, 5):
        with pytest.raises(lq.LumiqError, match="dir_res"):
            oct_.proxy_guide(2, u, dir_res=D, weights=torch.zeros(24 * 25, device="cuda"))


@pytest.mark.parametrize("which", ["c0", "empty", "opaque"])
@pytest.mark.parametrize("model", ["linear", "exp"])
@pytest.mark.parametrize("beta", [0.0, 0.25])
def test_guided_irradiance_parity(lq, c0_tree, which, model, beta):
    """The guided estimator against the oracle, sample by sample (the cell
    choice is bit-exact: the same FP64 table and walk on both sides) and
    point by point, on scattered points that see one to three faces."""
    import torch
    G = 8
    tree = _trees(c0_tree)[which]
    pts, nrm = inputs.rays.scattered_points(400, 21)
    u = inputs.rays.sample_numbers(400, 64, 23)
    w = inputs.rays.guide_weights(shade.guide_cells(G), 24)
    B = (0.2, 0.5, 1.0)
    _say(f"guided proxy irradiance {which} {model} beta {beta}")
    oct_ = lq.Octree(tree, "f32")
    E, terms = oct_.proxy_irradiance_guided(_dev(pts), _dev(nrm), _dev(u), _dev(w), G, defensive=beta,
                                            background=B, model=model, want_terms=True)
    torch.cuda.synchronize()
    m = 0 if model == "linear" else 1
    orc = shade.proxy_irradiance_guided(tree, pts, nrm, u, w, G, beta, background=B, model=m)
    _check(tree, pts, nrm, u, B, model, terms.cpu().numpy().astype(np.float64),
           E.cpu().numpy().astype(np.float64), orc=orc)


@pytest.mark.parametrize("G", [1, 40, 256])
@pytest.mark.parametrize("beta", [0.0, 0.25])
def test_guided_grid_sizes(lq, c0_tree, G, beta):
    """The smallest guide (one cell per face), one of 9,600 cells (more
    than one LDS chunk of the cell table, 2,048 cells) and the largest grid
    the call accepts (256: 393,216 cells): the guided estimator against the
    oracle sample by sample and point by point."""
    import torch
    pts, nrm = inputs.rays.scattered_points(300, 25)
    u = inputs.rays.sample_numbers(300, 32, 26)
    w = inputs.rays.guide_weights(shade.guide_cells(G), 27)
    B = (0.2, 0.5, 1.0)
    _say(f"guided proxy irradiance, grid {G} ({shade.guide_cells(G)} cells), beta {beta}")
    oct_ = lq.Octree(c0_tree, "f32")
    E, terms = oct_.proxy_irradiance_guided(_dev(pts), _dev(nrm), _dev(u), _dev(w), G, defensive=beta,
                                            background=B, want_terms=True)
    torch.cuda.synchronize()
    orc = shade.proxy_irradiance_guided(c0_tree, pts, nrm, u, w, G, beta, background=B)
    _check(c0_tree, pts, nrm, u, B, "linear", terms.cpu().numpy().astype(np.float64),
           E.cpu().numpy().astype(np.float64), orc=orc)


def test_guided_invalid_weights(lq, c0_tree):
    """Negative, NaN and infinite guide weights count as 0 on both sides."""
    import torch
    G = 8
    pts, nrm = inputs.rays.scattered_points(200, 28)
    u = inputs.rays.sample_numbers(200, 32, 29)
    w = inputs.rays.guide_weights(shade.guide_cells(G), 30)
    w[[3, 50, 77, 200, 301]] = [-1.0, np.nan, np.inf, -np.inf, -0.0]
    B = (0.2, 0.5, 1.0)
    _say("guided proxy irradiance with invalid guide weights")
    oct_ = lq.Octree(c0_tree, "f32")
    E, terms = oct_.proxy_irradiance_guided(_dev(pts), _dev(nrm), _dev(u), _dev(w), G, defensive=0.1,
                                            background=B, want_terms=True)
    torch.cuda.synchronize()
    orc = shade.proxy_irradiance_guided(c0_tree, pts, nrm, u, w, G, 0.1, background=B)
    _check(c0_tree, pts, nrm, u, B, "linear", terms.cpu().numpy().astype(np.float64),
           E.cpu().numpy().astype(np.float64), orc=orc)


def test_guided_sampling_reduces_variance(lq, c0_tree):
    """On the floor below the luminaire, with the guide built on the GPU
    from probe rays: the guided and uniform estimates agree within their
    statistical error (the guided one is unbiased) and the guided terms have
    a smaller variance (median over points at least 1.5 times smaller)."""
    import torch
    G, R, S = 8, 32, 4096
    oct_ = lq.Octree(c0_tree, "f32")
    w = oct_.proxy_guide(G, _dev(inputs.rays.probe_numbers(shade.guide_cells(G), R, 80)))
    pts, nrm = inputs.rays.floor_points(8, 8)
    u = _dev(inputs.rays.sample_numbers(len(pts), S, 81))
    P, N = _dev(pts), _dev(nrm)
    B = (0.05, 0.05, 0.08)
    Eu, tu = oct_.proxy_irradiance(P, N, u, background=B, want_terms=True)
    Eg, tg = oct_.proxy_irradiance_guided(P, N, u, w, G, defensive=0.25, background=B, want_terms=True)
    torch.cuda.synchronize()
    tu, tg = tu.double().mean(2).cpu().numpy(), tg.double().mean(2).cpu().numpy()
    vu, vg = tu.var(1), tg.var(1)
    z = np.abs(tu.mean(1) - tg.mean(1)) / np.sqrt((vu + vg) / S)
    ratio = vu / vg
    _say(f"guided vs uniform on 64 floor points x {S}: variance ratio median {np.median(ratio):.2f} "
         f"(min {ratio.min():.2f}), |z| max {z.max():.2f}")
    assert np.median(ratio) >= 1.5
    assert np.median(z) < 2.0 and z.max() < 8.0


def test_guided_full_size_configuration(lq, c1_tree):
    """The benchmark's guided configuration on the depth-9 luminaire: the
    guide (16 x 16 cells per face, 256 probes per cell) against the oracle's,
    and the guided sampler on floor points (a seeded sample of the
    1024 x 1024 grid, 16 samples each) sample by sample against the oracle,
    with a synthetic guide of the same size."""
    import torch
    G, R = 16, 256
    oct_ = lq.Octree(c1_tree, "f32")
    u = inputs.rays.probe_numbers(shade.guide_cells(G), R, 90)
    w = oct_.proxy_guide(G, _dev(u))
    torch.cuda.synchronize()
    w = w.cpu().numpy().astype(np.float64)
    ref, q = shade.guide_weights(c1_tree, G, u)
    slack = (np.abs(q["alt_L"].mean(1) - q["L"].mean(1)) * q["alt_valid"]).reshape(-1, R).sum(1) / R
    err = np.abs(w - ref) - slack
    tol = 1e-4 * np.maximum(np.abs(ref), 1e-3 * ref.max())
    _say(f"full-size guide: max |dw| / tol {(err / tol).max():.3f}")
    assert np.all(err <= tol)
    pts, nrm = inputs.rays.floor_points(1024, 1024)
    idx = np.sort(np.random.default_rng(92).choice(len(pts), 300, replace=False))
    pts, nrm = pts[idx], nrm[idx]
    uu = inputs.rays.sample_numbers(len(pts), 16, 93)
    gw = inputs.rays.guide_weights(shade.guide_cells(G), 94)
    B = (0.05, 0.05, 0.08)
    E, terms = oct_.proxy_irradiance_guided(_dev(pts), _dev(nrm), _dev(uu), _dev(gw), G, defensive=0.25,
                                            background=B, want_terms=True)
    torch.cuda.synchronize()
    orc = shade.proxy_irradiance_guided(c1_tree, pts, nrm, uu, gw, G, 0.25, background=B)
    _check(c1_tree, pts, nrm, uu, B, "linear", terms.cpu().numpy().astype(np.float64),
           E.cpu().numpy().astype(np.float64), orc=orc)
    # the benchmark's directional guide (2 x 2 bins) at the same size
    D = 2
    wd = oct_.proxy_guide(G, _dev(u), dir_res=D)
    torch.cuda.synchronize()
    wd = wd.cpu().numpy().astype(np.float64)
    refd, qd = shade.guide_weights(c1_tree, G, u, D=D)
    err = np.abs(wd - refd) - _directional_slack(qd, G, R, D, u)
    tol = 1e-4 * np.maximum(np.abs(refd), 1e-3 * refd.max())
    _say(f"full-size directional guide: max |dw| / tol {(err / tol).max():.3f}")
    assert np.all(err <= tol)
    gwd = inputs.rays.guide_weights(shade.guide_cells(G) * D * D, 95)
    E, terms = oct_.proxy_irradiance_guided(_dev(pts), _dev(nrm), _dev(uu), _dev(gwd), G, defensive=0.5,
                                            background=B, want_terms=True, dir_res=D)
    torch.cuda.synchronize()
    orc = shade.proxy_irradiance_guided(c1_tree, pts, nrm, uu, gwd, G, 0.5, background=B, D=D)
    _check(c1_tree, pts, nrm, uu, B, "linear", terms.cpu().numpy().astype(np.float64),
           E.cpu().numpy().astype(np.float64), orc=orc)
