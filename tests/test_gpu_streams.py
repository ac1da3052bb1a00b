"""The C ABI's stream argument: calls on side streams (torch streams of the
default priority) are ordered after the work queued before them on that
stream, and calls on two streams at once each get their own ray counters,
so every result matches the default-stream call bit for bit."""
import sys

import numpy as np
import pytest

import inputs

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


def test_query_on_side_streams(lq, c0_tree):
    import torch
    o, d = inputs.rays.sphere_to_cube(200_003, 41)
    O, D = _dev(o), _dev(d)
    oct_ = lq.Octree(c0_tree, "f32")
    ref_rgb, ref_a = oct_.query(O, D)
    torch.cuda.synchronize()
    _say("query on one side stream, inputs produced on that stream just before")
    s1 = torch.cuda.Stream()
    with torch.cuda.stream(s1):
        O1, D1 = O * 1.0, D * 1.0            # kernels queued on s1 right before the query
        rgb1, a1 = oct_.query(O1, D1)
    s1.synchronize()
    assert torch.equal(rgb1, ref_rgb) and torch.equal(a1, ref_a)
    _say("two queries at once on two side streams")
    s2 = torch.cuda.Stream()
    o2, d2 = inputs.rays.sphere_to_cube(150_001, 42)
    O2, D2 = _dev(o2), _dev(d2)
    ref2_rgb, ref2_a = oct_.query(O2, D2)
    torch.cuda.synchronize()
    outs = []
    for _ in range(3):
        with torch.cuda.stream(s1):
            r1 = oct_.query(O, D)
        with torch.cuda.stream(s2):
            r2 = oct_.query(O2, D2)
        outs.append((r1, r2))
    torch.cuda.synchronize()
    for (rgb_a, a_a), (rgb_b, a_b) in outs:
        assert torch.equal(rgb_a, ref_rgb) and torch.equal(a_a, ref_a)
        assert torch.equal(rgb_b, ref2_rgb) and torch.equal(a_b, ref2_a)


def test_image_and_irradiance_on_a_side_stream(lq, c0_tree):
    import torch
    W, H = 333, 211
    o, d = inputs.rays.pinhole(W, H)
    O, D = _dev(o), _dev(d)
    oct_ = lq.Octree(c0_tree, "f32")
    pts, nrm = inputs.rays.scattered_points(500, 43)
    u = inputs.rays.sample_numbers(500, 32, 44)
    P, N, U = _dev(pts), _dev(nrm), _dev(u)
    B = (0.2, 0.5, 1.0)
    ref_img, _ = oct_.query_image(O, D, W, H)
    ref_E, _ = oct_.proxy_irradiance(P, N, U, background=B)
    torch.cuda.synchronize()
    _say("camera batch and proxy irradiance on a side stream")
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        img, _ = oct_.query_image(O * 1.0, D * 1.0, W, H)
        E, _ = oct_.proxy_irradiance(P * 1.0, N * 1.0, U * 1.0, background=B)
    s.synchronize()
    assert torch.equal(img, ref_img)
    assert torch.equal(E, ref_E)
