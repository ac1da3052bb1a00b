"""The seeded input generators produce well-formed octrees and ray batches."""
import numpy as np

import inputs
from inputs import trees


def _walk(tree):
    """Decode the child table back into {morton: leaf index} and check the
    breadth-first layout."""
    D = tree.depth
    found = {}
    stack = [(0, 0, 0, 0, 0)]     # node, level, x, y, z (node coords at its level)
    seen = set()
    while stack:
        node, lvl, x, y, z = stack.pop()
        assert node not in seen
        seen.add(node)
        for oc in range(8):
            cx, cy, cz = 2 * x + (oc & 1), 2 * y + ((oc >> 1) & 1), 2 * z + ((oc >> 2) & 1)
            c = int(tree.child[node, oc])
            if c > 0:
                assert lvl + 1 < D and c > node
                stack.append((c, lvl + 1, cx, cy, cz))
            elif c < 0:
                assert lvl + 1 == D
                found[int(trees.morton3(cx, cy, cz))] = -c - 1
    assert len(seen) == tree.n_nodes
    return found


def test_octree_roundtrip_random_sets():
    rng = np.random.default_rng(0)
    for D in (1, 2, 3, 5):
        n = 1 << D
        cells = np.unique(rng.integers(0, n, size=(max(1, n ** 3 // 3), 3)), axis=0)
        t = inputs.tree_from_cells(D, cells, np.ones(len(cells)), np.zeros((len(cells), 3, 1)))
        found = _walk(t)
        codes = trees.morton3(t.leaf_cells[:, 0], t.leaf_cells[:, 1], t.leaf_cells[:, 2])
        assert sorted(found) == sorted(codes.tolist())
        # leaves are numbered in Morton order
        assert np.all(np.diff(codes.astype(np.int64)) > 0)
        assert all(found[int(c)] == i for i, c in enumerate(codes))


def test_small_config_tree(c0_tree):
    t = c0_tree
    assert t.depth == 6 and t.sh_degree == 2
    assert abs(t.n_leaves / 64 ** 3 - 0.30) < 0.01
    assert np.all(t.sigma >= np.float32(0.0099999)) and np.all(t.sigma <= 50)
    assert t.sh.shape == (t.n_leaves, 3, 9) and np.all(np.isfinite(t.sh))
    assert len(_walk(t)) == t.n_leaves


def test_morton_roundtrip():
    rng = np.random.default_rng(1)
    xyz = rng.integers(0, 1024, size=(1000, 3))
    c = trees.morton3(xyz[:, 0], xyz[:, 1], xyz[:, 2])
    x, y, z = trees.demorton3(c)
    assert np.array_equal(np.stack([x, y, z], 1).astype(np.int64), xyz)


def test_ray_generators():
    o, d = inputs.rays.sphere_to_cube(1000, 1)
    assert o.dtype == np.float32 and d.dtype == np.float32
    assert np.allclose(np.linalg.norm(o, axis=1), 3.0, atol=1e-5)
    assert np.allclose(np.linalg.norm(d, axis=1), 1.0, atol=1e-6)
    o, d = inputs.rays.pinhole(64, 64)
    assert o.shape == (4096, 3) and np.allclose(o, o[0])
    assert not np.any(d == 0)
    o, d = inputs.rays.room_to_proxy(2000, 2)
    assert np.all(np.abs(o).max(1) > 1)
    assert np.all(np.abs(o[:, :2]) <= 5) and np.all(np.abs(o[:, 2]) <= 1.5)


def test_treefile_roundtrip(tmp_path, c0_tree):
    p = str(tmp_path / "t.lqot")
    inputs.treefile.save(c0_tree, p)
    t = inputs.treefile.load(p)
    assert np.array_equal(t.child, c0_tree.child)
    assert np.array_equal(t.sigma, c0_tree.sigma) and np.array_equal(t.sh, c0_tree.sh)
    assert t.depth == c0_tree.depth and t.l_max == c0_tree.l_max


def test_uneven_batch_recipe():
    """The uneven multi-luminaire batch: 16 trees of depth 6..10 with at least
    one of depth 10, SH degree 3; ray counts log-uniform in [2^10, 2^23]."""
    from inputs import uneven
    sp = uneven.specs()
    assert len(sp) == 16 and max(s.depth for s in sp) == 10
    assert all(6 <= s.depth <= 10 and s.sh_degree == 3 for s in sp)
    assert [s.seed for s in sp] == list(range(40, 56))
    c = uneven.ray_counts()
    assert len(c) == 16 and all(2 ** 10 <= x <= 2 ** 23 for x in c)
    assert c == uneven.ray_counts()   # deterministic


def test_shading_point_recipes():
    p, n = inputs.rays.floor_points(8, 4)
    assert p.shape == (32, 3) and p.dtype == np.float32 and np.all(p[:, 2] == -1.5)
    assert np.all(np.abs(p[:, :2]) < 5) and np.all(n == np.array([0, 0, 1], np.float32))
    assert np.allclose(p[1, 0] - p[0, 0], 10 / 8) and np.allclose(p[8, 1] - p[0, 1], 10 / 4)
    p, n = inputs.rays.scattered_points(5000, 3)
    assert p.dtype == np.float32 and np.all(np.abs(p).max(1) > 1.05)
    assert np.all(np.linalg.norm(p, axis=1) <= 6.0 + 1e-5)
    assert np.mean(np.einsum("ij,ij->i", n, -p) > 0) > 0.9      # mostly facing the luminaire
    u = inputs.rays.sample_numbers(10, 7, 4)
    assert u.shape == (10, 7, 3) and u.dtype == np.float32 and u.min() >= 0 and u.max() < 1
    assert np.array_equal(u, inputs.rays.sample_numbers(10, 7, 4))
