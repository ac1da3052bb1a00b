"""Seeded synthetic inputs (trees and rays) shared by the oracle, the GPU
library's tests and the benchmark.  Holds no arithmetic of the query itself."""
from .trees import (ALPHA_MAX, C0_TREE, C1_TREE, L_MAX, SIGMA_MIN, Tree, TreeSpec, cached_tree,
                    build_octree, demorton3, empty_tree, make_tree, morton3,
                    random_tree, tree_from_cells, uniform_tree)
from . import rays, treefile

__all__ = [
    "ALPHA_MAX", "C0_TREE", "C1_TREE", "L_MAX", "SIGMA_MIN", "Tree", "TreeSpec", "cached_tree",
    "build_octree", "demorton3", "empty_tree", "make_tree", "morton3", "random_tree",
    "tree_from_cells", "uniform_tree", "rays", "treefile",
]
