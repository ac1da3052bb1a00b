import functools
import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def _gpu_available() -> bool:
    try:
        import torch
        return bool(torch.cuda.is_available())
    except Exception:
        return False


def pytest_collection_modifyitems(config, items):
    if _gpu_available():
        return
    skip = pytest.mark.skip(reason="no GPU in this environment")
    for item in items:
        if "gpu" in item.keywords:
            item.add_marker(skip)


@functools.lru_cache(maxsize=None)
def _tree(name):
    import inputs
    spec = {"c0": inputs.C0_TREE, "c1": inputs.C1_TREE}[name]
    return inputs.cached_tree(spec)


@pytest.fixture(scope="session")
def c0_tree():
    return _tree("c0")


@pytest.fixture(scope="session")
def c1_tree():
    return _tree("c1")
