import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_sessionstart(session):
    # a fresh checkout has no libeofa.so (built artefacts are not versioned):
    # build it once, in-tree (hipcc cross-compiles for gfx950 without a GPU)
    lib = os.path.join(ROOT, "paper_1611_00298_amd", "libeofa.so")
    if not os.path.exists(lib) and not os.environ.get("EOFA_LIB"):
        from paper_1611_00298_amd import build
        build.build()


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU")
    config.addinivalue_line("markers", "slow: long-running CPU test")


def _gpu_available():
    try:
        import torch
        return torch.cuda.is_available()
    except Exception:
        return False


def pytest_collection_modifyitems(config, items):
    if _gpu_available():
        return
    skip = pytest.mark.skip(reason="no GPU in this container")
    for item in items:
        if "gpu" in item.keywords:
            item.add_marker(skip)
