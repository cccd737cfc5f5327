import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: takes more than a few seconds on the CPU")


def gpu_available() -> bool:
    try:
        import torch

        return torch.cuda.is_available()
    except Exception:
        return False


@pytest.fixture(scope="session")
def dl():
    """The product binding, loaded from the in-tree library (fails loudly if it is missing)."""
    import paper_1012_5168_amd as pkg

    pkg.load()
    return pkg


def pytest_sessionstart(session):
    """Build the in-tree libraries only when nothing is built yet."""
    import importlib.util

    lib = os.path.join(ROOT, "paper_1012_5168_amd", "libdloops.so")
    if not os.path.exists(lib):
        spec = importlib.util.spec_from_file_location("_dl_build", os.path.join(ROOT, "paper_1012_5168_amd",
                                                                                "_build.py"))
        mod = importlib.util.module_from_spec(spec)
        spec.loader.exec_module(mod)
        mod.build()
