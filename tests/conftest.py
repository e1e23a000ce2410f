import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) and the built HIP library")


def gpu_available():
    try:
        import torch
        return torch.cuda.is_available()
    except Exception:
        return False


@pytest.fixture(scope="session", autouse=True)
def _private_tile_cache(tmp_path_factory):
    """Batches created with tuned tiles read and write a cache of this session only."""
    old = os.environ.get("MISSLAM_TILE_CACHE")
    os.environ["MISSLAM_TILE_CACHE"] = str(tmp_path_factory.mktemp("tiles") / "tiles.json")
    yield
    if old is None:
        os.environ.pop("MISSLAM_TILE_CACHE", None)
    else:
        os.environ["MISSLAM_TILE_CACHE"] = old


@pytest.fixture(scope="session")
def lib():
    """The C-ABI library through its Python binding; GPU tests only."""
    if not gpu_available():
        pytest.skip("no GPU")
    from paper_1803_02009_amd import misslam
    return misslam
