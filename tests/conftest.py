import os
import shutil
import sys
import tempfile

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

# Tuned plans in the tests take the tile shapes the benchmark takes: those shipped with the
# package, read from a private copy so that shapes tuned during the tests stay out of it.
if "CHFDTD_TUNE_CACHE" not in os.environ:
    _shipped = os.path.join(ROOT, "paper_1001_5341_amd", "tune_cache_gfx950.json")
    _copy = os.path.join(tempfile.mkdtemp(prefix="chfdtd-tune-"), "tune.json")
    if os.path.exists(_shipped):
        shutil.copy(_shipped, _copy)
    os.environ["CHFDTD_TUNE_CACHE"] = _copy


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (runs through the C-ABI library)")
    config.addinivalue_line("markers", "slow: long CPU test (oracle physics at larger sizes)")


def gpu_available() -> bool:
    try:
        import torch

        return torch.cuda.is_available()
    except Exception:
        return False


@pytest.fixture(scope="session")
def gpu():
    if not gpu_available():
        pytest.skip("no GPU in this environment")
    import torch

    return torch.device("cuda:0")
