import os
import sys

import pytest

try:  # import once at collection, outside per-test time limits
    import torch  # noqa: F401
except Exception:  # pragma: no cover
    torch = None

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line(
        "markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")


@pytest.fixture(scope="session")
def gpu_lib():
    """The built C-ABI library, loaded through the Python binding.

    GPU tests fail loudly when the library is missing: there is no CPU
    fallback for the search path.
    """
    import torch
    if not torch.cuda.is_available():
        pytest.fail("GPU test selected but no GPU is visible")
    from paper_1006_4644_amd import ci
    return ci.load()
