import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: takes more than a few seconds on the CPU")


def _ensure_host_libs():
    """Build the gcc-only pieces (input generators, oracle) when absent."""
    from paper_2510_27517_amd import inputs
    import oracle

    if not os.path.exists(inputs.LIB_PATH):
        inputs.build()
    if not os.path.exists(oracle.LIB_PATH):
        oracle.build()


_ensure_host_libs()


@pytest.fixture(scope="session")
def gpu_lib():
    """The HIP library's Python binding; fails loudly if not built or no GPU."""
    import torch

    if not torch.cuda.is_available():
        pytest.fail("GPU test collected without a GPU (run with -m 'not gpu' on CPU hosts)")
    from paper_2510_27517_amd import pcg

    pcg.load()
    return pcg
