import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) and the built HIP library")
    config.addinivalue_line("markers", "slow: long CPU test")


def rel_l2(y, ref):
    """||y - ref||_2 / ||ref||_2 over the whole array (complex norm)."""
    import numpy as np
    y = np.asarray(y)
    ref = np.asarray(ref)
    den = np.linalg.norm(ref.ravel())
    num = np.linalg.norm((y.astype(np.complex128) - ref.astype(np.complex128)).ravel())
    return num / den if den > 0 else num


@pytest.fixture(scope="session")
def hv():
    """The HIP library binding; GPU tests only."""
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2508_03911_amd import hv as _hv
    return _hv


@pytest.fixture(scope="session")
def hv_host():
    """The binding for its host-only calls (file I/O); needs no GPU."""
    from paper_2508_03911_amd import hv as _hv
    return _hv
