import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: longer CPU oracle runs")


import pytest  # noqa: E402


@pytest.fixture(scope="session")
def gpctx():
    """One library context for the GPU tests (grids up to 4096 x 4096)."""
    import torch
    from paper_1805_09453_amd import Context
    from paper_1805_09453_amd import build as B
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    if not os.path.exists(B.LIB):
        B.build()
    ctx = Context(4096, 4096)
    yield ctx
    torch.cuda.synchronize()
    ctx.close()


def announce(msg):
    """Name the case before a GPU step (flushed, so a crash log still shows it)."""
    print(f"\n[gpu case] {msg}", flush=True)


def field_err(a, b):
    """Error of a field a against a reference b: the larger of the relative L2 error
    ||a - b|| / ||b|| and the elementwise error max|a - b| / max|b|, so that an error
    confined to a few cells (one halo row, a tile or strip edge) is not diluted by
    the rest of the field."""
    import numpy as np
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    nb = np.linalg.norm(b)
    l2 = np.linalg.norm(a - b) / (nb if nb > 0 else 1.0)
    mb = np.abs(b).max() if b.size else 0.0
    mx = np.abs(a - b).max() / (mb if mb > 0 else 1.0) if b.size else 0.0
    return float(max(l2, mx))
