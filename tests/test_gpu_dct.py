"""GPU parity of the screened Poisson solve (dct_poisson) against the FP64 oracle."""
import numpy as np
import pytest

from conftest import announce, field_err
from oracle import grid

pytestmark = pytest.mark.gpu


def smooth_field(ny, nx, seed, noise=1e-3):
    rng = np.random.default_rng(seed)
    y = (np.arange(ny) + 0.5) / ny
    x = (np.arange(nx) + 0.5) / nx
    X, Y = np.meshgrid(x, y)
    f = np.zeros((ny, nx))
    for _ in range(6):
        cx, cy, s, w = rng.uniform(0.1, 0.9), rng.uniform(0.1, 0.9), rng.uniform(0.03, 0.2), rng.uniform(-1, 1)
        f += w * np.exp(-((X - cx) ** 2 + (Y - cy) ** 2) / (2 * s * s))
    return f + noise * rng.standard_normal((ny, nx))


def rel_l2(a, b):
    """relative L2 and elementwise (relative to max|b|) error, the larger"""
    return field_err(a, b)


CASES = [
    # (ny, nx, h, alpha, kind)
    (64, 64, 1.0, 0.04, "noise"),
    (64, 64, 1.0 / 64, 0.0, "smooth"),
    (64, 128, 0.5, 3.0, "noise"),
    (256, 64, 1.0, 1.0, "noise"),
    (256, 256, 1.0 / 256, 0.0, "smooth"),
    (256, 256, 1.0, 0.08, "smooth"),
    (512, 1024, 1.0, 0.5, "noise"),
    (2048, 2048, 1.0 / 2048, 0.0, "smooth"),
    (4096, 4096, 1.0, 0.04, "smooth"),
    (4096, 4096, 1.0 / 4096, 0.0, "smooth"),
]


@pytest.mark.parametrize("ny,nx,h,alpha,kind", CASES)
def test_dct_poisson_matches_oracle(gpctx, ny, nx, h, alpha, kind):
    import torch
    b = smooth_field(ny, nx, ny + nx) if kind == "smooth" else np.random.default_rng(ny * nx).standard_normal((ny, nx))
    b32 = b.astype(np.float32).astype(np.float64)  # the GPU sees the FP32 input
    x_ref = grid.poisson_solve(b32, h, alpha)
    announce(f"dct_poisson {ny}x{nx} h={h} alpha={alpha} {kind}")
    x = gpctx.dct_poisson(torch.tensor(b32, dtype=torch.float32, device="cuda"), h=h, alpha=alpha)
    err = rel_l2(x.cpu().double().numpy(), x_ref)
    tol = 1e-6 if max(ny, nx) <= 256 else 5e-6
    print(f"rel L2 error {err:.3e} (gate {tol:.0e})")
    assert err <= tol
    if alpha == 0.0:
        assert abs(float(x.double().mean())) <= 1e-6 * float(x.double().abs().max())


@pytest.mark.parametrize("ny,nx,h,alpha", [(64, 64, 1.0 / 64, 0.0), (256, 512, 1.0, 0.3), (4096, 4096, 1.0 / 4096, 0.0)])
def test_dct_poisson_f64_matches_oracle(gpctx, ny, nx, h, alpha):
    import torch
    b = smooth_field(ny, nx, 7)
    x_ref = grid.poisson_solve(b, h, alpha)
    announce(f"dct_poisson_f64 {ny}x{nx} h={h} alpha={alpha}")
    x = gpctx.dct_poisson_f64(torch.tensor(b, dtype=torch.float64, device="cuda"), h=h, alpha=alpha)
    err = rel_l2(x.cpu().numpy(), x_ref)
    print(f"rel L2 error {err:.3e}")
    assert err <= 1e-13


def test_dct_poisson_in_place_and_sampled_residual(gpctx):
    """In-place call; at full size check the discrete equation (alpha - Delta) x = b
    on sampled interior cells with the textbook 5-point stencil."""
    import torch
    ny = nx = 4096
    h, alpha = 1.0, 0.04
    b = np.random.default_rng(3).standard_normal((ny, nx)).astype(np.float32)
    t = torch.tensor(b, device="cuda")
    announce("dct_poisson 4096x4096 in place, sampled residual")
    gpctx.dct_poisson(t, x=t, h=h, alpha=alpha)
    x = t.cpu().double().numpy()
    rng = np.random.default_rng(4)
    ii = rng.integers(1, ny - 1, 2000)
    jj = rng.integers(1, nx - 1, 2000)
    lap = (x[ii + 1, jj] + x[ii - 1, jj] + x[ii, jj + 1] + x[ii, jj - 1] - 4 * x[ii, jj]) / h ** 2
    res = alpha * x[ii, jj] - lap - b[ii, jj]
    assert np.max(np.abs(res)) <= 2e-5 * np.max(np.abs(b))
