"""Pins for the oracle's discrete operators (CPU only).

Each check compares the oracle against something other than itself: a dense
matrix assembled here from the textbook 5-point stencil, the textbook DCT-II
sum, adjointness, or the optimality condition of a projection.
"""
import numpy as np
import pytest
import scipy.fft as sfft

from oracle import grid


def dense_neumann_laplacian(ny, nx, h):
    """Graph Laplacian of the 4-neighbour grid with weights 1/h^2 (the mirror /
    Neumann 5-point Laplacian), assembled cell by cell."""
    N = ny * nx
    A = np.zeros((N, N))
    for i in range(ny):
        for j in range(nx):
            c = i * nx + j
            for di, dj in ((1, 0), (-1, 0), (0, 1), (0, -1)):
                a, b = i + di, j + dj
                if 0 <= a < ny and 0 <= b < nx:
                    A[c, a * nx + b] += 1.0 / h ** 2
                    A[c, c] -= 1.0 / h ** 2
    return A


def naive_dct2_ortho(x):
    N = len(x)
    k = np.arange(N)[:, None]
    j = np.arange(N)[None, :]
    C = np.cos(np.pi * k * (2 * j + 1) / (2 * N))
    s = np.full(N, np.sqrt(2.0 / N))
    s[0] = np.sqrt(1.0 / N)
    return s * (C @ x)


@pytest.mark.parametrize("ny,nx,h", [(5, 7, 1.0), (8, 8, 0.125), (3, 11, 0.3)])
def test_grad_div_adjoint(ny, nx, h):
    rng = np.random.default_rng(1)
    u = rng.standard_normal((ny, nx))
    px, py = rng.standard_normal((2, ny, nx))
    gx, gy = grid.grad(u, h)
    lhs = grid.inner(gx, px, h) + grid.inner(gy, py, h)
    rhs = -grid.inner(u, grid.div(px, py, h), h)
    assert abs(lhs - rhs) <= 1e-13 * max(1.0, abs(lhs))
    # normal component on the far faces vanishes
    assert np.all(gx[:, -1] == 0) and np.all(gy[-1, :] == 0)


def test_grad_textbook_values():
    u = np.arange(12.0).reshape(3, 4) ** 2
    gx, gy = grid.grad(u, 0.5)
    assert gx[1, 2] == (u[1, 3] - u[1, 2]) / 0.5
    assert gy[0, 3] == (u[1, 3] - u[0, 3]) / 0.5


@pytest.mark.parametrize("ny,nx,h", [(6, 7, 1.0), (9, 5, 0.2)])
def test_laplacian_matches_dense_stencil(ny, nx, h):
    A = dense_neumann_laplacian(ny, nx, h)
    u = np.random.default_rng(2).standard_normal((ny, nx))
    assert np.allclose(grid.laplacian(u, h).ravel(), A @ u.ravel(), rtol=0, atol=1e-12 / h ** 2)


def test_scipy_dct_matches_textbook_sum():
    x = np.random.default_rng(3).standard_normal(13)
    assert np.allclose(sfft.dct(x, type=2, norm="ortho"), naive_dct2_ortho(x), atol=1e-14)


@pytest.mark.parametrize("ny,nx,h", [(6, 7, 1.0), (8, 8, 1.0 / 8)])
def test_eigenvalues_of_dense_laplacian(ny, nx, h):
    A = dense_neumann_laplacian(ny, nx, h)
    mu = grid.neg_laplacian_eigs(ny, nx, h)
    for k in range(ny):
        for l in range(nx):
            vy = np.cos(np.pi * k * (2 * np.arange(ny) + 1) / (2 * ny))
            vx = np.cos(np.pi * l * (2 * np.arange(nx) + 1) / (2 * nx))
            v = np.outer(vy, vx).ravel()
            assert np.allclose(A @ v, -mu[k, l] * v, atol=1e-10 / h ** 2)


@pytest.mark.parametrize("alpha", [0.3, 2.0, 64.0])
@pytest.mark.parametrize("ny,nx,h", [(6, 6, 1.0), (7, 10, 0.1), (16, 16, 1.0 / 16)])
def test_screened_poisson_matches_dense_solve(alpha, ny, nx, h):
    A = dense_neumann_laplacian(ny, nx, h)
    b = np.random.default_rng(4).standard_normal((ny, nx))
    x_ref = np.linalg.solve(alpha * np.eye(ny * nx) - A, b.ravel())
    x = grid.poisson_solve(b, h, alpha)
    assert np.max(np.abs(x.ravel() - x_ref)) <= 1e-12 * max(1.0, np.abs(x_ref).max())


@pytest.mark.parametrize("ny,nx,h", [(6, 6, 1.0), (5, 9, 0.25)])
def test_pure_neumann_poisson_is_min_norm_lstsq(ny, nx, h):
    A = dense_neumann_laplacian(ny, nx, h)
    b = np.random.default_rng(5).standard_normal((ny, nx))
    bm = b - b.mean()
    x_ref = np.linalg.lstsq(-A, bm.ravel(), rcond=None)[0]  # min-norm => mean zero
    x = grid.poisson_solve(b, h, 0.0)
    assert abs(x.mean()) < 1e-13
    assert np.max(np.abs(x.ravel() - x_ref)) <= 1e-11 * max(1.0, np.abs(x_ref).max())
    # Delta psi = f for the inverse Laplacian helper
    psi = grid.inv_laplacian(b, h)
    assert np.allclose(A @ psi.ravel(), bm.ravel(), atol=1e-10 / h ** 2)


def test_projection_closed_form_and_kkt():
    rng = np.random.default_rng(6)
    qx, qy = 3 * rng.standard_normal((2, 40, 40))
    px, py = grid.project_unit_ball(qx, qy)
    n = np.hypot(qx, qy)
    inside = n <= 1
    assert np.all(px[inside] == qx[inside]) and np.all(py[inside] == qy[inside])
    assert np.allclose(np.hypot(px, py)[~inside], 1.0)
    # variational inequality <q - P q, p' - P q> <= 0 for every feasible p'
    for _ in range(20):
        ax, ay = rng.standard_normal((2, 40, 40))
        s = np.maximum(1.0, np.hypot(ax, ay)) * rng.uniform(1.0, 3.0, (40, 40))
        ax, ay = ax / s, ay / s
        vi = (qx - px) * (ax - px) + (qy - py) * (ay - py)
        assert vi.max() <= 1e-12
    # anisotropic dual ball is the box
    bx, by = grid.project_unit_ball(qx, qy, grid.ANISO)
    assert np.all(np.abs(bx) <= 1) and np.all(np.abs(by) <= 1)
    assert np.array_equal(bx, np.clip(qx, -1, 1))
