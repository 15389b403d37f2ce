"""Discrete operators on an ny x nx cell-centred grid with spacing h (FP64).

TEST INFRASTRUCTURE ONLY (see the package docstring).

Discretisation (the paper does not print one; this is the reading under which
the u-step of Algorithm 2 is an exact argmin and the Leray projection of
section 3.2 is an exact projector):

* inner product (a, b) = h^2 * sum(a * b)                       (L2 on [0,1]^d)
* gradient: forward differences, zero in the last column / row, i.e. the
  normal component vanishes on the far faces (m . n = 0 in section 3.2)
* divergence: div = -grad^T (backward differences)
* Laplacian: Delta = div grad, the 5-point mirror (Neumann) Laplacian.  The
  even reflection of appendix A turns its inverse into a cosine series: the
  orthonormal 2-D DCT-II diagonalises it with eigenvalues of -Delta
      mu_kl = (4/h^2) (sin^2(pi k / (2 ny)) + sin^2(pi l / (2 nx))).
* pointwise norm |p_ij| = sqrt(px_ij^2 + py_ij^2) (isotropic, the 2-norm of
  section 3.2); the anisotropic option uses |px| + |py| (dual ball: |.|_inf <= 1).
"""
from __future__ import annotations

import numpy as np
import scipy.fft as sfft

ISO, ANISO = 0, 1


def grad(u: np.ndarray, h: float):
    """Forward-difference gradient (gx, gy); gx[:, -1] = gy[-1, :] = 0."""
    gx = np.zeros_like(u, dtype=np.float64)
    gy = np.zeros_like(u, dtype=np.float64)
    gx[:, :-1] = (u[:, 1:] - u[:, :-1]) / h
    gy[:-1, :] = (u[1:, :] - u[:-1, :]) / h
    return gx, gy


def div(px: np.ndarray, py: np.ndarray, h: float) -> np.ndarray:
    """Divergence as the negative adjoint of ``grad`` under h^2 * sum.

    (div p)_ij = (px_ij - px_i,j-1)/h + (py_ij - py_i-1,j)/h with the
    out-of-grid terms zero and the far-face components px[:, -1], py[-1, :]
    taken as zero (they are structurally zero for fields in the range of grad).
    """
    qx = np.array(px, dtype=np.float64, copy=True)
    qy = np.array(py, dtype=np.float64, copy=True)
    qx[:, -1] = 0.0
    qy[-1, :] = 0.0
    d = qx.copy()
    d[:, 1:] -= qx[:, :-1]
    d += qy
    d[1:, :] -= qy[:-1, :]
    return d / h


def laplacian(u: np.ndarray, h: float) -> np.ndarray:
    """Delta u = div(grad u)."""
    return div(*grad(u, h), h)


def neg_laplacian_eigs(ny: int, nx: int, h: float) -> np.ndarray:
    """Eigenvalues of -Delta in the orthonormal DCT-II basis, shape [ny][nx]."""
    ky = np.arange(ny, dtype=np.float64)
    kx = np.arange(nx, dtype=np.float64)
    my = 4.0 / h ** 2 * np.sin(np.pi * ky / (2 * ny)) ** 2
    mx = 4.0 / h ** 2 * np.sin(np.pi * kx / (2 * nx)) ** 2
    return my[:, None] + mx[None, :]


def poisson_solve(b: np.ndarray, h: float, alpha: float) -> np.ndarray:
    """Solve (alpha I - Delta) x = b with Neumann boundary conditions.

    alpha > 0: the screened solve of the ROF u-step (alpha = lambda * tau).
    alpha = 0: b is first projected to mean zero (mean taken in FP64), the
    zero mode of the solution is set to 0, so x has mean zero.
    """
    b = np.asarray(b, dtype=np.float64)
    ny, nx = b.shape
    if alpha < 0:
        raise ValueError("alpha must be >= 0")
    if alpha == 0.0:
        b = b - b.mean()
    B = sfft.dctn(b, type=2, norm="ortho")
    den = alpha + neg_laplacian_eigs(ny, nx, h)
    if alpha == 0.0:
        den[0, 0] = 1.0
        B[0, 0] = 0.0
    return sfft.idctn(B / den, type=2, norm="ortho")


def inv_laplacian(f: np.ndarray, h: float) -> np.ndarray:
    """Mean-zero psi with Delta psi = f - mean(f) (Neumann)."""
    return poisson_solve(-np.asarray(f, dtype=np.float64), h, 0.0)


def pointwise_norm(px, py, norm: int = ISO) -> np.ndarray:
    if norm == ISO:
        return np.sqrt(px * px + py * py)
    return np.abs(px) + np.abs(py)


def project_unit_ball(qx, qy, norm: int = ISO):
    """Pointwise projection onto {|p| <= 1} of the dual norm: the p-step
    of Algorithm 2 for f* = indicator of the unit ball (section 3.1 and 3.2).
    Isotropic: q / max(1, |q|_2).  Anisotropic (dual of |.|_1): clip to [-1, 1]."""
    if norm == ISO:
        s = np.maximum(1.0, np.sqrt(qx * qx + qy * qy))
        return qx / s, qy / s
    return np.clip(qx, -1.0, 1.0), np.clip(qy, -1.0, 1.0)


def dual_norm_max(gx, gy, norm: int = ISO) -> float:
    """max over cells of the dual pointwise norm of (gx, gy)."""
    if norm == ISO:
        return float(np.sqrt(gx * gx + gy * gy).max())
    return float(np.maximum(np.abs(gx), np.abs(gy)).max())


def inner(a, b, h: float) -> float:
    return float(h * h * np.sum(np.asarray(a, np.float64) * np.asarray(b, np.float64)))
