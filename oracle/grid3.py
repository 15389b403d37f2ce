"""Discrete operators, the ROF and the EMD iterations on an nz x ny x nx
cell-centred grid with spacing h (FP64): the d = 3 case of section 3, whose
theory holds for any dimension d.

TEST INFRASTRUCTURE ONLY (see the package docstring).

The discretisation is the 2-D one of ``grid`` with a third axis (arrays are
[z][y][x], x the last axis):

* inner product (a, b) = h^3 * sum(a * b)
* gradient: forward differences along x, y, z, zero on the far faces
* divergence: div = -grad^T (backward differences)
* Laplacian: the 7-point mirror Laplacian; the orthonormal 3-D DCT-II
  diagonalises it with eigenvalues of -Delta
      mu_klm = (4/h^2) (sin^2(pi k/(2 nz)) + sin^2(pi l/(2 ny)) + sin^2(pi m/(2 nx)))
* pointwise norms: isotropic sqrt(px^2 + py^2 + pz^2); anisotropic
  |px| + |py| + |pz| (dual ball: |.|_inf <= 1).

The ROF and EMD updates are those of sections 3.1 and 3.2 with these
operators (ROF in the literal form of section 3.1, EMD in the projected form
u+ = P(u - tau pbar) of the 2-D oracle); values and certificates as in 2-D
with h^3 for h^2.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np
import scipy.fft as sfft

ISO, ANISO = 0, 1


# ---------------------------------------------------------------- operators
def grad(u, h):
    """Forward-difference gradient (gx, gy, gz); zero on the far faces."""
    u = np.asarray(u, np.float64)
    gx = np.zeros_like(u)
    gy = np.zeros_like(u)
    gz = np.zeros_like(u)
    gx[:, :, :-1] = (u[:, :, 1:] - u[:, :, :-1]) / h
    gy[:, :-1, :] = (u[:, 1:, :] - u[:, :-1, :]) / h
    gz[:-1, :, :] = (u[1:, :, :] - u[:-1, :, :]) / h
    return gx, gy, gz


def div(px, py, pz, h):
    """Divergence as the negative adjoint of ``grad`` under h^3 * sum (far-face
    components taken as zero)."""
    qx = np.array(px, dtype=np.float64, copy=True)
    qy = np.array(py, dtype=np.float64, copy=True)
    qz = np.array(pz, dtype=np.float64, copy=True)
    qx[:, :, -1] = 0.0
    qy[:, -1, :] = 0.0
    qz[-1, :, :] = 0.0
    d = qx + qy + qz
    d[:, :, 1:] -= qx[:, :, :-1]
    d[:, 1:, :] -= qy[:, :-1, :]
    d[1:, :, :] -= qz[:-1, :, :]
    return d / h


def laplacian(u, h):
    return div(*grad(u, h), h)


def neg_laplacian_eigs(nz, ny, nx, h):
    m = [4.0 / h ** 2 * np.sin(np.pi * np.arange(n, dtype=np.float64) / (2 * n)) ** 2 for n in (nz, ny, nx)]
    return m[0][:, None, None] + m[1][None, :, None] + m[2][None, None, :]


def poisson_solve(b, h, alpha):
    """(alpha I - Delta) x = b, Neumann; alpha = 0: b projected to mean zero
    and the solution's zero mode set to 0."""
    b = np.asarray(b, np.float64)
    if alpha < 0:
        raise ValueError("alpha must be >= 0")
    if alpha == 0.0:
        b = b - b.mean()
    B = sfft.dctn(b, type=2, norm="ortho")
    den = alpha + neg_laplacian_eigs(*b.shape, h)
    if alpha == 0.0:
        den[0, 0, 0] = 1.0
        B[0, 0, 0] = 0.0
    return sfft.idctn(B / den, type=2, norm="ortho")


def inv_laplacian(f, h):
    """Mean-zero psi with Delta psi = f - mean(f)."""
    return poisson_solve(-np.asarray(f, np.float64), h, 0.0)


def pointwise_norm(px, py, pz, norm=ISO):
    if norm == ISO:
        return np.sqrt(px * px + py * py + pz * pz)
    return np.abs(px) + np.abs(py) + np.abs(pz)


def project_unit_ball(qx, qy, qz, norm=ISO):
    """Projection onto {|p| <= 1} of the dual norm, pointwise."""
    if norm == ISO:
        s = np.maximum(1.0, np.sqrt(qx * qx + qy * qy + qz * qz))
        return qx / s, qy / s, qz / s
    return np.clip(qx, -1.0, 1.0), np.clip(qy, -1.0, 1.0), np.clip(qz, -1.0, 1.0)


def dual_norm_max(gx, gy, gz, norm=ISO):
    if norm == ISO:
        return float(np.sqrt(gx * gx + gy * gy + gz * gz).max())
    return float(np.maximum(np.maximum(np.abs(gx), np.abs(gy)), np.abs(gz)).max())


def rel_gap(P, D):
    return (P - D) / abs(P) if P != 0 else abs(P - D)


# ---------------------------------------------------------------- ROF (section 3.1)
def rof_primal(u, I, h, lam, norm=ISO):
    """P(u) = h^3 sum |grad u| + lambda/2 h^3 sum (u - I)^2."""
    g = grad(u, h)
    return h ** 3 * float(np.sum(pointwise_norm(*g, norm))) + \
        0.5 * lam * h ** 3 * float(np.sum((np.asarray(u) - I) ** 2))


def rof_dual(px, py, pz, I, h, lam):
    """D(p) = -h^3 sum I div p - h^3/(2 lambda) sum (div p)^2 (p feasible)."""
    d = div(px, py, pz, h)
    return -h ** 3 * float(np.sum(I * d)) - h ** 3 / (2.0 * lam) * float(np.sum(d * d))


def rof_step(u, p, pbar, I, h, lam, tau, sigma, norm=ISO):
    """One iteration: u+ = (lambda tau - Delta)^{-1}(lambda tau I + tau div pbar - Delta u),
    p+ = proj(p + sigma grad u+), pbar+ = 2 p+ - p.  p, pbar: 3-tuples."""
    rhs = lam * tau * I + tau * div(*pbar, h) - laplacian(u, h)
    u1 = poisson_solve(rhs, h, lam * tau)
    g = grad(u1, h)
    q = project_unit_ball(*(a + sigma * b for a, b in zip(p, g)), norm)
    return u1, q, tuple(2.0 * a - b for a, b in zip(q, p))


@dataclass
class RofResult:
    u: np.ndarray
    p: tuple
    iters: int
    primal: float
    dual: float
    rel_gap: float
    converged: bool
    history: list = field(default_factory=list)


def rof_solve(I, h, lam, tau, sigma=None, tol=1e-8, max_iter=100000, check_every=10, norm=ISO, ergodic=False):
    """From u0 = 0, p0 = 0: iterate until the relative gap of the last iterate
    is <= tol (checked every check_every iterations) or max_iter.  ergodic:
    evaluate the gap on, and return, the averages of the iterates n = 1..N."""
    I = np.asarray(I, np.float64)
    sigma = 1.0 / tau if sigma is None else sigma
    u = np.zeros_like(I)
    p = tuple(np.zeros_like(I) for _ in range(3))
    pbar = tuple(a.copy() for a in p)
    sums = [np.zeros_like(I) for _ in range(4)]
    it, P, D, g, conv, hist = 0, np.nan, np.nan, np.nan, False, []
    while it < max_iter:
        u, p, pbar = rof_step(u, p, pbar, I, h, lam, tau, sigma, norm)
        it += 1
        if ergodic:
            for acc, x in zip(sums, (u,) + p):
                acc += x
        if it % check_every == 0 or it == max_iter:
            eu, *ep = [a / it for a in sums] if ergodic else (u,) + p
            P, D = rof_primal(eu, I, h, lam, norm), rof_dual(*ep, I, h, lam)
            g = rel_gap(P, D)
            hist.append((it, P, D, g))
            if g <= tol:
                conv = True
                break
    if ergodic:
        u, *pl = [a / it for a in sums]
        p = tuple(pl)
    return RofResult(u, p, it, P, D, g, conv, hist)


# ---------------------------------------------------------------- EMD (section 3.2)
def emd_setup(rho0, rho1, h, mass_rtol=1e-6):
    """FP64 mass check; f = rho1 - rho0 - mean, psi with Delta psi = f, mean zero."""
    rho0 = np.asarray(rho0, np.float64)
    rho1 = np.asarray(rho1, np.float64)
    if (rho0 < 0).any() or (rho1 < 0).any():
        raise ValueError("densities must be non-negative")
    m0, m1 = float(rho0.sum()), float(rho1.sum())
    if abs(m0 - m1) > mass_rtol * abs(m0):
        raise ValueError(f"mass mismatch {m0} vs {m1}")
    f = rho1 - rho0
    f = f - f.mean()
    return f, inv_laplacian(f, h)


def leray(v, h):
    """P v = v - grad Delta^{-1} div v."""
    phi = inv_laplacian(div(*v, h), h)
    return tuple(a - b for a, b in zip(v, grad(phi, h)))


def emd_primal(u, gpsi, h, norm=ISO):
    """P = h^3 sum |u + grad psi|."""
    return h ** 3 * float(np.sum(pointwise_norm(*(a + b for a, b in zip(u, gpsi)), norm)))


def emd_certificate(p, f, h, norm=ISO):
    """(D, L, phi~): phi = Delta^{-1} div p, L = max |grad phi|, phi~ = phi / max(1, L),
    D = -h^3 sum phi~ f (a lower bound on EMD)."""
    phi = inv_laplacian(div(*p, h), h)
    L = dual_norm_max(*grad(phi, h), norm)
    phit = phi / max(1.0, L)
    return -h ** 3 * float(np.sum(phit * f)), L, phit


def emd_step(u, p, pbar, gpsi, h, tau, sigma, norm=ISO):
    """u+ = P(u - tau pbar), p+ = proj(p + sigma (u+ + grad psi)), pbar+ = 2 p+ - p."""
    u1 = leray(tuple(a - tau * b for a, b in zip(u, pbar)), h)
    q = project_unit_ball(*(a + sigma * (b + c) for a, b, c in zip(p, u1, gpsi)), norm)
    return u1, q, tuple(2.0 * a - b for a, b in zip(q, p))


@dataclass
class EmdResult:
    u: tuple
    p: tuple
    f: np.ndarray
    psi: np.ndarray
    m: tuple
    iters: int
    primal: float
    dual: float
    rel_gap: float
    converged: bool
    history: list = field(default_factory=list)


def emd_solve(rho0, rho1, h, tau=1.0, sigma=None, tol=1e-5, max_iter=100000, check_every=10, norm=ISO,
              ergodic=False, phi0=None):
    """From u0 = 0 and p0 = 0 (or p0 = proj(grad phi0) for a warm start from a
    potential) until the relative gap (P - D)/|P| <= tol or max_iter; ``m`` is
    the flux u + grad psi.  ergodic: evaluate the gap on, and return, the
    averages of the iterates n = 1..N (u, p and so m)."""
    sigma = 1.0 / tau if sigma is None else sigma
    f, psi = emd_setup(rho0, rho1, h)
    gpsi = grad(psi, h)
    u = tuple(np.zeros_like(f) for _ in range(3))
    if phi0 is None:
        p = tuple(np.zeros_like(f) for _ in range(3))
    else:
        p = project_unit_ball(*grad(np.asarray(phi0, np.float64), h), norm)
    pbar = tuple(a.copy() for a in p)
    sums = [np.zeros_like(f) for _ in range(6)]
    it, P, D, g, conv, hist = 0, np.nan, np.nan, np.nan, False, []
    while it < max_iter:
        u, p, pbar = emd_step(u, p, pbar, gpsi, h, tau, sigma, norm)
        it += 1
        if ergodic:
            for acc, x in zip(sums, u + p):
                acc += x
        if it % check_every == 0 or it == max_iter:
            avg = [a / it for a in sums] if ergodic else list(u + p)
            P = emd_primal(tuple(avg[:3]), gpsi, h, norm)
            D = emd_certificate(tuple(avg[3:]), f, h, norm)[0]
            g = rel_gap(P, D)
            hist.append((it, P, D, g))
            if g <= tol:
                conv = True
                break
    if ergodic:
        avg = [a / it for a in sums]
        u, p = tuple(avg[:3]), tuple(avg[3:])
    m = tuple(a + b for a, b in zip(u, gpsi))
    return EmdResult(u, p, f, psi, m, it, P, D, g, conv, hist)


# ---------------------------------------------------------------- single-variable form (sigma tau = 1)
# With sigma = 1/tau the two-variable iteration above depends on (u_n, p_n, pbar_n)
# only through y_n = p_{n-1} + sigma grad u_n (ROF) or y_n = p_{n-1} + sigma (u_n +
# grad psi) (EMD), with p_n = proj(y_n): the boundary case tau sigma = 1 that
# section 2 relates to Douglas-Rachford splitting.  Writing R(y) = 2 proj(y) - y:
#   ROF  u_{n+1} = (lambda tau - Delta)^{-1} (lambda tau I + tau div R(y_n)),
#        y_{n+1} = proj(y_n) + sigma grad u_{n+1}
#   EMD  y_{n+1} = y_n - proj(y_n) + grad Delta^{-1} div R(y_n) + sigma grad psi,
#        u_{n+1} = -tau (R(y_n) - grad Delta^{-1} div R(y_n))
# (the EMD u-update is the projection P applied to u_n - tau pbar_n = -tau R(y_n)
# - grad psi, P grad psi = 0).  The zero start u_0 = 0, p_0 = pbar_0 = 0 is y_0 = 0
# in both.  Derived here from the updates of sections 3.1 and 3.2.
def reflect(y, norm=ISO):
    q = project_unit_ball(*y, norm)
    return q, tuple(2.0 * a - b for a, b in zip(q, y))


def rof_drs_step(y, I, h, lam, tau, norm=ISO):
    """One single-variable ROF step (sigma = 1/tau): returns (u_{n+1}, y_{n+1})."""
    q, R = reflect(y, norm)
    u1 = poisson_solve(lam * tau * I + tau * div(*R, h), h, lam * tau)
    g = grad(u1, h)
    return u1, tuple(a + b / tau for a, b in zip(q, g))


def emd_drs_step(y, gpsi, h, tau, norm=ISO):
    """One single-variable EMD step (sigma = 1/tau): returns (u_{n+1}, y_{n+1})."""
    q, R = reflect(y, norm)
    gphi = grad(inv_laplacian(div(*R, h), h), h)
    u1 = tuple(-tau * (r - g) for r, g in zip(R, gphi))
    return u1, tuple(a - b + g + c / tau for a, b, g, c in zip(y, q, gphi, gpsi))
