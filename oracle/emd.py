"""L1 earth mover's distance (Beckmann form) by G-prox PDHG, FP64 (section 3.2).

TEST INFRASTRUCTURE ONLY (see the package docstring).

Problem (section 3.2): EMD(rho1, rho0) = min { int |m| : div m = rho1 - rho0,
m . n = 0 }.  Hodge split m = u + grad psi with Delta psi = rho1 - rho0
(Neumann) and div u = 0:   min_u  int |u + grad psi| + chi_{div-free}(u).

Saddle form (u + grad psi, p) + chi_{div-free}(u) - chi_inf(p); the G-prox
PDHG updates of section 3.2, in the paper's order:
    u+    = u - tau P(pbar),     P = Id - grad Delta^{-1} div   (Leray)
    p+    = proj_{|.|<=1}(p + sigma (u+ + grad psi))
    pbar+ = 2 p+ - p
with u0 = 0 (so m0 = grad psi) and p0 = 0, or p0 = proj(grad phi0) for a
warm start from a potential phi0.

Values:
    primal  P(u) = h^2 sum |u + grad psi|                 (upper bound on EMD)
    dual certificate (the paper gives none; see Kantorovich duality
    EMD = max { int phi (rho0 - rho1) : |grad phi| <= 1 }):
        phi = Delta^{-1} div p,   L = max |grad phi|,   phi~ = phi / max(1, L),
        D = h^2 sum phi~ (rho0 - rho1)                     (lower bound on EMD)
    valid because (u, grad phi~) = 0 for divergence-free u and |grad phi~| <= 1.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

from . import grid
from .grid import ISO


class MassMismatch(ValueError):
    pass


def setup(rho0, rho1, h, mass_rtol=1e-6):
    """Mass check in FP64 and the Hodge potential: returns (f, psi) where
    f = rho1 - rho0 - mean(rho1 - rho0) and Delta psi = f, mean(psi) = 0."""
    rho0 = np.asarray(rho0, dtype=np.float64)
    rho1 = np.asarray(rho1, dtype=np.float64)
    if (rho0 < 0).any() or (rho1 < 0).any():
        raise ValueError("densities must be non-negative")
    m0, m1 = float(rho0.sum()), float(rho1.sum())
    if abs(m0 - m1) > mass_rtol * abs(m0):
        raise MassMismatch(f"mass mismatch {m0} vs {m1}")
    f = rho1 - rho0
    f = f - f.mean()
    psi = grid.inv_laplacian(f, h)
    return f, psi


def leray(vx, vy, h):
    """P v = v - grad Delta^{-1} div v (projection onto divergence-free fields)."""
    phi = grid.inv_laplacian(grid.div(vx, vy, h), h)
    gx, gy = grid.grad(phi, h)
    return vx - gx, vy - gy


def primal(ux, uy, gpx, gpy, h, norm=ISO) -> float:
    return h * h * float(np.sum(grid.pointwise_norm(ux + gpx, uy + gpy, norm)))


def certificate(px, py, f, h, norm=ISO):
    """(D, L, phi~): the scaled-potential lower bound on EMD from the dual iterate."""
    phi = grid.inv_laplacian(grid.div(px, py, h), h)
    gx, gy = grid.grad(phi, h)
    L = grid.dual_norm_max(gx, gy, norm)
    phit = phi / max(1.0, L)
    return -h * h * float(np.sum(phit * f)), L, phit


def step(ux, uy, px, py, pbx, pby, gpx, gpy, h, tau, sigma, norm=ISO):
    """One G-prox PDHG iteration (section 3.2 updates)."""
    lx, ly = leray(pbx, pby, h)
    ux1 = ux - tau * lx
    uy1 = uy - tau * ly
    qx, qy = grid.project_unit_ball(px + sigma * (ux1 + gpx), py + sigma * (uy1 + gpy), norm)
    return ux1, uy1, qx, qy, 2.0 * qx - px, 2.0 * qy - py


@dataclass
class Result:
    ux: np.ndarray
    uy: np.ndarray
    px: np.ndarray
    py: np.ndarray
    psi: np.ndarray
    f: np.ndarray
    iters: int
    primal: float
    dual: float
    rel_gap: float
    converged: bool
    history: list = field(default_factory=list)
    m: tuple = None


def rel_gap(P, D):
    return (P - D) / abs(P) if P != 0 else abs(P - D)


def solve(rho0, rho1, h, tau=1.0, sigma=None, tol=1e-5, max_iter=100000, check_every=10,
          phi0=None, norm=ISO, callback=None, ergodic=False):
    """Iterate until (P - D)/|P| <= tol on the last iterate or max_iter.
    Returns a Result whose ``m`` attribute is the flux u + grad psi.
    ergodic: evaluate the gap on, and return, the averages u^N, p^N of the
    iterates n = 1..N (the iterates the section-2 theorems bound)."""
    if sigma is None:
        sigma = 1.0 / tau
    f, psi = setup(rho0, rho1, h)
    gpx, gpy = grid.grad(psi, h)
    ux = np.zeros_like(f)
    uy = np.zeros_like(f)
    if phi0 is None:
        px = np.zeros_like(f)
        py = np.zeros_like(f)
    else:
        px, py = grid.project_unit_ball(*grid.grad(np.asarray(phi0, np.float64), h), norm)
    pbx, pby = px.copy(), py.copy()
    hist = []
    it = 0
    P = D = g = np.nan
    conv = False
    sums = [np.zeros_like(f) for _ in range(4)]
    while it < max_iter:
        ux, uy, px, py, pbx, pby = step(ux, uy, px, py, pbx, pby, gpx, gpy, h, tau, sigma, norm)
        it += 1
        if ergodic:
            for acc, x in zip(sums, (ux, uy, px, py)):
                acc += x
        if it % check_every == 0 or it == max_iter:
            eux, euy, epx, epy = [a / it for a in sums] if ergodic else (ux, uy, px, py)
            P = primal(eux, euy, gpx, gpy, h, norm)
            D = certificate(epx, epy, f, h, norm)[0]
            g = rel_gap(P, D)
            hist.append((it, P, D, g))
            if callback is not None:
                callback(it, P, D, g)
            if g <= tol:
                conv = True
                break
    if ergodic:
        ux, uy, px, py = [a / it for a in sums]
    res = Result(ux, uy, px, py, psi, f, it, P, D, g, conv, hist)
    res.m = (ux + gpx, uy + gpy)
    return res


def flux_value(mx, my, f, h, norm=ISO):
    """h^2 sum |m'| where m' is m re-projected onto {div m' = f} in FP64:
    m' = m - grad Delta^{-1}(div m - f).  Also returns the divergence residual
    max |div m - f| before re-projection."""
    mx = np.asarray(mx, np.float64)
    my = np.asarray(my, np.float64)
    r = grid.div(mx, my, h) - f
    corr = grid.inv_laplacian(r, h)
    gx, gy = grid.grad(corr, h)
    return h * h * float(np.sum(grid.pointwise_norm(mx - gx, my - gy, norm))), float(np.abs(r).max())


def step_rule_tau_singular(eps, M):
    """Section 4.2 rule for singular (Dirac) measures: tau = min(sqrt(1/(eps |log eps|)), 2 M^{1/4})."""
    return float(min(np.sqrt(1.0 / (eps * abs(np.log(eps)))), 2.0 * M ** 0.25))


def drs_step(yx, yy, gpx, gpy, h, tau, norm=ISO):
    """One step of the single-variable form at sigma = 1/tau (the Douglas-Rachford
    case of section 2): with y_n = p_{n-1} + sigma (u_n + grad psi), p_n = proj(y_n)
    and R(y) = 2 proj(y) - y, the updates of section 3.2 become
        phi = Delta^{-1} div R(y_n),  u_{n+1} = -tau (R(y_n) - grad phi),
        y_{n+1} = y_n - proj(y_n) + grad phi + sigma grad psi;
    the zero start is y_0 = 0 and a warm start p_0 = proj(grad phi0) is y_0 = p_0.
    Returns (ux+, uy+, yx+, yy+)."""
    qx, qy = grid.project_unit_ball(yx, yy, norm)
    rx, ry = 2.0 * qx - yx, 2.0 * qy - yy
    gx, gy = grid.grad(grid.inv_laplacian(grid.div(rx, ry, h), h), h)
    return (-tau * (rx - gx), -tau * (ry - gy), yx - qx + gx + gpx / tau, yy - qy + gy + gpy / tau)
