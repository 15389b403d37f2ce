"""ROF total-variation denoising by G-prox PDHG, FP64 (section 3.1).

TEST INFRASTRUCTURE ONLY (see the package docstring).

Problem (section 3.1, the functional F_lambda and its saddle form):
    min_u  TV(u) + lambda/2 ||u - I||^2,   TV(u) = h^2 sum |grad u|
    L(u, p) = (grad u, p) + lambda/2 ||u - I||^2 - chi_inf(p)

G-prox PDHG (Algorithm 2, H-inner product (grad u, grad v)) gives the updates
of section 3.1, taken here literally in the paper's order:
    u+   = (lambda tau Id - Delta)^{-1} (lambda tau I + tau div pbar - Delta u)
    p+   = (p + sigma grad u+) / max(1, |p + sigma grad u+|)
    pbar+ = 2 p+ - p
starting from u0 = 0 (the proposition on the ROF gap takes u0 = 0), p0 = 0.

Duality gap (section 2.1, the primal-dual gap G(u, p) = sup_p' L(u,p') -
inf_u' L(u',p)): the sup is the primal value P(u); the inf over u' is attained
at u' = I + div p / lambda, giving
    D(p) = -(I, div p) - ||div p||^2 / (2 lambda)
for |p| <= 1 everywhere (every p-iterate is).  P - D >= P - F* >= 0.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

from . import grid
from .grid import ISO


def primal(u, I, h, lam, norm=ISO) -> float:
    """P(u) = h^2 sum |grad u| + lambda/2 h^2 sum (u - I)^2."""
    gx, gy = grid.grad(u, h)
    tv = h * h * float(np.sum(grid.pointwise_norm(gx, gy, norm)))
    fid = 0.5 * lam * h * h * float(np.sum((np.asarray(u) - I) ** 2))
    return tv + fid


def dual(px, py, I, h, lam) -> float:
    """D(p) = -h^2 sum I div p - h^2/(2 lambda) sum (div p)^2 (p feasible)."""
    d = grid.div(px, py, h)
    return -h * h * float(np.sum(I * d)) - h * h / (2.0 * lam) * float(np.sum(d * d))


def step(u, px, py, pbx, pby, I, h, lam, tau, sigma, norm=ISO):
    """One G-prox PDHG iteration (section 3.1 updates).  Returns (u+, px+, py+, pbx+, pby+)."""
    rhs = lam * tau * I + tau * grid.div(pbx, pby, h) - grid.laplacian(u, h)
    u1 = grid.poisson_solve(rhs, h, lam * tau)
    gx, gy = grid.grad(u1, h)
    qx, qy = grid.project_unit_ball(px + sigma * gx, py + sigma * gy, norm)
    return u1, qx, qy, 2.0 * qx - px, 2.0 * qy - py


@dataclass
class Result:
    u: np.ndarray
    px: np.ndarray
    py: np.ndarray
    iters: int
    primal: float
    dual: float
    rel_gap: float
    converged: bool
    history: list = field(default_factory=list)


def rel_gap(P: float, D: float) -> float:
    return (P - D) / abs(P) if P != 0 else abs(P - D)


def solve(I, h, lam, tau, sigma=None, tol=1e-8, max_iter=100000, check_every=10,
          u0=None, p0=None, norm=ISO, callback=None, ergodic=False) -> Result:
    """Iterate until the relative gap (P - D)/|P| of the last iterate is <= tol
    (checked every ``check_every`` iterations) or ``max_iter`` is reached.
    sigma defaults to 1/tau, the choice of every step rule in the paper.
    ergodic: evaluate the gap on, and return, the averages u^N = (1/N) sum u_n,
    p^N = (1/N) sum p_n over n = 1..N (the iterates the section-2 theorems bound)."""
    I = np.asarray(I, dtype=np.float64)
    if sigma is None:
        sigma = 1.0 / tau
    u = np.zeros_like(I) if u0 is None else np.array(u0, dtype=np.float64)
    if p0 is None:
        px = np.zeros_like(I)
        py = np.zeros_like(I)
    else:
        px, py = (np.array(a, dtype=np.float64) for a in p0)
    pbx, pby = px.copy(), py.copy()
    hist = []
    it = 0
    P = D = g = np.nan
    conv = False
    su, sx, sy = np.zeros_like(I), np.zeros_like(I), np.zeros_like(I)
    while it < max_iter:
        u, px, py, pbx, pby = step(u, px, py, pbx, pby, I, h, lam, tau, sigma, norm)
        it += 1
        if ergodic:
            su += u
            sx += px
            sy += py
        if it % check_every == 0 or it == max_iter:
            eu, ex, ey = (su / it, sx / it, sy / it) if ergodic else (u, px, py)
            P = primal(eu, I, h, lam, norm)
            D = dual(ex, ey, I, h, lam)
            g = rel_gap(P, D)
            hist.append((it, P, D, g))
            if callback is not None:
                callback(it, P, D, g)
            if g <= tol:
                conv = True
                break
    if ergodic:
        u, px, py = su / it, sx / it, sy / it
    return Result(u, px, py, it, P, D, g, conv, hist)


def tv_norm(u, h, norm=ISO) -> float:
    """||u||_TV = h^2 sum |grad u| (the discrete total variation of section 3.1)."""
    gx, gy = grid.grad(u, h)
    return h * h * float(np.sum(grid.pointwise_norm(gx, gy, norm)))


def step_rule_tau(I, h, lam, eps) -> float:
    """Section 4.1 step rule: tau = min(sqrt(lambda) ||I||_TV / sqrt(eps),
    ||grad I||_L2), sigma = 1/tau (dimensional constants dropped, as in the paper)."""
    gx, gy = grid.grad(I, h)
    l2 = np.sqrt(h * h * float(np.sum(gx * gx + gy * gy)))
    return float(min(np.sqrt(lam) * tv_norm(I, h) / np.sqrt(eps), l2))


def tv_bound(I, h, lam) -> float:
    """Section 3.1 bound ||u*||_TV <= min(||I||_TV, lambda/2 ||I0 - I||^2), I0 = mean(I)."""
    I = np.asarray(I, dtype=np.float64)
    return float(min(tv_norm(I, h), 0.5 * lam * h * h * float(np.sum((I - I.mean()) ** 2))))
