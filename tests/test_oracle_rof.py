"""Pins for the ROF oracle (CPU only).

References used here are independent of the oracle's iteration: a bounded-
variable least-squares solve of the 1-D dual, an accelerated projected
gradient (FISTA) run on the 2-D dual, the disc closed form, and invariants
the paper states (mean preservation, maximum principle, strong convexity).
"""
import json
import os

import numpy as np
import pytest
from scipy.optimize import lsq_linear

import synth
from oracle import grid, rof

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def rof_1d_exact(I1, h, lam):
    """Exact 1-D ROF minimiser from its dual: min_{|p|<=1} ||div p + lam I||^2
    (a box-constrained least-squares problem, solved by BVLS); u = I + div p / lam."""
    n = len(I1)
    A = np.zeros((n, n - 1))  # (div p)_j = (p_j - p_{j-1}) / h, p_{-1} = p_{n-1} = 0
    for j in range(n - 1):
        A[j, j] += 1.0 / h
        A[j + 1, j] -= 1.0 / h
    res = lsq_linear(A, -lam * I1, bounds=(-1.0, 1.0), method="bvls", tol=1e-15, max_iter=10000)
    return I1 + A @ res.x / lam


def fista_dual(I, h, lam, iters=20000):
    """Accelerated projected gradient on the ROF dual min_{|p|<=1} 1/(2 lam) ||div p + lam I||^2."""
    Lc = 8.0 / (h * h * lam)
    px = np.zeros_like(I)
    py = np.zeros_like(I)
    yx, yy, t = px.copy(), py.copy(), 1.0
    for _ in range(iters):
        d = grid.div(yx, yy, h) + lam * I
        gx, gy = grid.grad(d, h)
        nx_, ny_ = grid.project_unit_ball(yx + gx / (lam * Lc), yy + gy / (lam * Lc))
        t1 = 0.5 * (1 + np.sqrt(1 + 4 * t * t))
        yx = nx_ + (t - 1) / t1 * (nx_ - px)
        yy = ny_ + (t - 1) / t1 * (ny_ - py)
        px, py, t = nx_, ny_, t1
    return px, py


def test_rof_1d_reduces_to_bvls():
    n, h, lam = 48, 1.0 / 48, 40.0
    x = (np.arange(n) + 0.5) / n
    rng = np.random.default_rng(11)
    I1 = (x > 0.3).astype(float) - 0.6 * (x > 0.7) + 0.05 * rng.standard_normal(n)
    I = np.tile(I1, (4, 1))  # constant along y
    u_ref = rof_1d_exact(I1, h, lam)
    r = rof.solve(I, h, lam, tau=0.5, tol=1e-12, max_iter=200000, check_every=50)
    assert r.converged
    # strong convexity (corollary in section 3.1): lam/2 ||u - u*||^2 <= P - F* <= gap
    bound = np.sqrt(2 * (r.primal - r.dual) / lam / (4 * h * h)) + 1e-10
    assert np.all(np.abs(r.u - u_ref[None, :]) <= max(bound, 1e-6))
    assert np.abs(r.py).max() < 1e-12  # no y-flux


def test_rof_2d_matches_independent_fista():
    I = synth.rof_scene(32, synth.config_seed(0, 99))
    h, lam = 1.0, 8.0
    px, py = fista_dual(I, h, lam, iters=6000)
    Fstar_lo = rof.dual(px, py, I, h, lam)
    Fstar_hi = rof.primal(I + grid.div(px, py, h) / lam, I, h, lam)
    assert (Fstar_hi - Fstar_lo) / Fstar_hi < 1e-7
    r = rof.solve(I, h, lam, tau=0.005, tol=1e-9, max_iter=100000, check_every=50)
    assert r.converged
    # both are certified brackets of the same F*
    assert r.dual <= Fstar_hi * (1 + 1e-12) and Fstar_lo <= r.primal * (1 + 1e-12)
    assert abs(r.primal - Fstar_hi) / Fstar_hi < 2e-7


def test_constant_image_is_fixed_point():
    I = np.full((16, 20), 0.37)
    r = rof.solve(I, 1.0, 8.0, tau=0.7, tol=0.0, max_iter=3, check_every=1)
    assert np.allclose(r.u, I, atol=1e-15)
    assert np.abs(r.px).max() < 1e-15 and abs(r.primal - r.dual) < 1e-12


def test_mean_preserved_every_iterate():
    I = synth.rof_scene(40, 7)
    means = []
    u, px, py = np.zeros_like(I), np.zeros_like(I), np.zeros_like(I)
    pbx, pby = px.copy(), py.copy()
    for _ in range(30):
        u, px, py, pbx, pby = rof.step(u, px, py, pbx, pby, I, 1.0, 8.0, 0.3, 1 / 0.3)
        means.append(u.mean())
    assert np.max(np.abs(np.array(means) - I.mean())) < 1e-13


def test_gap_nonnegative_and_reaches_1e8_on_64px_scene():
    I = synth.rof_scene(64, synth.config_seed(0))
    seen = []
    r = rof.solve(I, 1.0, 8.0, tau=0.005, tol=1e-8, max_iter=20000, check_every=100,
                  callback=lambda it, P, D, g: seen.append(g))
    assert r.converged and r.iters <= 12000
    assert min(seen) >= 0.0
    # maximum principle (section 3.1, proof of the ROF gap proposition): min I <= u* <= max I
    assert r.u.min() >= I.min() - 1e-6 and r.u.max() <= I.max() + 1e-6
    # field bound from strong convexity against an earlier, looser iterate
    r2 = rof.solve(I, 1.0, 8.0, tau=0.005, tol=1e-5, max_iter=20000, check_every=10)
    gap_abs = r2.primal - r2.dual
    dist2 = float(np.sum((r2.u - r.u) ** 2))  # h = 1
    assert dist2 <= 2 * (gap_abs + (r.primal - r.dual)) / 8.0 * 1.0001


def test_large_lambda_approaches_image():
    I = synth.rof_scene(24, 3)
    r = rof.solve(I, 1.0, 1e5, tau=1e-4, tol=1e-9, max_iter=20000, check_every=20)
    # u - I = div p / lambda and |div p| <= 4 / h
    assert np.abs(r.u - I).max() <= 4.0 / 1e5 + 1e-9


def disc_closed_form(lam, r):
    """Two-valued minimiser for the disc indicator on the unit square with
    Neumann boundary (corrected form of the paper's section 3.1 / 4.1 formula;
    see tests/golden/paper_values.json)."""
    a = 1.0 - 2.0 / (lam * r)
    b = 2 * np.pi * r / (lam * (1 - np.pi * r * r))
    return a, b


def test_disc_golden_values_and_threshold():
    with open(os.path.join(GOLDEN, "paper_values.json")) as fh:
        g = json.load(fh)["rof_disc"]
    a, b = disc_closed_form(g["lambda"], g["radius"])
    assert abs(a - g["inside_corrected"]) < 1e-12 and abs(b - g["outside_corrected"]) < 1e-12
    # the printed form does not preserve the mean; the corrected one does
    r = g["radius"]
    assert abs(a * np.pi * r * r + b * (1 - np.pi * r * r) - np.pi * r * r) < 1e-14
    printed_inside = 1 - 2 / (g["lambda"] * r) + b
    assert abs(printed_inside - g["inside_as_printed"]) < 1e-12


@pytest.mark.slow
def test_disc_converges_to_corrected_closed_form():
    lam, rad = 20.0, 0.25
    a, b = disc_closed_form(lam, rad)
    errs = []
    for n in (32, 64, 128):
        I = synth.disc_image(n, rad)
        r = rof.solve(I, 1.0 / n, lam, tau=2.0, tol=1e-6, max_iter=20000, check_every=50)
        X, Y = synth.cell_centres(n, n)
        dist = np.hypot(X - 0.5, Y - 0.5)
        inside = r.u[dist < rad - 0.1].mean()
        outside = r.u[dist > rad + 0.1].mean()
        errs.append((abs(inside - a), abs(outside - b)))
        assert abs(r.u.mean() - I.mean()) < 1e-12
    assert errs[2][0] < errs[0][0] and errs[2][1] < errs[0][1]
    assert errs[2][0] < 0.01 and errs[2][1] < 0.005


def test_ergodic_average_is_the_mean_of_the_iterates_and_brackets_the_optimum():
    """ergodic=True returns (1/N) sum_{n=1..N} (u_n, p_n), checked against a
    separate loop over rof.step; the averages are feasible (|p| <= 1 is convex),
    so weak duality D(p^N) <= F* <= P(u^N) holds; the averaged gap closes."""
    I = synth.rof_scene(16, 3)
    h, lam, tau = 1.0, 8.0, 0.05
    K = 7
    st = (np.zeros_like(I),) + tuple(np.zeros_like(I) for _ in range(4))
    acc = [np.zeros_like(I) for _ in range(3)]
    for _ in range(K):
        st = rof.step(*st, I, h, lam, tau, 1.0 / tau)
        for a, x in zip(acc, st[:3]):
            a += x
    r = rof.solve(I, h, lam, tau, tol=0.0, max_iter=K, check_every=K, ergodic=True)
    for got, a in zip((r.u, r.px, r.py), acc):
        np.testing.assert_allclose(got, a / K, rtol=0, atol=1e-14)
    assert abs(r.primal - rof.primal(acc[0] / K, I, h, lam)) < 1e-12
    assert abs(r.dual - rof.dual(acc[1] / K, acc[2] / K, I, h, lam)) < 1e-12
    fstar = rof.solve(I, h, lam, tau, tol=1e-11, max_iter=200000, check_every=100).primal
    long = rof.solve(I, h, lam, tau, tol=0.0, max_iter=3000, check_every=3000, ergodic=True)
    for res in (r, long):
        assert res.dual <= fstar * (1 + 1e-12) and fstar <= res.primal * (1 + 1e-12)
    assert long.rel_gap < 1e-2 < r.rel_gap
