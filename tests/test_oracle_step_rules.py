"""Pins for the oracle's step-size helpers (CPU only).

* ``rof.tv_norm`` and the two terms of the section 4.1 rule
  tau = min(sqrt(lambda) ||I||_TV / sqrt(eps), ||grad I||_L2): images whose
  forward differences are worked out by hand at h = 1/n.
* ``rof.tv_bound``, the section 3.1 bound ||u*||_TV <= min(||I||_TV,
  lambda/2 ||I0 - I||^2) with I0 the mean of I: a constant-plus-step image,
  where both terms have closed forms, and the bound itself checked on a solved
  minimiser.
* ``emd.step_rule_tau_singular``, the section 4.2 rule
  tau = min(sqrt(1 / (eps |log eps|)), 2 M^(1/4)): values worked out by hand
  with the natural logarithm, and the regime statements the paper makes about
  the rule on its 512^2 ... 4096^2 grids (which term is smaller at each eps),
  which hold for the natural logarithm with M the side length.
"""
import math

import numpy as np
import pytest

from oracle import emd, grid, rof


def vertical_step(n, c=0.0, d=1.0):
    """c + d on the columns j < n/2, c on the others."""
    I = np.full((n, n), c, dtype=np.float64)
    I[:, : n // 2] += d
    return I


def corner_square(n, c):
    """c on the cells (i, j) with i, j < n/2, 0 elsewhere."""
    I = np.zeros((n, n))
    I[: n // 2, : n // 2] = c
    return I


# --------------------------------------------------------------- ||I||_TV
def test_tv_of_a_vertical_step_is_the_jump_times_the_edge_length():
    # the x-difference is -n at the n cells of column n/2 - 1, zero elsewhere:
    # h^2 * n * n = 1 per unit jump, for every n
    for n in (8, 16, 64):
        assert rof.tv_norm(vertical_step(n), 1.0 / n) == pytest.approx(1.0, abs=1e-14)
        assert rof.tv_norm(vertical_step(n, 0.3, 2.5), 1.0 / n) == pytest.approx(2.5, abs=1e-13)
    # per-pixel units (h = 1): n cells of |grad| = 1
    assert rof.tv_norm(vertical_step(16), 1.0) == pytest.approx(16.0, abs=1e-13)


def test_tv_of_a_corner_square_collocates_the_norm():
    # n = 16, value 1/2 on the 8 x 8 corner: 7 cells with only an x-jump (rows 0..6 of
    # column 7), 7 with only a y-jump (columns 0..6 of row 7), and cell (7, 7) with both,
    # each jump of size 8 (= 0.5 / h).  Isotropic: h^2 (14 * 8 + 8 sqrt 2) = (14 + sqrt 2) / 32;
    # l1 norm: h^2 * 16 * 8 = 1/2.
    I = corner_square(16, 0.5)
    assert rof.tv_norm(I, 1.0 / 16) == pytest.approx((14.0 + math.sqrt(2.0)) / 32.0, abs=1e-14)
    assert rof.tv_norm(I, 1.0 / 16, norm=grid.ANISO) == pytest.approx(0.5, abs=1e-14)


# --------------------------------------------------------------- section 4.1 rule
@pytest.mark.parametrize("lam, eps, tau", [
    # vertical unit step at n = 16: ||I||_TV = 1 and ||grad I||_L2 = sqrt(h^2 * 16 * 16^2) = 4
    (4.0, 1.0, 2.0),       # sqrt(4) * 1 / sqrt(1) = 2 < 4          (lambda, not sqrt(lambda), would give 4)
    (1.0, 0.25, 2.0),      # sqrt(1) * 1 / sqrt(0.25) = 2 < 4       (eps, not sqrt(eps), would give 4)
    (100.0, 0.01, 4.0),    # 10 / 0.1 = 100 > 4: the L2 term binds  (its square would give 16)
    (0.01, 1e-4, 4.0),     # 0.1 / 0.01 = 10 > 4
])
def test_rof_step_rule_on_a_vertical_step(lam, eps, tau):
    assert rof.step_rule_tau(vertical_step(16), 1.0 / 16, lam, eps) == pytest.approx(tau, abs=1e-13)


def test_rof_step_rule_on_a_corner_square():
    # n = 16, value 1/2: ||grad I||_L2^2 = h^2 (16 * 8^2) = 4 (the corner cell holds 8^2 + 8^2),
    # so the L2 term is 2; the TV term is sqrt(lambda) (14 + sqrt 2) / 32 / sqrt(eps)
    I, h = corner_square(16, 0.5), 1.0 / 16
    assert rof.step_rule_tau(I, h, 1.0e4, 1.0) == pytest.approx(2.0, abs=1e-13)
    lam, eps = 2.0, 0.5
    assert rof.step_rule_tau(I, h, lam, eps) == pytest.approx(
        math.sqrt(lam) * (14.0 + math.sqrt(2.0)) / 32.0 / math.sqrt(eps), abs=1e-13)


# --------------------------------------------------------------- section 3.1 bound
@pytest.mark.parametrize("c, d, lam, bound", [
    # I = c + d [j < n/2]: mean c + d/2, |I - I0| = d/2 on every cell, so
    # ||I0 - I||^2 = d^2 / 4 on the unit square and ||I||_TV = d
    (0.3, 2.0, 0.5, 0.25),    # min(2, 0.25 * 4 / 4)     = 0.25
    (0.3, 2.0, 10.0, 2.0),    # min(2, 5 * 4 / 4)        = 2
    (-1.0, 0.5, 8.0, 0.25),   # min(0.5, 4 * 0.25 / 4)   = 0.25
    (5.0, 0.5, 1.0, 0.03125),  # min(0.5, 0.5 * 0.0625)  = 1/32
])
def test_tv_bound_on_constant_plus_step(c, d, lam, bound):
    for n in (16, 32):
        assert rof.tv_bound(vertical_step(n, c, d), 1.0 / n, lam) == pytest.approx(bound, abs=1e-13)


def test_tv_bound_holds_for_the_solved_minimiser():
    # the bound of section 3.1 is an inequality on u*: check it on a solved noisy scene
    # in both regimes (lambda 5: the fidelity term is the smaller one; lambda 200: ||I||_TV)
    rng = np.random.default_rng(5)
    n, h = 32, 1.0 / 32
    I = corner_square(n, 1.0) + 0.1 * rng.standard_normal((n, n))
    for lam in (5.0, 200.0):
        r = rof.solve(I, h, lam, tau=0.5, tol=1e-7, max_iter=200000, check_every=50)
        assert r.converged
        # ||u||_TV <= P(u) <= F* + (P - D) for the returned iterate, and F* <= the bound
        gap = r.primal - r.dual
        assert rof.tv_norm(r.u, h) <= rof.tv_bound(I, h, lam) + gap
        # and the objective value itself lies below both comparison points
        assert r.primal <= rof.primal(I, I, h, lam) + 1e-9
        assert r.primal <= rof.primal(np.full_like(I, I.mean()), I, h, lam) + 1e-9


# --------------------------------------------------------------- section 4.2 rule
@pytest.mark.parametrize("eps, M, tau", [
    # 0.01 * ln 100 = 0.0460517019; 1 / that = 21.7147241; sqrt = 4.65990602
    (1e-2, 4096, 4.659906),
    # 0.001 * ln 1000 = 0.00690775528; 1 / that = 144.764827; sqrt = 12.0318256
    (1e-3, 4096, 12.031826),
    (1e-3, 16, 4.0),           # 2 * 16^(1/4) = 4 binds
    # 1e-4 * ln 1e4 = 9.21034037e-4; 1 / that = 1085.73620; sqrt = 32.9505114; 2 * 4096^(1/4) = 16 binds
    (1e-4, 4096, 16.0),
    (1e-4, 1e6, 32.950511),    # 2 * (1e6)^(1/4) = 63.2 does not bind
])
def test_emd_singular_rule_by_hand(eps, M, tau):
    assert emd.step_rule_tau_singular(eps, M) == pytest.approx(tau, rel=2e-7)


def test_emd_singular_rule_matches_the_papers_regime_statements():
    """Section 4.2 says which term of the rule is smaller on the 512^2 ... 4096^2
    grids.  With M the side length and the natural logarithm every statement
    holds; log10 (eps = 1e-3: 18.3) or M the number of cells (2 M^(1/4) = 45 at
    512^2) contradict them."""
    def first(eps):
        return emd.step_rule_tau_singular(eps, 1e12)  # the cap far away: the eps term alone

    def cap(n):
        return emd.step_rule_tau_singular(1e-12, n)   # eps tiny: the cap alone

    sizes = (512, 1024, 2048, 4096)
    # eps = 1e-2: the eps term is smaller on every grid
    assert all(first(1e-2) < cap(n) for n in sizes)
    # eps = 1e-3: larger on 512^2, approximately equal on 1024^2, smaller on 2048^2 and 4096^2
    assert first(1e-3) > cap(512)
    assert abs(first(1e-3) - cap(1024)) / cap(1024) < 0.07
    assert first(1e-3) < cap(2048) and first(1e-3) < cap(4096)
    # eps = 1e-4: the cap is smaller on every grid
    assert all(cap(n) < first(1e-4) for n in sizes)
    assert cap(512) == pytest.approx(2.0 * 512 ** 0.25, rel=1e-15)
