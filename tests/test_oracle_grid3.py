"""Pins of the 3-D oracle (oracle/grid3.py) against things other than itself:
the adjoint identity, a dense linear solve of the assembled 7-point operator,
exact reduction to the pinned 2-D oracle for data constant along one axis
(each axis in turn, both norms), the 1-D closed form of the EMD for
densities that vary along z only, the ROF invariants (mean preservation,
maximum principle, weak duality), and, on volumes with structure along every
axis, the anisotropic EMD against a linear program and a min-cost flow and the
anisotropic ROF against a box-constrained maximisation of its dual, and the
isotropic ROF inside the primal-dual bracket of an accelerated projected
gradient on its dual, and the isotropic EMD inside a polygonal-LP bracket (all with the divergence assembled in the test from its
definition)."""
import numpy as np
import pytest

from oracle import emd as oemd
from oracle import grid
from oracle import grid3 as g3
from oracle import rof as orof

RNG = np.random.default_rng(20260303)


def test_adjointness():
    h = 0.37
    u = RNG.standard_normal((5, 6, 7))
    p = tuple(RNG.standard_normal((5, 6, 7)) for _ in range(3))
    # far-face components of p are structurally zero
    p[0][:, :, -1] = 0
    p[1][:, -1, :] = 0
    p[2][-1, :, :] = 0
    lhs = h ** 3 * sum(float(np.sum(a * b)) for a, b in zip(g3.grad(u, h), p))
    rhs = -h ** 3 * float(np.sum(u * g3.div(*p, h)))
    assert abs(lhs - rhs) <= 1e-13 * abs(lhs)


@pytest.mark.parametrize("alpha", [0.7, 0.0])
def test_poisson_against_dense_solve(alpha):
    nz, ny, nx, h = 3, 4, 5, 0.5
    n = nz * ny * nx
    A = np.zeros((n, n))
    for k in range(n):
        e = np.zeros(n)
        e[k] = 1.0
        A[:, k] = alpha * e - g3.laplacian(e.reshape(nz, ny, nx), h).ravel()
    b = RNG.standard_normal((nz, ny, nx))
    x = g3.poisson_solve(b, h, alpha)
    if alpha > 0:
        ref = np.linalg.solve(A, b.ravel())
    else:
        ref = np.linalg.lstsq(A, (b - b.mean()).ravel(), rcond=None)[0]
        ref -= ref.mean()
    assert np.abs(x.ravel() - ref).max() <= 1e-12 * np.abs(ref).max()


def _embed(a2, axis, n):
    """a 2-D field repeated n times along the given 3-D axis"""
    return np.repeat(np.expand_dims(a2, axis), n, axis=axis)


# for data constant along `axis`, the 3-D components that map to the 2-D (x, y) ones
# (the 2-D array's last axis is its x): axis 0 (z): (x, y); axis 1 (y): (x, z); axis 2 (x): (y, z)
COMP = {0: (0, 1), 1: (0, 2), 2: (1, 2)}


@pytest.mark.parametrize("axis", [0, 1, 2])
@pytest.mark.parametrize("norm", [grid.ISO, grid.ANISO])
def test_rof_reduces_to_2d(axis, norm):
    J = RNG.random((12, 10))
    I = _embed(J, axis, 6)
    h, lam, tau = 0.9, 8.0, 0.05
    u3 = np.zeros_like(I)
    p3 = tuple(np.zeros_like(I) for _ in range(3))
    pb3 = tuple(a.copy() for a in p3)
    z = np.zeros_like(J)
    s2 = (z, z.copy(), z.copy(), z.copy(), z.copy())
    cx, cy = COMP[axis]
    for _ in range(5):
        u3, p3, pb3 = g3.rof_step(u3, p3, pb3, I, h, lam, tau, 1 / tau, norm)
        s2 = orof.step(*s2, J, h, lam, tau, 1 / tau, norm)
    assert np.abs(u3 - _embed(s2[0], axis, 6)).max() <= 1e-12
    assert np.abs(p3[cx] - _embed(s2[1], axis, 6)).max() <= 1e-12
    assert np.abs(p3[cy] - _embed(s2[2], axis, 6)).max() <= 1e-12
    assert np.abs(p3[axis_component(axis)]).max() == 0.0
    # values: h^3 sums over 6 slices = 6 h times the 2-D h^2 sums
    P3, P2 = g3.rof_primal(u3, I, h, lam, norm), orof.primal(s2[0], J, h, lam, norm)
    D3, D2 = g3.rof_dual(*p3, I, h, lam), orof.dual(s2[1], s2[2], J, h, lam)
    assert abs(P3 - 6 * h * P2) <= 1e-12 * abs(P3)
    assert abs(D3 - 6 * h * D2) <= 1e-12 * abs(P3)


def axis_component(axis):
    """the gradient component along the constant axis (x is component 0)"""
    return {0: 2, 1: 1, 2: 0}[axis]


@pytest.mark.parametrize("axis", [0, 2])
def test_emd_reduces_to_2d(axis):
    n2 = 16
    h = 1.0 / n2
    a = RNG.random((n2, n2)) + 0.5
    b = RNG.random((n2, n2)) + 0.5
    b *= a.sum() / b.sum()
    r0, r1 = _embed(a, axis, 4), _embed(b, axis, 4)
    f3, psi3 = g3.emd_setup(r0, r1, h)
    f2, psi2 = oemd.setup(a, b, h)
    assert np.abs(psi3 - _embed(psi2, axis, 4)).max() <= 1e-12 * np.abs(psi2).max()
    gp3 = g3.grad(psi3, h)
    gp2 = grid.grad(psi2, h)
    tau = 0.3
    u3 = tuple(np.zeros_like(f3) for _ in range(3))
    p3 = tuple(np.zeros_like(f3) for _ in range(3))
    pb3 = tuple(x.copy() for x in p3)
    z = np.zeros_like(f2)
    s2 = (z, z.copy(), z.copy(), z.copy(), z.copy(), z.copy())
    cx, cy = COMP[axis]
    for _ in range(6):
        u3, p3, pb3 = g3.emd_step(u3, p3, pb3, gp3, h, tau, 1 / tau)
        s2 = oemd.step(*s2, gp2[0], gp2[1], h, tau, 1 / tau)
    scale = np.abs(s2[0]).max() + np.abs(s2[2]).max()
    assert np.abs(u3[cx] - _embed(s2[0], axis, 4)).max() <= 1e-11 * scale
    assert np.abs(u3[cy] - _embed(s2[1], axis, 4)).max() <= 1e-11 * scale
    assert np.abs(p3[cx] - _embed(s2[2], axis, 4)).max() <= 1e-11 * scale
    assert np.abs(p3[cy] - _embed(s2[3], axis, 4)).max() <= 1e-11 * scale
    P3, P2 = g3.emd_primal(u3, gp3, h), oemd.primal(s2[0], s2[1], gp2[0], gp2[1], h)
    D3, D2 = g3.emd_certificate(p3, f3, h)[0], oemd.certificate(s2[2], s2[3], f2, h)[0]
    assert abs(P3 - 4 * h * P2) <= 1e-10 * P3 and abs(D3 - 4 * h * D2) <= 1e-10 * P3


def test_emd_z_only_closed_form():
    """Densities varying along z only: EMD = (area of a z-slice) x the 1-D value
    h sum_k |C_k|, C_k = h sum_{j<=k} (rho1_j - rho0_j); the starting flux
    grad psi is already optimal and the certificate stays below it."""
    nz, ny, nx = 32, 4, 4
    h = 1.0 / nz
    z = (np.arange(nz) + 0.5) * h
    a = np.exp(-((z - 0.3) / 0.08) ** 2) + 1e-3
    b = np.exp(-((z - 0.6) / 0.1) ** 2) + 1e-3
    b *= a.sum() / b.sum()
    C = h * np.cumsum(b - a)
    exact = (nx * h) * (ny * h) * h * float(np.sum(np.abs(C)))
    r0 = np.broadcast_to(a[:, None, None], (nz, ny, nx)).copy()
    r1 = np.broadcast_to(b[:, None, None], (nz, ny, nx)).copy()
    f, psi = g3.emd_setup(r0, r1, h)
    gp = g3.grad(psi, h)
    P0 = g3.emd_primal(tuple(np.zeros_like(f) for _ in range(3)), gp, h)
    assert abs(P0 - exact) <= 1e-12 * exact
    res = g3.emd_solve(r0, r1, h, tau=0.3, tol=0.0, max_iter=300, check_every=300)
    assert res.dual <= exact * (1 + 1e-12) and abs(res.primal - exact) <= 1e-6 * exact
    assert res.rel_gap < 0.05


def test_rof_converges_with_invariants():
    I = np.zeros((16, 16, 16))
    I[3:9, 4:12, 2:7] = 1.0
    I[8:14, 1:6, 9:15] = 0.5
    I += 0.1 * np.random.default_rng(7).standard_normal(I.shape)
    h, lam = 1.0, 8.0
    res = g3.rof_solve(I, h, lam, 0.01, tol=1e-6, max_iter=20000, check_every=20)
    assert res.converged and res.dual <= res.primal
    assert abs(res.u.sum() - I.sum()) <= 1e-9 * np.abs(I).sum()
    assert res.u.min() >= I.min() - 1e-6 and res.u.max() <= I.max() + 1e-6
    # field bound of the strongly convex problem, ||u - u*||^2 <= 2 gap / lambda (h^3 norm),
    # against a tighter solve (its own distance to u* bounded the same way)
    ref = g3.rof_solve(I, h, lam, 0.01, tol=2e-8, max_iter=40000, check_every=20)
    assert ref.converged and ref.rel_gap < 0.05 * res.rel_gap
    dist = np.sqrt(h ** 3 * float(np.sum((res.u - ref.u) ** 2)))
    bound = np.sqrt(2 * (res.primal - res.dual) / lam) + np.sqrt(2 * (ref.primal - ref.dual) / lam)
    assert dist <= bound
    assert dist >= 1e-3 * bound  # (the bound is not vacuous: the two solves differ)


@pytest.mark.parametrize("norm", [grid.ISO, grid.ANISO])
def test_single_variable_rof_equals_the_two_variable_iteration(norm):
    """sigma = 1/tau: from y_0 = 0 the single-variable iteration reproduces the
    iterates of rof_step from the zero start, u_n and p_n = proj(y_n)."""
    rng = np.random.default_rng(31)
    I = rng.random((6, 8, 10))
    h, lam, tau = 0.7, 8.0, 0.3
    u = np.zeros_like(I)
    p = tuple(np.zeros_like(I) for _ in range(3))
    pb = tuple(a.copy() for a in p)
    y = tuple(np.zeros_like(I) for _ in range(3))
    for _ in range(12):
        u, p, pb = g3.rof_step(u, p, pb, I, h, lam, tau, 1 / tau, norm)
        u2, y = g3.rof_drs_step(y, I, h, lam, tau, norm)
        q = g3.project_unit_ball(*y, norm)
        assert np.abs(u2 - u).max() <= 1e-12 * np.abs(u).max()
        assert max(np.abs(a - b).max() for a, b in zip(q, p)) <= 1e-12


@pytest.mark.parametrize("norm", [grid.ISO, grid.ANISO])
def test_single_variable_emd_equals_the_two_variable_iteration(norm):
    rng = np.random.default_rng(32)
    a = rng.random((8, 8, 8)) + 0.5
    b = rng.random((8, 8, 8)) + 0.5
    b *= a.sum() / b.sum()
    h, tau = 1.0 / 8, 0.4
    f, psi = g3.emd_setup(a, b, h)
    gp = g3.grad(psi, h)
    u = tuple(np.zeros_like(f) for _ in range(3))
    p = tuple(np.zeros_like(f) for _ in range(3))
    pb = tuple(x.copy() for x in p)
    y = tuple(np.zeros_like(f) for _ in range(3))
    for _ in range(12):
        u, p, pb = g3.emd_step(u, p, pb, gp, h, tau, 1 / tau, norm)
        u2, y = g3.emd_drs_step(y, gp, h, tau, norm)
        q = g3.project_unit_ball(*y, norm)
        scale = max(np.abs(x).max() for x in u) + 1.0
        assert max(np.abs(x - z).max() for x, z in zip(u2, u)) <= 1e-12 * scale
        assert max(np.abs(x - z).max() for x, z in zip(q, p)) <= 1e-12


def test_ergodic_averages_are_the_means_and_bracket_the_optimum():
    """ergodic=True returns (1/N) sum_{n<=N} of the iterates (against a separate
    step loop) and, the averages being feasible, D <= F* <= P brackets the
    optimum (ROF: F* from a tight solve; EMD: the certificate below the primal)."""
    rng = np.random.default_rng(41)
    I = rng.random((6, 8, 8))
    h, lam, tau, K = 1.0, 8.0, 0.05, 7
    u = np.zeros_like(I)
    p = tuple(np.zeros_like(I) for _ in range(3))
    pb = tuple(a.copy() for a in p)
    acc = [np.zeros_like(I) for _ in range(4)]
    for _ in range(K):
        u, p, pb = g3.rof_step(u, p, pb, I, h, lam, tau, 1 / tau)
        for a, x in zip(acc, (u,) + p):
            a += x
    r = g3.rof_solve(I, h, lam, tau, tol=0.0, max_iter=K, check_every=K, ergodic=True)
    for got, a in zip((r.u,) + r.p, acc):
        np.testing.assert_allclose(got, a / K, rtol=0, atol=1e-14)
    assert abs(r.primal - g3.rof_primal(acc[0] / K, I, h, lam)) < 1e-12
    fstar = g3.rof_solve(I, h, lam, tau, tol=1e-10, max_iter=100000, check_every=50).primal
    assert r.dual <= fstar * (1 + 1e-12) <= r.primal * (1 + 2e-12)
    a = rng.random((8, 8, 8)) + 0.5
    b = rng.random((8, 8, 8)) + 0.5
    b *= a.sum() / b.sum()
    e = g3.emd_solve(a, b, 1 / 8, tau=0.3, tol=0.0, max_iter=K, check_every=K, ergodic=True)
    f, psi = g3.emd_setup(a, b, 1 / 8)
    gp = g3.grad(psi, 1 / 8)
    u = tuple(np.zeros_like(f) for _ in range(3))
    p = tuple(np.zeros_like(f) for _ in range(3))
    pb = tuple(x.copy() for x in p)
    acc = [np.zeros_like(f) for _ in range(6)]
    for _ in range(K):
        u, p, pb = g3.emd_step(u, p, pb, gp, 1 / 8, 0.3, 1 / 0.3)
        for s_, x in zip(acc, u + p):
            s_ += x
    for got, s_ in zip(e.u + e.p, acc):
        np.testing.assert_allclose(got, s_ / K, rtol=0, atol=1e-14)
    assert e.dual <= e.primal


def test_single_variable_emd_from_a_warm_start():
    """A warm start u0 = 0, p0 = pbar0 = proj(grad phi0) is y0 = p0 in the
    single-variable form: the iterates agree with the two-variable ones."""
    rng = np.random.default_rng(43)
    a = rng.random((8, 8, 8)) + 0.5
    b = rng.random((8, 8, 8)) + 0.5
    b *= a.sum() / b.sum()
    h, tau = 1.0 / 8, 0.4
    f, psi = g3.emd_setup(a, b, h)
    gp = g3.grad(psi, h)
    phi0 = 0.7 * rng.standard_normal((8, 8, 8)) * h
    p0 = g3.project_unit_ball(*g3.grad(phi0, h))
    u = tuple(np.zeros_like(f) for _ in range(3))
    p, pb, y = p0, p0, p0
    for _ in range(8):
        u, p, pb = g3.emd_step(u, p, pb, gp, h, tau, 1 / tau)
        u2, y = g3.emd_drs_step(y, gp, h, tau)
        q = g3.project_unit_ball(*y)
        assert max(np.abs(x - z).max() for x, z in zip(u2, u)) <= 1e-12 * (1 + max(np.abs(x).max() for x in u))
        assert max(np.abs(x - z).max() for x, z in zip(q, p)) <= 1e-12
    # and the solve's warm start is that start
    r = g3.emd_solve(a, b, h, tau=tau, tol=0.0, max_iter=8, check_every=8, phi0=phi0)
    assert max(np.abs(x - z).max() for x, z in zip(r.p, p)) <= 1e-12


def _face_divergence(nz, ny, nx, h):
    """Divergence of a face field assembled from its definition, independently of
    oracle/grid3.py: one variable per interior face (x faces, then y, then z;
    far-face components are zero and have no variable), each entering the cell
    on its low side with +1/h and the cell on its high side with -1/h (backward
    differences).  Returns the (cells x faces) matrix."""
    cell = np.arange(nz * ny * nx).reshape(nz, ny, nx)
    cols = []
    for (dz, dy, dx) in ((0, 0, 1), (0, 1, 0), (1, 0, 0)):
        lo = cell[:nz - dz, :ny - dy, :nx - dx].ravel()
        hi = cell[dz:, dy:, dx:].ravel()
        for a, b in zip(lo, hi):
            c = np.zeros(nz * ny * nx)
            c[a], c[b] = 1.0 / h, -1.0 / h
            cols.append(c)
    return np.array(cols).T


def test_emd_anisotropic_3d_matches_lp_and_min_cost_flow():
    """Anisotropic 3-D EMD of integer masses on a 4x4x4 grid (all three axes
    carry flux): the oracle's converged value equals the Beckmann linear program
    min h^3 sum |m| s.t. div m = rho1 - rho0, assembled here from the
    definition, and the min-cost flow on the 6-neighbour grid graph."""
    import networkx as nx_
    from scipy.optimize import linprog
    n, h = 4, 0.25
    rng = np.random.default_rng(41)
    c0 = rng.integers(0, 6, (n, n, n))
    c1 = rng.integers(0, 6, (n, n, n))
    c1[0, 0, 0] += c0.sum() - c1.sum() if c0.sum() >= c1.sum() else 0
    c0[0, 0, 0] += c1.sum() - c0.sum() if c1.sum() > c0.sum() else 0
    assert c0.sum() == c1.sum()
    rho0, rho1 = c0 / (c0.sum() * h ** 3), c1 / (c1.sum() * h ** 3)
    A = _face_divergence(n, n, n, h)
    f = (rho1 - rho0).ravel()
    nf = A.shape[1]
    lp = linprog(h ** 3 * np.ones(2 * nf), A_eq=np.hstack([A, -A]), b_eq=f, bounds=(0, None), method="highs")
    G = nx_.DiGraph()
    for k in range(n):
        for i in range(n):
            for j in range(n):
                G.add_node((k, i, j), demand=int(c1[k, i, j] - c0[k, i, j]))
                for d in ((0, 0, 1), (0, 1, 0), (1, 0, 0), (0, 0, -1), (0, -1, 0), (-1, 0, 0)):
                    q = (k + d[0], i + d[1], j + d[2])
                    if all(0 <= x < n for x in q):
                        G.add_edge((k, i, j), q, weight=1)
    v_flow = h * nx_.min_cost_flow_cost(G) / float(c0.sum())
    assert abs(lp.fun - v_flow) <= 1e-12 * v_flow
    r = g3.emd_solve(rho0, rho1, h, tau=0.3, tol=1e-10, max_iter=200000, check_every=10, norm=g3.ANISO)
    assert r.converged
    assert r.dual <= v_flow * (1 + 1e-12) <= r.primal * (1 + 2e-12)
    assert abs(r.primal - v_flow) <= 1e-9 * v_flow


def test_rof_anisotropic_3d_matches_box_constrained_dual():
    """Anisotropic 3-D ROF on a 4x4x4 volume with structure along every axis:
    the oracle's converged energy equals the maximum of the dual
    -h^3 I.(A p) - h^3/(2 lambda) |A p|^2 over the box |p| <= 1 (the l-infinity
    ball, dual of the l1 norm), with A the face divergence assembled here and the
    maximum found by L-BFGS-B; the minimiser is I + A p / lambda."""
    from scipy.optimize import minimize
    n, h, lam = 4, 1.0, 3.0
    rng = np.random.default_rng(43)
    I = np.zeros((n, n, n))
    I[1:3, 0:3, 1:4] = 1.0
    I[2:4, 2:4, 0:2] += 0.6
    I += 0.2 * rng.standard_normal(I.shape)
    A = _face_divergence(n, n, n, h)
    Iv = I.ravel()

    def neg_dual(p):
        d = A @ p
        val = -h ** 3 * (Iv @ d) - h ** 3 / (2 * lam) * (d @ d)
        grad_ = -h ** 3 * (A.T @ (Iv + d / lam))
        return -val, -grad_

    res = minimize(neg_dual, np.zeros(A.shape[1]), jac=True, method="L-BFGS-B",
                   bounds=[(-1.0, 1.0)] * A.shape[1], options=dict(ftol=1e-16, gtol=1e-13, maxiter=50000))
    d_star = -res.fun
    u_star = (Iv + A @ res.x / lam).reshape(I.shape)
    r = g3.rof_solve(I, h, lam, 0.05, tol=1e-11, max_iter=200000, check_every=10, norm=g3.ANISO)
    assert r.converged
    assert r.dual <= d_star * (1 + 1e-9) and d_star <= r.primal * (1 + 1e-12)
    assert abs(r.primal - d_star) <= 1e-9 * abs(d_star)
    # strong convexity: h^3 |u - u*|^2 <= 2 (P(u) - P*) / lambda
    assert np.sqrt(h ** 3 * np.sum((r.u - u_star) ** 2)) <= 1e-4


def test_rof_isotropic_3d_inside_an_independent_dual_bracket():
    """Isotropic 3-D ROF on a 4x4x4 volume with structure along every axis: the
    oracle's converged energy lies in the bracket [D(p), P(I + A p / lambda)]
    that accelerated projected gradient (FISTA) on the dual reaches, with A the
    face divergence assembled in the test and the unit l2 ball taken over the
    three faces each cell owns (its x, y and z faces on the high side), a
    method and operators shared with nothing in oracle/grid3.py."""
    n, h, lam = 4, 1.0, 3.0
    rng = np.random.default_rng(47)
    I = np.zeros((n, n, n))
    I[0:3, 1:4, 1:3] = 1.0
    I[2:4, 0:2, 2:4] += 0.7
    I += 0.2 * rng.standard_normal(I.shape)
    Iv = I.ravel()
    A = _face_divergence(n, n, n, h)
    owner = np.argmax(A > 0, axis=0)  # the cell on a face's low side

    def proj(p):
        s = np.maximum(1.0, np.sqrt(np.bincount(owner, p * p, minlength=A.shape[0])))
        return p / s[owner]

    def dual(p):
        d = A @ p
        return -h ** 3 * (Iv @ d) - h ** 3 / (2 * lam) * (d @ d)

    def primal(u):
        g = -(A.T @ u)  # forward differences
        return h ** 3 * np.sum(np.sqrt(np.bincount(owner, g * g, minlength=A.shape[0]))) + \
            0.5 * lam * h ** 3 * np.sum((u - Iv) ** 2)

    L = h ** 3 * np.linalg.norm(A, 2) ** 2 / lam
    p = np.zeros(A.shape[1])
    q, t = p.copy(), 1.0
    for _ in range(20000):
        p_new = proj(q + (h ** 3 * (A.T @ (Iv + (A @ q) / lam))) * (-1.0 / L))
        t_new = 0.5 * (1 + np.sqrt(1 + 4 * t * t))
        q = p_new + ((t - 1) / t_new) * (p_new - p)
        p, t = p_new, t_new
    lo, hi = dual(p), primal(Iv + A @ p / lam)
    assert hi - lo <= 1e-7 * abs(hi)
    r = g3.rof_solve(I, h, lam, 0.05, tol=1e-10, max_iter=200000, check_every=10)
    assert r.converged
    assert lo * (1 - 1e-12) <= r.primal and r.dual <= hi * (1 + 1e-12)
    assert abs(r.primal - hi) <= 2e-7 * abs(hi)


def test_emd_isotropic_3d_inside_a_polygonal_lp_bracket():
    """Isotropic 3-D EMD of a 4x4x4 pair with structure along every axis.  With
    unit directions d_k (a Fibonacci sphere), max_k <d_k, m> <= |m|_2 per cell,
    so the linear program min h^3 sum_c t_c, t_c >= <d_k, m_c>, div m = f is a
    lower bound, and the l2 cost of its own feasible flux an upper bound; the
    oracle's converged value lies in that bracket (divergence assembled in the
    test; each cell's vector is its x, y and z faces on the high side)."""
    import scipy.sparse as sp
    from scipy.optimize import linprog
    n, h, K = 4, 0.25, 1600
    rng = np.random.default_rng(53)
    rho0 = rng.random((n, n, n)) + 0.2
    rho1 = rng.random((n, n, n)) + 0.2
    rho1 *= rho0.sum() / rho1.sum()
    A = _face_divergence(n, n, n, h)
    nc, nf = A.shape
    owner = np.argmax(A > 0, axis=0)
    axis_of = np.concatenate([np.full(n * n * (n - 1), a) for a in range(3)])  # x faces, y faces, z faces
    k = np.arange(K) + 0.5
    zc = 1 - 2 * k / K
    th = np.pi * (1 + 5 ** 0.5) * k
    D = np.stack([np.sqrt(1 - zc * zc) * np.cos(th), np.sqrt(1 - zc * zc) * np.sin(th), zc], axis=1)
    # rows (cell c, direction j): sum over c's faces of d_j[axis] m_face - t_c <= 0
    rows, cols, vals = [], [], []
    for fidx in range(nf):
        c, a = owner[fidx], axis_of[fidx]
        for j in range(K):
            rows.append(c * K + j)
            cols.append(fidx)
            vals.append(D[j, a])
    for c in range(nc):
        for j in range(K):
            rows.append(c * K + j)
            cols.append(nf + c)
            vals.append(-1.0)
    Aub = sp.csr_matrix((vals, (rows, cols)), shape=(nc * K, nf + nc))
    f = (rho1 - rho0).ravel()
    f = f - f.mean()
    Aeq = sp.hstack([sp.csr_matrix(A), sp.csr_matrix((nc, nc))])
    res = linprog(np.concatenate([np.zeros(nf), h ** 3 * np.ones(nc)]), A_ub=Aub, b_ub=np.zeros(nc * K),
                  A_eq=Aeq, b_eq=f, bounds=(None, None), method="highs")
    assert res.status == 0
    m = res.x[:nf]
    assert np.abs(A @ m - f).max() <= 1e-9 * np.abs(f).max()
    lo = res.fun
    hi = h ** 3 * np.sum(np.sqrt(np.bincount(owner, m * m, minlength=nc)))
    assert hi - lo <= 2e-3 * hi
    r = g3.emd_solve(rho0, rho1, h, tau=0.3, tol=1e-9, max_iter=200000, check_every=10)
    assert r.converged
    assert lo * (1 - 1e-12) <= r.primal and r.dual <= hi * (1 + 1e-12)
