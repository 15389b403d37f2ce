"""Direct pins of the oracle's small helpers (values worked out by hand or by
brute-force finite differences), in addition to their coverage through the
solvers that call them."""
import numpy as np
import pytest

from oracle import emd, grid, grid3, rof, unet


def test_pointwise_norms():
    # |(3, -4)|_2 = 5, |(3, -4)|_1 = 7; |(1, 2, -2)|_2 = 3, |.|_1 = 5
    assert grid.pointwise_norm(np.array([3.0]), np.array([-4.0]), grid.ISO)[0] == 5.0
    assert grid.pointwise_norm(np.array([3.0]), np.array([-4.0]), grid.ANISO)[0] == 7.0
    assert grid3.pointwise_norm(np.array([1.0]), np.array([2.0]), np.array([-2.0]), grid3.ISO)[0] == 3.0
    assert grid3.pointwise_norm(np.array([1.0]), np.array([2.0]), np.array([-2.0]), grid3.ANISO)[0] == 5.0


def test_dual_norm_max():
    # the dual of l2 is l2, the dual of l1 is l_inf; the max runs over cells
    gx, gy = np.array([[3.0, 0.5]]), np.array([[-4.0, 0.5]])
    assert grid.dual_norm_max(gx, gy, grid.ISO) == 5.0
    assert grid.dual_norm_max(gx, gy, grid.ANISO) == 4.0
    gz = np.array([[2.0, -6.0]])
    gx3, gy3 = np.array([[1.0, 0.0]]), np.array([[2.0, 0.0]])
    assert grid3.dual_norm_max(gx3, gy3, np.array([[-2.0, 0.0]]), grid3.ISO) == 3.0
    assert grid3.dual_norm_max(gx3, gy3, gz, grid3.ANISO) == 6.0


@pytest.mark.parametrize("f", [rof.rel_gap, emd.rel_gap, grid3.rel_gap])
def test_rel_gap(f):
    assert f(2.0, 1.5) == pytest.approx(0.25)
    assert f(-4.0, -5.0) == pytest.approx(0.25)  # divided by |P|
    assert f(0.0, -0.5) == pytest.approx(0.5)    # |P - D| when P = 0


def test_reflect():
    # R(y) = 2 proj(y) - y: identity inside the ball, a point beyond it maps
    # through the projection
    y = (np.array([0.3]), np.array([-0.4]), np.array([0.0]))
    q, R = grid3.reflect(y, grid3.ISO)
    assert np.allclose([r[0] for r in R], [0.3, -0.4, 0.0]) and np.allclose([a[0] for a in q], [0.3, -0.4, 0.0])
    q, R = grid3.reflect((np.array([2.0]), np.array([0.0]), np.array([0.0])), grid3.ISO)
    assert np.allclose([a[0] for a in q], [1.0, 0.0, 0.0]) and np.allclose([r[0] for r in R], [0.0, 0.0, 0.0])
    q, R = grid3.reflect((np.array([2.0]), np.array([-3.0]), np.array([0.5])), grid3.ANISO)
    assert np.allclose([a[0] for a in q], [1.0, -1.0, 0.5]) and np.allclose([r[0] for r in R], [0.0, 1.0, 0.5])


def test_relu_and_its_backward():
    X = np.array([-1.0, 0.0, 2.5])
    assert np.array_equal(unet.relu(X), [0.0, 0.0, 2.5])
    assert np.array_equal(unet.relu_bwd(unet.relu(X), np.array([7.0, 7.0, 7.0])), [0.0, 0.0, 7.0])


def test_head_and_its_backward_by_finite_differences():
    rng = np.random.default_rng(3)
    X = rng.standard_normal((2, 3, 4, 5))
    W = rng.standard_normal((1, 5))
    b = rng.standard_normal(1)
    # one hand value: phi = sum_c X[c] W[c] + b
    assert unet.head(X, W, b)[1, 2, 3] == pytest.approx(float(X[1, 2, 3] @ W[0] + b[0]))
    dphi = rng.standard_normal((2, 3, 4))
    dX, dW, db = unet.head_bwd(X, W, dphi)
    loss = lambda X_, W_, b_: float(np.sum(unet.head(X_, W_, b_) * dphi))
    eps = 1e-6
    for idx in [(0, 0, 0, 0), (1, 2, 3, 4), (0, 1, 2, 3)]:
        Xp, Xm = X.copy(), X.copy()
        Xp[idx] += eps
        Xm[idx] -= eps
        assert dX[idx] == pytest.approx((loss(Xp, W, b) - loss(Xm, W, b)) / (2 * eps), rel=1e-6, abs=1e-8)
    for c in range(5):
        Wp, Wm = W.copy(), W.copy()
        Wp[0, c] += eps
        Wm[0, c] -= eps
        assert dW[0, c] == pytest.approx((loss(X, Wp, b) - loss(X, Wm, b)) / (2 * eps), rel=1e-6, abs=1e-8)
    assert db[0] == pytest.approx((loss(X, W, b + eps) - loss(X, W, b - eps)) / (2 * eps), rel=1e-6)
