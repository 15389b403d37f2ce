"""Pins of the warm-start network oracle (oracle/unet.py) to things other than
itself: SciPy's correlation, explicit block constructions, adjointness, central
finite differences of the whole network and of the loss, and closed forms."""
import numpy as np
import pytest
from scipy import signal

from oracle import grid
from oracle import unet


def rng(s=0):
    return np.random.default_rng(s)


def test_conv3_matches_scipy_correlate():
    r = rng(1)
    X = r.standard_normal((2, 7, 9, 3))
    W = r.standard_normal((4, 3, 3, 3))
    b = r.standard_normal(4)
    Y = unet.conv3(X, W, b)
    for n in range(2):
        for o in range(4):
            ref = b[o] + sum(signal.correlate(X[n, :, :, i], W[o, :, :, i], mode="same") for i in range(3))
            np.testing.assert_allclose(Y[n, :, :, o], ref, rtol=0, atol=1e-12)


def fd_check(f, x, g, idx, eps=1e-6):
    """central difference of scalar f at x along the flat indices idx vs analytic g."""
    for i in idx:
        xp, xm = x.copy(), x.copy()
        xp.flat[i] += eps
        xm.flat[i] -= eps
        num = (f(xp) - f(xm)) / (2 * eps)
        assert abs(num - g.flat[i]) <= 1e-6 * max(1.0, abs(num)), (i, num, g.flat[i])


def test_conv3_bwd_finite_differences():
    r = rng(2)
    X = r.standard_normal((2, 5, 6, 3))
    W = r.standard_normal((4, 3, 3, 3))
    b = r.standard_normal(4)
    R = r.standard_normal((2, 5, 6, 4))
    dX, dW, db = unet.conv3_bwd(X, W, R)
    idx = r.integers(0, 10 ** 6, 12)
    fd_check(lambda x: np.sum(R * unet.conv3(x, W, b)), X, dX, idx % X.size)
    fd_check(lambda w: np.sum(R * unet.conv3(X, w, b)), W, dW, idx % W.size)
    fd_check(lambda bb: np.sum(R * unet.conv3(X, W, bb)), b, db, range(4))


def test_tconv2_block_construction_and_bwd():
    r = rng(3)
    X = r.standard_normal((1, 3, 4, 2))
    W = r.standard_normal((2, 2, 2, 5))
    b = r.standard_normal(5)
    Y = unet.tconv2(X, W, b)
    # each output channel is sum_c kron(X[..., c], W[c, :, :, o]) + b
    for o in range(5):
        ref = sum(np.kron(X[0, :, :, c], W[c, :, :, o]) for c in range(2)) + b[o]
        np.testing.assert_allclose(Y[0, :, :, o], ref, atol=1e-12)
    R = r.standard_normal(Y.shape)
    dX, dW, db = unet.tconv2_bwd(X, W, R)
    idx = r.integers(0, 10 ** 6, 10)
    fd_check(lambda x: np.sum(R * unet.tconv2(x, W, b)), X, dX, idx % X.size)
    fd_check(lambda w: np.sum(R * unet.tconv2(X, w, b)), W, dW, idx % W.size)
    fd_check(lambda bb: np.sum(R * unet.tconv2(X, W, bb)), b, db, range(5))


def test_pool_blocks_and_adjoint():
    r = rng(4)
    X = r.standard_normal((2, 6, 8, 3))
    P = unet.pool2(X)
    assert abs(P[1, 2, 3, 1] - X[1, 4:6, 6:8, 1].mean()) < 1e-14
    Y = r.standard_normal(P.shape)
    assert abs(np.sum(P * Y) - np.sum(X * unet.pool2_bwd(Y))) < 1e-12


def test_loss_gradient_finite_differences_and_gauge():
    r = rng(5)
    phi, star = r.standard_normal((2, 8, 8)), r.standard_normal((2, 8, 8))
    h = 1.0 / 8
    L, d = unet.loss(phi, star, h)
    fd_check(lambda p: unet.loss(p, star, h)[0], phi, d, r.integers(0, 128, 12))
    # a constant shift (the gauge) changes nothing; equal gradients give zero
    assert abs(unet.loss(phi + 3.0, star, h)[0] - L) < 1e-12
    assert unet.loss(star - 1.5, star, h)[0] < 1e-20
    # closed form on a linear ramp: grad = (1, 0) except the far face
    ramp = np.broadcast_to(np.arange(8) * h, (1, 8, 8)).copy()
    zero = np.zeros((1, 8, 8))
    assert abs(unet.loss(ramp, zero, h)[0] - 7 * 8 / 64) < 1e-12


@pytest.mark.parametrize("base", [2])
def test_network_backward_finite_differences(base):
    r = rng(6)
    P = unet.init_params(7, base)
    # non-zero biases so every path is exercised
    for k in P:
        P[k] = (P[k][0], r.standard_normal(P[k][1].shape) * 0.1)
    rho0 = 1 + 0.5 * r.standard_normal((2, 8, 8))
    rho1 = 1 + 0.5 * r.standard_normal((2, 8, 8))
    R = r.standard_normal((2, 8, 8))
    phi, c = unet.forward(P, rho0, rho1)
    G = unet.backward(P, c, R)
    blob = unet.to_blob(P, base)
    gblob = unet.to_blob(G, base)

    def f(bl):
        return float(np.sum(R * unet.forward(unet.from_blob(bl, base), rho0, rho1)[0]))
    # a few entries of every layer
    o, idx = 0, []
    for name, kind, cin, cout in unet.layer_specs(base):
        n = int(np.prod(unet.weight_shape(kind, cin, cout))) + cout
        idx += list(o + r.integers(0, n, 2)) + [o + n - 1]
        o += n
    assert o == blob.size == unet.n_params(base)
    fd_check(f, blob, gblob, idx, eps=1e-6)


def test_blob_roundtrip_and_count():
    P = unet.init_params(1)
    assert unet.n_params() == 1925313
    b = unet.to_blob(P)
    Q = unet.from_blob(b)
    for k in P:
        assert np.array_equal(P[k][0], Q[k][0]) and np.array_equal(P[k][1], Q[k][1])


def test_zero_weights_give_head_bias():
    P = unet.init_params(2, 2)
    for k in P:
        P[k] = (np.zeros_like(P[k][0]), np.zeros_like(P[k][1]))
    P["head"] = (P["head"][0], np.array([0.25]))
    phi, _ = unet.forward(P, np.ones((1, 16, 16)), np.ones((1, 16, 16)))
    assert np.all(phi == 0.25)


def test_adam_first_step_closed_form():
    w, g = np.array([1.0, -2.0, 3.0]), np.array([0.5, -4.0, 0.0])
    w1, m, v = unet.adam(w, g, np.zeros(3), np.zeros(3), 1, 0.01)
    # first bias-corrected step is lr * g / (|g| + eps)
    np.testing.assert_allclose(w1, w - 0.01 * g / (np.abs(g) + 1e-8), rtol=0, atol=1e-15)


def test_resolution_change():
    r = rng(8)
    rho = np.abs(r.standard_normal((16, 16))) + 0.1
    d = unet.downsample(rho, 4)
    assert abs(d.sum() * 16 - rho.sum()) < 1e-12  # mass on the unit square is kept
    # bilinear upsampling reproduces an affine function between the outermost centres
    c = np.add.outer(0.3 * np.arange(4), -0.2 * np.arange(4))
    up = unet.upsample_bilinear(c, 4)
    Y, X = np.meshgrid((np.arange(16) + 0.5) / 4 - 0.5, (np.arange(16) + 0.5) / 4 - 0.5, indexing="ij")
    inner = (Y >= 0) & (Y <= 3) & (X >= 0) & (X <= 3)
    np.testing.assert_allclose(up[inner], (0.3 * Y - 0.2 * X)[inner], atol=1e-12)
    # difference quotients bounded by 1 stay bounded by 1 (unit-square units)
    phi = r.standard_normal((8, 8))
    gx, gy = grid.grad(phi, 1 / 8)
    phi = phi / max(np.abs(gx).max(), np.abs(gy).max())
    gx, gy = grid.grad(unet.upsample_bilinear(phi, 4), 1 / 32)
    assert max(np.abs(gx).max(), np.abs(gy).max()) <= 1 + 1e-12
