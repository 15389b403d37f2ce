"""FP64 reference of the learned warm start for the EMD iteration.

TEST INFRASTRUCTURE ONLY (see the package docstring).

The warm start is not part of the paper.  It predicts an initial dual
potential phi0 from the two densities; the EMD iteration of section 3.2
(Algorithm 2) then starts from p0 = proj(grad phi0), u0 = 0, and its duality
gap still decides when the solve is done.  At a saddle point of that iteration the dual
p is a gradient field (its divergence-free part vanishes) bounded by 1, i.e.
the gradient of a 1-Lipschitz Kantorovich potential, which is what the
network is trained to approximate.

Network (a 4-level U-Net, plain definitions, NHWC arrays (batch, y, x, c)):
  input      x = (rho0 - 1, rho1 - 1)                      2 channels
  encoder    per level: two 3x3 convolutions (zero padding), each + ReLU;
             2x2 average pooling between levels; widths base, 2b, 4b, 8b
  decoder    per level: 2x2 stride-2 transposed convolution (no activation),
             concatenation [upsampled, encoder skip], two 3x3 conv + ReLU
  head       1x1 convolution to one channel (no activation): phi
Parameter blob (FP32, layer after layer, weights then bias): 3x3 conv
weights are [cout][3][3][cin] (tap (ky, kx) reads the input at offset
(ky - 1, kx - 1)); transposed-conv weights are [cin][2][2][cout] (output
pixel (2y + i, 2x + j) takes input pixel (y, x) times W[:, i, j, :]); the
head is [1][cin] and one bias.

Loss: the gauge-invariant mean squared gradient error
  L = 1/(B ny nx) sum |grad_h phi - grad_h phi*|^2
with the forward-difference gradient of ``grid`` (h = 1/n: phi in unit-square
units, where an optimal potential is 1-Lipschitz).

Every function is a direct transcription of its definition with NumPy loops
over taps; the tests pin them to scipy.signal.correlate, explicit block
constructions, adjointness and central finite differences.
"""
from __future__ import annotations

import numpy as np

from . import grid

BASE = 32


def layer_specs(base: int = BASE):
    """[(name, kind, cin, cout)] in parameter-blob order."""
    c0, c1, c2, c3 = base, 2 * base, 4 * base, 8 * base
    return [("enc0a", "conv3", 2, c0), ("enc0b", "conv3", c0, c0),
            ("enc1a", "conv3", c0, c1), ("enc1b", "conv3", c1, c1),
            ("enc2a", "conv3", c1, c2), ("enc2b", "conv3", c2, c2),
            ("mid_a", "conv3", c2, c3), ("mid_b", "conv3", c3, c3),
            ("up2", "tconv2", c3, c2), ("dec2a", "conv3", 2 * c2, c2), ("dec2b", "conv3", c2, c2),
            ("up1", "tconv2", c2, c1), ("dec1a", "conv3", 2 * c1, c1), ("dec1b", "conv3", c1, c1),
            ("up0", "tconv2", c1, c0), ("dec0a", "conv3", 2 * c0, c0), ("dec0b", "conv3", c0, c0),
            ("head", "conv1", c0, 1)]


def weight_shape(kind, cin, cout):
    return {"conv3": (cout, 3, 3, cin), "tconv2": (cin, 2, 2, cout), "conv1": (cout, cin)}[kind]


def init_params(seed: int, base: int = BASE):
    """He-normal weights (fan-in of the layer), zero biases."""
    rng = np.random.default_rng(seed)
    P = {}
    for name, kind, cin, cout in layer_specs(base):
        shp = weight_shape(kind, cin, cout)
        fan_in = {"conv3": 9 * cin, "tconv2": cin, "conv1": cin}[kind]
        P[name] = (rng.standard_normal(shp) * np.sqrt(2.0 / fan_in), np.zeros(cout))
    return P


def to_blob(P, base: int = BASE) -> np.ndarray:
    parts = []
    for name, _, _, _ in layer_specs(base):
        W, b = P[name]
        parts += [np.asarray(W, np.float64).ravel(), np.asarray(b, np.float64).ravel()]
    return np.concatenate(parts)


def from_blob(blob, base: int = BASE):
    P, o = {}, 0
    for name, kind, cin, cout in layer_specs(base):
        shp = weight_shape(kind, cin, cout)
        nw = int(np.prod(shp))
        P[name] = (np.asarray(blob[o:o + nw], np.float64).reshape(shp), np.asarray(blob[o + nw:o + nw + cout],
                                                                                    np.float64))
        o += nw + cout
    return P


def n_params(base: int = BASE) -> int:
    return sum(int(np.prod(weight_shape(k, ci, co))) + co for _, k, ci, co in layer_specs(base))


# ---------------------------------------------------------------- layers
def conv3(X, W, b):
    """Y[n,y,x,o] = b[o] + sum_{ky,kx,i} X[n, y+ky-1, x+kx-1, i] W[o,ky,kx,i] (zero outside)."""
    B, H, Wd, _ = X.shape
    Xp = np.pad(X, ((0, 0), (1, 1), (1, 1), (0, 0)))
    Y = np.zeros((B, H, Wd, W.shape[0])) + b
    for ky in range(3):
        for kx in range(3):
            Y += Xp[:, ky:ky + H, kx:kx + Wd, :] @ W[:, ky, kx, :].T
    return Y


def conv3_bwd(X, W, dY):
    """Gradients of <dY, conv3(X, W, b)> with respect to X, W, b."""
    B, H, Wd, _ = X.shape
    Xp = np.pad(X, ((0, 0), (1, 1), (1, 1), (0, 0)))
    dXp = np.zeros_like(Xp)
    dW = np.zeros_like(W)
    for ky in range(3):
        for kx in range(3):
            win = Xp[:, ky:ky + H, kx:kx + Wd, :]
            dW[:, ky, kx, :] = np.einsum("nhwo,nhwi->oi", dY, win)
            dXp[:, ky:ky + H, kx:kx + Wd, :] += dY @ W[:, ky, kx, :]
    return dXp[:, 1:-1, 1:-1, :], dW, dY.sum(axis=(0, 1, 2))


def relu(X):
    return np.maximum(X, 0.0)


def relu_bwd(Y, dY):
    """Y is the ReLU output; the derivative is 1 where Y > 0."""
    return dY * (Y > 0)


def pool2(X):
    B, H, Wd, C = X.shape
    return X.reshape(B, H // 2, 2, Wd // 2, 2, C).mean(axis=(2, 4))


def pool2_bwd(dY):
    return np.repeat(np.repeat(dY, 2, axis=1), 2, axis=2) / 4.0


def tconv2(X, W, b):
    """Y[n, 2y+i, 2x+j, o] = b[o] + sum_c X[n,y,x,c] W[c,i,j,o]."""
    B, H, Wd, _ = X.shape
    Y = np.zeros((B, 2 * H, 2 * Wd, W.shape[3]))
    for i in range(2):
        for j in range(2):
            Y[:, i::2, j::2, :] = X @ W[:, i, j, :] + b
    return Y


def tconv2_bwd(X, W, dY):
    dX = np.zeros_like(X)
    dW = np.zeros_like(W)
    for i in range(2):
        for j in range(2):
            g = dY[:, i::2, j::2, :]
            dX += g @ W[:, i, j, :].T
            dW[:, i, j, :] = np.einsum("nhwc,nhwo->co", X, g)
    return dX, dW, dY.sum(axis=(0, 1, 2))


def head(X, W, b):
    return X @ W[0] + b[0]


def head_bwd(X, W, dphi):
    return dphi[..., None] * W[0], np.einsum("nhwc,nhw->c", X, dphi)[None, :], np.array([dphi.sum()])


# ---------------------------------------------------------------- network
def _same(a):
    return a


def forward(P, rho0, rho1, rnd=None):
    """rho0, rho1: (B, H, W) with H, W multiples of 8.  Returns (phi (B,H,W), cache).
    rnd (optional) is applied to every stored activation (the input, each layer
    output); it models a storage format such as BF16 and defaults to none."""
    r = rnd or _same
    x = r(np.stack([np.asarray(rho0, np.float64) - 1.0, np.asarray(rho1, np.float64) - 1.0], axis=-1))
    c = {"x": x}
    h = x
    skips = []
    for lvl, (a, bn) in enumerate((("enc0a", "enc0b"), ("enc1a", "enc1b"), ("enc2a", "enc2b"))):
        c[a + "_in"] = h
        h = r(relu(conv3(h, *P[a])))
        c[a] = h
        h = r(relu(conv3(h, *P[bn])))
        c[bn] = h
        skips.append(h)
        h = r(pool2(h))
    c["mid_a_in"] = h
    h = r(relu(conv3(h, *P["mid_a"])))
    c["mid_a"] = h
    h = r(relu(conv3(h, *P["mid_b"])))
    c["mid_b"] = h
    for up, a, bn, skip in (("up2", "dec2a", "dec2b", skips[2]), ("up1", "dec1a", "dec1b", skips[1]),
                            ("up0", "dec0a", "dec0b", skips[0])):
        c[up + "_in"] = h
        h = r(tconv2(h, *P[up]))
        h = np.concatenate([h, skip], axis=-1)
        c[a + "_in"] = h
        h = r(relu(conv3(h, *P[a])))
        c[a] = h
        h = r(relu(conv3(h, *P[bn])))
        c[bn] = h
    c["head_in"] = h
    return head(h, *P["head"]), c


def backward(P, c, dphi, rnd=None):
    """Parameter gradients {name: (dW, db)} of <dphi, forward(P, ...)>; rnd (optional)
    is applied to every stored activation gradient."""
    r = rnd or _same
    G = {}
    dh, dW, db = head_bwd(c["head_in"], P["head"][0], dphi)
    G["head"] = (dW, db)
    dh = r(relu_bwd(c["head_in"], dh))
    dskips = {}
    for up, a, bn, lvl in (("up0", "dec0a", "dec0b", 0), ("up1", "dec1a", "dec1b", 1),
                           ("up2", "dec2a", "dec2b", 2)):
        g = dh if lvl == 0 else relu_bwd(c[bn], dh)
        dh, dW, db = conv3_bwd(c[a], P[bn][0], g)
        G[bn] = (dW, db)
        g = relu_bwd(c[a], r(dh))
        dh, dW, db = conv3_bwd(c[a + "_in"], P[a][0], g)
        G[a] = (dW, db)
        dh = r(dh)
        cu = P[up][0].shape[3]
        dskips[lvl] = dh[..., cu:]
        dh, dW, db = tconv2_bwd(c[up + "_in"], P[up][0], dh[..., :cu])
        G[up] = (dW, db)
        dh = r(dh)
    g = relu_bwd(c["mid_b"], dh)
    dh, dW, db = conv3_bwd(c["mid_a"], P["mid_b"][0], g)
    G["mid_b"] = (dW, db)
    g = relu_bwd(c["mid_a"], r(dh))
    dh, dW, db = conv3_bwd(c["mid_a_in"], P["mid_a"][0], g)
    G["mid_a"] = (dW, db)
    dh = r(dh)
    for lvl, (a, bn) in reversed(list(enumerate((("enc0a", "enc0b"), ("enc1a", "enc1b"), ("enc2a", "enc2b"))))):
        g = r(relu_bwd(c[bn], pool2_bwd(dh) + dskips[lvl]))
        dh, dW, db = conv3_bwd(c[a], P[bn][0], g)
        G[bn] = (dW, db)
        g = relu_bwd(c[a], r(dh))
        dh, dW, db = conv3_bwd(c[a + "_in"], P[a][0], g)
        G[a] = (dW, db)
        dh = r(dh)
    return G


def loss(phi, phi_star, h: float):
    """(L, dL/dphi) of the mean squared gradient error over a batch (B, ny, nx)."""
    B, ny, nx = phi.shape
    N = B * ny * nx
    L = 0.0
    dphi = np.zeros_like(phi, dtype=np.float64)
    for k in range(B):
        gx, gy = grid.grad(phi[k], h)
        sx, sy = grid.grad(phi_star[k], h)
        ex, ey = gx - sx, gy - sy
        L += float(np.sum(ex * ex + ey * ey))
        # d/dphi sum |grad phi - s|^2 = 2 grad^T e = -2 div e  (div = -grad^T)
        dphi[k] = -2.0 * grid.div(ex, ey, h) / N
    return L / N, dphi


def adam(w, g, m, v, t: int, lr: float, b1: float = 0.9, b2: float = 0.999, eps: float = 1e-8):
    """One Adam step (bias-corrected moments); returns (w, m, v)."""
    m = b1 * m + (1.0 - b1) * g
    v = b2 * v + (1.0 - b2) * g * g
    mh = m / (1.0 - b1 ** t)
    vh = v / (1.0 - b2 ** t)
    return w - lr * mh / (np.sqrt(vh) + eps), m, v


# ---------------------------------------------------------------- resolution change (4096^2 use)
def downsample(rho, f: int):
    """Mass-preserving f x f block average (unit-mass densities stay unit-mass)."""
    ny, nx = rho.shape
    return np.asarray(rho, np.float64).reshape(ny // f, f, nx // f, f).mean(axis=(1, 3))


def upsample_bilinear(phi, f: int):
    """Bilinear interpolation between cell centres of a coarse grid onto the f-times finer
    cell-centred grid, constant extension beyond the outermost centres.  Every fine
    difference quotient is a convex combination of coarse ones along the same axis, so
    a bound on the coarse ones carries over."""
    ny, nx = phi.shape
    out = np.zeros((ny * f, nx * f))
    for I in range(ny * f):
        yc = (I + 0.5) / f - 0.5
        y0 = int(np.floor(yc))
        wy = yc - y0
        ya, yb = min(max(y0, 0), ny - 1), min(max(y0 + 1, 0), ny - 1)
        for J in range(nx * f):
            xc = (J + 0.5) / f - 0.5
            x0 = int(np.floor(xc))
            wx = xc - x0
            xa, xb = min(max(x0, 0), nx - 1), min(max(x0 + 1, 0), nx - 1)
            out[I, J] = ((1 - wy) * ((1 - wx) * phi[ya, xa] + wx * phi[ya, xb])
                         + wy * ((1 - wx) * phi[yb, xa] + wx * phi[yb, xb]))
    return out
