"""3-D scene and density generators (inputs only; no solver arithmetic).

The d = 3 counterparts of the 2-D recipes: noisy piecewise-constant volumes
(balls and boxes) for ROF and Gaussian-mixture densities for EMD, sampled at
the cell centres of [0,1]^3 with arrays [nz][ny][nx] (x fastest).
"""
from __future__ import annotations

import numpy as np

from .scenes import DENSITY_FLOOR


def cell_centres3(nz: int, ny: int, nx: int):
    """(X, Y, Z) cell-centre coordinates on [0,1]^3, shape [nz][ny][nx]."""
    z = (np.arange(nz, dtype=np.float64) + 0.5) / nz
    y = (np.arange(ny, dtype=np.float64) + 0.5) / ny
    x = (np.arange(nx, dtype=np.float64) + 0.5) / nx
    Z, Y, X = np.meshgrid(z, y, x, indexing="ij")
    return X, Y, Z


def rof_volume(shape, seed: int, n_shapes: int = 12, size_range=(0.05, 0.25),
               noise_sigma: float = 0.1) -> np.ndarray:
    """Background 0, ``n_shapes`` balls or boxes (probability 1/2 each) with
    intensity U[0,1], centre U[0.1,0.9]^3, radius / half-sides U[size_range],
    painted in order; plus i.i.d. N(0, noise_sigma^2) noise, unclipped."""
    nz, ny, nx = shape
    rng = np.random.default_rng(seed)
    X, Y, Z = cell_centres3(nz, ny, nx)
    vol = np.zeros((nz, ny, nx), dtype=np.float64)
    for _ in range(n_shapes):
        is_ball = rng.random() < 0.5
        val = rng.random()
        c = rng.uniform(0.1, 0.9, size=3)
        if is_ball:
            r = rng.uniform(*size_range)
            mask = (X - c[0]) ** 2 + (Y - c[1]) ** 2 + (Z - c[2]) ** 2 <= r * r
        else:
            a = rng.uniform(*size_range, size=3)
            mask = (np.abs(X - c[0]) <= a[0]) & (np.abs(Y - c[1]) <= a[1]) & (np.abs(Z - c[2]) <= a[2])
        vol[mask] = val
    return vol + noise_sigma * rng.standard_normal((nz, ny, nx))


def _mixture3(shape, rng, k, floor):
    nz, ny, nx = shape
    X, Y, Z = cell_centres3(nz, ny, nx)
    centres = rng.uniform(0.1, 0.9, size=(k, 3))
    widths = rng.uniform(0.05, 0.12, size=k)
    weights = rng.uniform(0.5, 1.5, size=k)
    g = np.zeros(shape, dtype=np.float64)
    for c, s, w in zip(centres, widths, weights):
        g += w * np.exp(-((X - c[0]) ** 2 + (Y - c[1]) ** 2 + (Z - c[2]) ** 2) / (2.0 * s * s))
    zmass = g.sum() / g.size
    return (g / zmass + floor) / (1.0 + floor)


def emd_volume_pair(shape, seed: int, k: int = 4, floor: float = DENSITY_FLOOR):
    """(rho0, rho1): two k-Gaussian mixtures on [0,1]^3 (centres U[0.1,0.9]^3,
    widths U[0.05,0.12], weights U[0.5,1.5]), unit mass plus an additive floor,
    drawn in sequence from one stream."""
    rng = np.random.default_rng(seed)
    return _mixture3(shape, rng, k, floor), _mixture3(shape, rng, k, floor)
