"""Scene and density generators (inputs only; no solver arithmetic).

Workload recipes follow the paper's experiments (section 4: a disc image for
ROF, translated uniform discs and Dirac pairs for EMD) and their synthetic
generalisations: noisy piecewise-constant scenes for ROF and Gaussian-mixture
densities for EMD.
"""
from __future__ import annotations

import numpy as np

SEED_STRIDE = 1_000_003
DENSITY_FLOOR = 1e-3


def config_seed(config: int, instance: int = 0) -> int:
    """Seed for instance ``instance`` of workload configuration ``config``."""
    return SEED_STRIDE * int(config) + int(instance)


def cell_centres(ny: int, nx: int):
    """(X, Y) arrays of cell-centre coordinates on [0,1]^2, shape [ny][nx]."""
    x = (np.arange(nx, dtype=np.float64) + 0.5) / nx
    y = (np.arange(ny, dtype=np.float64) + 0.5) / ny
    return np.meshgrid(x, y, indexing="xy")


def shapes_image(n: int, rng: np.random.Generator, n_shapes: int,
                 size_range=(0.05, 0.25)) -> np.ndarray:
    """Piecewise-constant scene: background 0, ``n_shapes`` discs or rectangles
    (probability 1/2 each) with intensity U[0,1], centre U[0.1,0.9]^2 and
    radius / half-sides U[size_range], painted in order at cell centres."""
    X, Y = cell_centres(n, n)
    img = np.zeros((n, n), dtype=np.float64)
    for _ in range(n_shapes):
        is_disc = rng.random() < 0.5
        val = rng.random()
        cx, cy = rng.uniform(0.1, 0.9, size=2)
        if is_disc:
            r = rng.uniform(*size_range)
            mask = (X - cx) ** 2 + (Y - cy) ** 2 <= r * r
        else:
            ax, ay = rng.uniform(*size_range, size=2)
            mask = (np.abs(X - cx) <= ax) & (np.abs(Y - cy) <= ay)
        img[mask] = val
    return img


def rof_scene(n: int, seed: int, n_shapes=None, size_range=(0.05, 0.25),
              noise_sigma: float = 0.1) -> np.ndarray:
    """Noisy piecewise-constant ROF input.  ``n_shapes`` None draws U{3..6}
    (the 64x64 workload); an int fixes it (50 for the 4096x4096 workload).
    I.i.d. N(0, noise_sigma^2) noise is added, unclipped."""
    rng = np.random.default_rng(seed)
    k = int(rng.integers(3, 7)) if n_shapes is None else int(n_shapes)
    img = shapes_image(n, rng, k, size_range)
    return img + noise_sigma * rng.standard_normal((n, n))


def disc_image(n: int, radius: float = 0.25, centre=(0.5, 0.5)) -> np.ndarray:
    """Indicator of a disc sampled at cell centres (the paper's ROF test image:
    radius 1/4 centred at (1/2, 1/2), section 4.1)."""
    X, Y = cell_centres(n, n)
    return ((X - centre[0]) ** 2 + (Y - centre[1]) ** 2 <= radius ** 2).astype(np.float64)


def _normalise_density(g: np.ndarray, floor: float) -> np.ndarray:
    """Unit mass on [0,1]^2 (cell area 1/(ny*nx)) plus an additive floor,
    renormalised: rho = (g/Z + floor) / (1 + floor)."""
    ny, nx = g.shape
    z = g.sum() / (ny * nx)
    return (g / z + floor) / (1.0 + floor)


def _gaussians(n: int, centres, widths, weights) -> np.ndarray:
    X, Y = cell_centres(n, n)
    g = np.zeros((n, n), dtype=np.float64)
    for (cx, cy), s, w in zip(centres, widths, weights):
        g += w * np.exp(-((X - cx) ** 2 + (Y - cy) ** 2) / (2.0 * s * s))
    return g


def gaussian_mixture_density(n: int, rng: np.random.Generator, k: int,
                             floor: float = DENSITY_FLOOR) -> np.ndarray:
    """Mixture of ``k`` isotropic Gaussians, centres U[0.1,0.9]^2, widths
    U[0.03,0.1], weights U[0.5,1.5], unit mass with an additive floor."""
    centres = rng.uniform(0.1, 0.9, size=(k, 2))
    widths = rng.uniform(0.03, 0.1, size=k)
    weights = rng.uniform(0.5, 1.5, size=k)
    return _normalise_density(_gaussians(n, centres, widths, weights), floor)


def emd_mixture_pair(n: int, seed: int, k: int = 4, floor: float = DENSITY_FLOOR):
    """(rho0, rho1): two k-Gaussian mixtures drawn in sequence from one stream."""
    rng = np.random.default_rng(seed)
    rho0 = gaussian_mixture_density(n, rng, k, floor)
    rho1 = gaussian_mixture_density(n, rng, k, floor)
    return rho0, rho1


def translated_gaussian_pair(n: int, shift_px=None, width: float = 0.05,
                             centre=(0.35, 0.5), axis: str = "x",
                             floor: float = DENSITY_FLOOR):
    """One Gaussian and its translate by ``shift_px`` cells (default n/8),
    each re-evaluated analytically at cell centres.  Returns
    (rho0, rho1, shift_length) with the shift in [0,1]^2 units.  ``axis`` is
    "x", "y" or "xy" (diagonal, both components shifted)."""
    s = n // 8 if shift_px is None else int(shift_px)
    d = s / n
    dx = d if axis in ("x", "xy") else 0.0
    dy = d if axis in ("y", "xy") else 0.0
    c0 = [centre]
    c1 = [(centre[0] + dx, centre[1] + dy)]
    rho0 = _normalise_density(_gaussians(n, c0, [width], [1.0]), floor)
    rho1 = _normalise_density(_gaussians(n, c1, [width], [1.0]), floor)
    return rho0, rho1, float(np.hypot(dx, dy))


def uniform_disc_pair(n: int, radius: float = 0.25,
                      c0=(0.375, 0.375), c1=(0.625, 0.625)):
    """The paper's EMD disc experiment (section 4.2): uniform densities on discs
    of radius 1/4 centred at (3/8,3/8) and (5/8,5/8), each of unit mass."""
    X, Y = cell_centres(n, n)
    out = []
    for c in (c0, c1):
        g = ((X - c[0]) ** 2 + (Y - c[1]) ** 2 <= radius ** 2).astype(np.float64)
        out.append(g / (g.sum() / (n * n)))
    return out[0], out[1]


def delta_pair(n: int, p0=(0.375, 0.375), p1=(0.625, 0.625)):
    """The paper's Dirac experiment (section 4.2): unit mass in the single cell
    containing each point."""
    out = []
    for p in (p0, p1):
        g = np.zeros((n, n), dtype=np.float64)
        j = min(int(p[0] * n), n - 1)
        i = min(int(p[1] * n), n - 1)
        g[i, j] = float(n * n)
        out.append(g)
    return out[0], out[1]


def integer_mass_pair(n: int, seed: int, max_count: int = 4):
    """Small integer-mass densities (counts per cell scaled by n^2/total) for
    exact network-flow and linear-programming checks.  Returns
    (rho0, rho1, counts0, counts1) with equal total counts."""
    rng = np.random.default_rng(seed)
    c0 = rng.integers(0, max_count + 1, size=(n, n))
    c1 = rng.integers(0, max_count + 1, size=(n, n))
    # equalise totals by adding the deficit to random cells of the lighter one
    d = int(c0.sum() - c1.sum())
    tgt = c1 if d > 0 else c0
    for _ in range(abs(d)):
        i, j = rng.integers(0, n, size=2)
        tgt[i, j] += 1
    total = float(c0.sum())
    scale = n * n / total
    return c0 * scale, c1 * scale, c0, c1


def smooth_size(m: float, primes=(2, 3, 5, 7), lo: int = 64, hi: int = 1024) -> int:
    """Nearest integer in [lo, hi] whose prime factors all lie in ``primes``
    (ties go to the smaller)."""
    best, best_d = None, None
    for v in range(lo, hi + 1):
        r = v
        for p in primes:
            while r % p == 0:
                r //= p
        if r != 1:
            continue
        dv = abs(v - m)
        if best is None or dv < best_d:
            best, best_d = v, dv
    return best


def batch_instances(count: int = 512, seed: int = config_seed(3), lo_exp: float = 6.0,
                    hi_exp: float = 10.0, primes=(2,)):
    """Mixed ROF/EMD batch: kind ~ Bernoulli(1/2); side n = 2^U[lo_exp, hi_exp]
    snapped to the nearest size whose factors lie in ``primes``.  Shape counts
    scale with area (3..50).  Each instance gets its own seed.  Returns a list
    of dicts with keys kind ("rof"/"emd"), n, seed, n_raw."""
    rng = np.random.default_rng(seed)
    out = []
    for i in range(count):
        kind = "rof" if rng.random() < 0.5 else "emd"
        n_raw = 2.0 ** rng.uniform(lo_exp, hi_exp)
        n = smooth_size(n_raw, primes=primes, lo=int(2 ** lo_exp), hi=int(2 ** hi_exp))
        out.append({"kind": kind, "n": int(n), "n_raw": float(n_raw),
                    "seed": seed * 7919 + i})
    return out


def batch_instance_inputs(inst: dict):
    """Inputs for one batch instance: ROF image or EMD density pair."""
    n = inst["n"]
    if inst["kind"] == "rof":
        k = int(np.clip(round(3 + 47 * (n * n - 64 * 64) / (1024 * 1024 - 64 * 64)), 3, 50))
        return {"image": rof_scene(n, inst["seed"], n_shapes=k)}
    rho0, rho1 = emd_mixture_pair(n, inst["seed"], k=4)
    return {"rho0": rho0, "rho1": rho1}
