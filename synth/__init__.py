"""Seeded synthetic inputs for the G-prox PDHG solvers (ROF denoising and L1 EMD).

This package only *draws* inputs: images, densities and their parameters.  It
holds none of the method's arithmetic (no gradients, no Poisson solves, no
prox), so that both the FP64 oracle and the GPU path can take their inputs
from it without sharing any part of the computation.

All generators are FP64 NumPy, seeded with ``numpy.random.default_rng`` (PCG64).
Grids are cell-centred on [0,1]^2: cell (i, j) has centre ((j+1/2)/nx, (i+1/2)/ny),
row index i runs along y, column index j along x (row-major ``[ny][nx]``).
"""
from .scenes import (  # noqa: F401
    config_seed,
    cell_centres,
    shapes_image,
    rof_scene,
    disc_image,
    gaussian_mixture_density,
    emd_mixture_pair,
    translated_gaussian_pair,
    uniform_disc_pair,
    delta_pair,
    integer_mass_pair,
    batch_instances,
    batch_instance_inputs,
    smooth_size,
)
from .volumes import cell_centres3, emd_volume_pair, rof_volume  # noqa: F401
