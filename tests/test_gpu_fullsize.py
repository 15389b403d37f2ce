"""Full-size parity: the 4096x4096 ROF and EMD workloads that bench.py times,
run through the solver loops (the fused three-launch iteration in the launch
shapes the tuner picks on first use, i.e. the configuration bench.py times) for
two iterations and compared field by field with two iterations of the FP64
oracle from the same zero start, together with the loop's own gap values."""
import numpy as np
import pytest

import synth
from conftest import announce
from oracle import emd as oemd
from oracle import grid
from oracle import rof as orof

pytestmark = pytest.mark.gpu
N = 4096
ITERS = 2


def dev(a):
    import torch
    return torch.tensor(np.ascontiguousarray(a, dtype=np.float32), device="cuda")


def host(t):
    return t.cpu().double().numpy()


def rel(a, b):
    nb = np.linalg.norm(b)
    return float(np.linalg.norm(a - b) / (nb if nb > 0 else 1.0))


def test_rof_solver_loop_4096_matches_oracle(gpctx):
    """The headline workload: 50-shape noisy scene, lambda 8, h 1, tau 0.01."""
    from paper_1805_09453_amd import Options
    I = synth.rof_scene(N, synth.config_seed(2), n_shapes=50, size_range=(0.02, 0.15))
    I32 = np.asarray(I, np.float32).astype(np.float64)
    announce(f"rof_solve {N}x{N}, {ITERS} iterations, tuned launch shapes")
    u, p, rep = gpctx.rof_solve(dev(I32), 1.0, 8.0, Options(tau=0.01, tol=0.0, max_iter=ITERS, check_every=ITERS))
    print("launch shape (row groups, column groups, tile width):", gpctx.get_shape(False, N))
    ref = orof.solve(I32, 1.0, 8.0, 0.01, tol=0.0, max_iter=ITERS, check_every=ITERS)
    errs = [rel(host(u), ref.u), rel(host(p)[0], ref.px), rel(host(p)[1], ref.py)]
    print("rel err u, px, py:", ["%.2e" % e for e in errs], "P", rep["primal"], ref.primal, "D", rep["dual"], ref.dual)
    assert rep["iters"] == ITERS
    assert max(errs) <= 1e-5
    assert abs(rep["primal"] - ref.primal) <= 1e-6 * abs(ref.primal)
    assert abs(rep["dual"] - ref.dual) <= 1e-6 * abs(ref.primal)


def test_emd_solver_loop_4096_matches_oracle(gpctx):
    """16-Gaussian mixtures, h = 1/4096, tau 0.3: flux, certificate potential and
    the gap values after two iterations."""
    from paper_1805_09453_amd import Options
    rho0, rho1 = synth.emd_mixture_pair(N, synth.config_seed(2), k=16)
    r0, r1 = (np.asarray(a, np.float32).astype(np.float64) for a in (rho0, rho1))
    h = 1.0 / N
    announce(f"emd_solve {N}x{N}, {ITERS} iterations, tuned launch shapes")
    m, phi, rep = gpctx.emd_solve(dev(r0), dev(r1), h, Options(tau=0.3, tol=0.0, max_iter=ITERS,
                                                               check_every=ITERS))
    print("launch shape (row groups, column groups, tile width):", gpctx.get_shape(True, N))
    ref = oemd.solve(r0, r1, h, tau=0.3, tol=0.0, max_iter=ITERS, check_every=ITERS)
    D, L, phit = oemd.certificate(ref.px, ref.py, ref.f, h)
    gpx, gpy = grid.grad(ref.psi, h)
    mg = host(m)
    errs = {"mx": rel(mg[0], ref.m[0]), "my": rel(mg[1], ref.m[1]),
            "ux": rel(mg[0] - gpx, ref.ux), "uy": rel(mg[1] - gpy, ref.uy), "phi": rel(host(phi), phit)}
    print("rel err:", {k: "%.2e" % v for k, v in errs.items()}, "P", rep["primal"], ref.primal, "D", rep["dual"], D)
    assert rep["iters"] == ITERS
    assert max(errs["mx"], errs["my"], errs["phi"]) <= 1e-5
    # u alone is the small part of the flux after two steps; FP32 storage of grad psi bounds it
    assert max(errs["ux"], errs["uy"]) <= 5e-5
    assert abs(rep["primal"] - ref.primal) <= 1e-6 * ref.primal
    assert abs(rep["dual"] - D) <= 2e-6 * ref.primal
