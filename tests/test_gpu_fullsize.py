"""Full-size parity: the 4096x4096 ROF and EMD workloads that bench.py times,
run through the solver loops (the fused three-launch iteration in the launch
shapes the tuner picks on first use, i.e. the configuration bench.py times) for
two iterations and compared field by field with two iterations of the FP64
oracle from the same zero start, together with the loop's own gap values."""
import numpy as np
import pytest

import synth
from conftest import announce, field_err
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
    """relative L2 and elementwise (relative to max|b|) error, the larger"""
    return field_err(a, b)


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


def golden(name, max_gap):
    """The tightest stored oracle bracket for `name` (the final entry, else a
    checkpoint name@gap) whose relative gap is <= max_gap."""
    import json
    import os
    with open(os.path.join(os.path.dirname(__file__), "golden", "oracle_references.json")) as fh:
        refs = json.load(fh)
    cands = [v for k, v in refs.items() if k == name or k.startswith(name + "@")]
    cands = [v for v in cands if v["rel_gap"] <= max_gap]
    assert cands, f"no oracle reference {name} with gap <= {max_gap}"
    return min(cands, key=lambda v: v["rel_gap"])


def test_rof_4096_full_solve_objective_parity(gpctx):
    """The solve the benchmark times (4096^2 scene, lambda 8, h 1, tau 0.01, to a
    1e-5 relative gap in the tuned launch shapes): its objective, evaluated in
    FP64 on the downloaded u, is within 1e-5 of the oracle's F* (a 4096^2 oracle
    solve certified to a gap <= 1e-6), and the GPU's certificate brackets it."""
    from paper_1805_09453_amd import Options
    ref = golden("rof_c2_4096", 1e-6)
    I = synth.rof_scene(N, synth.config_seed(2), n_shapes=50, size_range=(0.02, 0.15))
    I32 = np.asarray(I, np.float32).astype(np.float64)
    announce(f"rof_solve {N}x{N} to 1e-5, objective vs oracle F* (gap {ref['rel_gap']:.1e})")
    u, p, rep = gpctx.rof_solve(dev(I32), 1.0, 8.0, Options(tau=0.01, tol=1e-5, max_iter=5000, check_every=10))
    Fg = orof.primal(host(u), I32, 1.0, 8.0)
    Dg = orof.dual(host(p)[0], host(p)[1], I32, 1.0, 8.0)
    err = abs(Fg - ref["primal"]) / ref["primal"]
    print(f"iters {rep['iters']} gpu gap {rep['rel_gap']:.2e}; FP64 objective {Fg!r} vs F* {ref['primal']!r}: "
          f"{err:.2e}; FP64 dual {Dg!r}")
    assert rep["converged"]
    assert err <= 1e-5
    assert Fg >= ref["dual"] * (1 - 1e-12)       # u is feasible: no value below the oracle's lower bound
    assert Dg <= ref["primal"] * (1 + 1e-12)     # the GPU dual is a lower bound
    assert abs(rep["primal"] - Fg) <= 1e-6 * Fg and abs(rep["dual"] - Dg) <= 1e-6 * Fg


def test_emd_1024_full_solve_objective_parity(gpctx):
    """16-Gaussian mixtures at 1024^2 (the 4096^2 recipe), tau 0.3, to a 1e-5 gap:
    the FP64 value of the re-projected GPU flux lies within 1e-5 of the oracle's
    primal value, inside the oracle's bracket widened by the GPU's own gap, and
    the GPU certificate lies below the oracle's upper bound."""
    from paper_1805_09453_amd import Options
    ref = golden("emd_c2_1024", 3e-5)
    n = 1024
    h = 1.0 / n
    r0, r1 = (np.asarray(a, np.float32).astype(np.float64)
              for a in synth.emd_mixture_pair(n, synth.config_seed(2, 1), k=16))
    announce(f"emd_solve {n}x{n} to 1e-5, objective vs oracle bracket (gap {ref['rel_gap']:.1e})")
    m, phi, rep = gpctx.emd_solve(dev(r0), dev(r1), h, Options(tau=0.3, tol=1e-5, max_iter=100000, check_every=50))
    f_ref, _ = oemd.setup(r0, r1, h)
    val, resid = oemd.flux_value(host(m)[0], host(m)[1], f_ref, h)
    err = abs(val - ref["primal"]) / ref["primal"]
    print(f"iters {rep['iters']} gap {rep['rel_gap']:.2e}; FP64 value {val!r} vs oracle [{ref['dual']!r}, "
          f"{ref['primal']!r}]: {err:.2e}; div residual {resid:.2e}")
    assert rep["converged"]
    assert err <= max(1e-5, ref["rel_gap"])
    assert val >= ref["dual"] * (1 - 1e-6)
    assert rep["dual"] <= ref["primal"] * (1 + 1e-6)
