"""Ergodic averages on the GPU (the averaged iterates u^N, p^N that the
convergence rates of section 2 are stated for): rof_solve and emd_solve with
the ergodic option against the FP64 oracle's ergodic solve from the same zero
start, field by field and in the gap values of the averages, for a count of
iterations that is not a multiple of the check interval (the average then
spans a final partial interval)."""
import numpy as np
import pytest

import synth
from conftest import announce, field_err
from oracle import emd as oemd
from oracle import rof as orof

pytestmark = pytest.mark.gpu


def f32(a):
    return np.asarray(a, dtype=np.float32).astype(np.float64)


def dev(a):
    import torch
    return torch.tensor(np.ascontiguousarray(a, dtype=np.float32), device="cuda")


def host(t):
    return t.cpu().double().numpy()


def rel(a, b):
    """relative L2 and elementwise (relative to max|b|) error, the larger"""
    return field_err(a, b)


@pytest.mark.parametrize("n,lam,tau,iters", [(256, 8.0, 0.02, 37), (512, 20.0, 0.05, 25)])
def test_rof_ergodic_solve_matches_oracle(gpctx, n, lam, tau, iters):
    from paper_1805_09453_amd import Options
    I = f32(synth.rof_scene(n, synth.config_seed(1)))
    announce(f"rof_solve ergodic {n}x{n}, {iters} iterations")
    u, p, rep = gpctx.rof_solve(dev(I), 1.0, lam, Options(tau=tau, tol=0.0, max_iter=iters, check_every=10,
                                                          ergodic=True))
    ref = orof.solve(I, 1.0, lam, tau, tol=0.0, max_iter=iters, check_every=10, ergodic=True)
    last = orof.solve(I, 1.0, lam, tau, tol=0.0, max_iter=iters, check_every=iters)
    errs = [rel(host(u), ref.u), rel(host(p)[0], ref.px), rel(host(p)[1], ref.py)]
    print("rel err u, px, py:", ["%.2e" % e for e in errs], "P", rep["primal"], ref.primal, "D", rep["dual"], ref.dual)
    assert rep["iters"] == iters
    assert max(errs) <= 1e-5
    assert abs(rep["primal"] - ref.primal) <= 1e-6 * abs(ref.primal)
    assert abs(rep["dual"] - ref.dual) <= 1e-6 * abs(ref.primal)
    # the average is not the last iterate (a wrong option routing would return that)
    assert rel(last.u, ref.u) > 1e3 * max(errs[0], 1e-9)


def test_rof_ergodic_solve_converges_and_certifies(gpctx):
    """With a tolerance the ergodic solve stops on the averaged gap, and the
    reported P and D are those of the returned averages (FP64 recomputation)."""
    from paper_1805_09453_amd import Options
    n, lam = 128, 8.0
    I = f32(synth.rof_scene(n, synth.config_seed(0)))
    announce("rof_solve ergodic to tol 1e-3")
    u, p, rep = gpctx.rof_solve(dev(I), 1.0, lam, Options(tau=0.05, tol=1e-3, max_iter=20000, check_every=10,
                                                          ergodic=True))
    print(rep)
    assert rep["converged"] and rep["rel_gap"] <= 1e-3 and rep["iters"] % 10 == 0
    P = orof.primal(host(u), I, 1.0, lam)
    D = orof.dual(host(p)[0], host(p)[1], I, 1.0, lam)
    assert abs(rep["primal"] - P) <= 1e-6 * P and abs(rep["dual"] - D) <= 1e-6 * P


@pytest.mark.parametrize("n,tau,iters", [(128, 0.3, 23), (256, 1.0, 16)])
def test_emd_ergodic_solve_matches_oracle(gpctx, n, tau, iters):
    from paper_1805_09453_amd import Options
    rho0, rho1 = synth.emd_mixture_pair(n, synth.config_seed(1), k=4)
    r0, r1 = f32(rho0), f32(rho1)
    h = 1.0 / n
    announce(f"emd_solve ergodic {n}x{n}, {iters} iterations")
    m, phi, rep = gpctx.emd_solve(dev(r0), dev(r1), h, Options(tau=tau, tol=0.0, max_iter=iters, check_every=7,
                                                               ergodic=True))
    ref = oemd.solve(r0, r1, h, tau=tau, tol=0.0, max_iter=iters, check_every=7, ergodic=True)
    D, L, phit = oemd.certificate(ref.px, ref.py, ref.f, h)
    mg = host(m)
    errs = {"mx": rel(mg[0], ref.m[0]), "my": rel(mg[1], ref.m[1]), "phi": rel(host(phi), phit)}
    print("rel err:", {k: "%.2e" % v for k, v in errs.items()}, "P", rep["primal"], ref.primal, "D", rep["dual"], D)
    assert rep["iters"] == iters
    assert max(errs.values()) <= 1e-5
    assert abs(rep["primal"] - ref.primal) <= 1e-6 * ref.primal
    assert abs(rep["dual"] - D) <= 2e-6 * ref.primal
    last = oemd.solve(r0, r1, h, tau=tau, tol=0.0, max_iter=iters, check_every=iters)
    assert rel(last.m[0], ref.m[0]) > 1e2 * max(errs["mx"], 1e-9)


def test_batch_rejects_ergodic(gpctx):
    from paper_1805_09453_amd import GPError, Options
    from paper_1805_09453_amd._lib import GP_EUNSUPPORTED, GP_KIND_ROF
    prob = {"kind": GP_KIND_ROF, "I": dev(synth.rof_scene(64, 1)), "h": 1.0, "lam": 8.0, "tau": 0.01}
    announce("gp_batch_solve ergodic rejected")
    with pytest.raises(GPError) as e:
        gpctx.batch_solve([prob], Options(tau=0.01, ergodic=True))
    assert e.value.code == GP_EUNSUPPORTED
