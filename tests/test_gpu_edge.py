"""Edge cases on the GPU: the anisotropic (l1) grid norm against the oracle,
degenerate problems (identical densities, a constant image), a rectangular EMD
grid, and the error paths of the solver entry points."""
import numpy as np
import pytest

import synth
from conftest import announce, field_err
from oracle import emd as oemd
from oracle import grid
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


def emd_state(n_y, n_x, seed, tau, norm, steps=4):
    """A non-trivial EMD state after `steps` oracle iterations (u made divergence-free
    so that the projected and the literal update agree)."""
    # smooth densities (a window of a square mixture pair); rough ones saturate the
    # dual everywhere and leave u ~ 0, where a relative comparison means nothing
    h = 1.0 / max(n_y, n_x)
    rho0, rho1 = synth.emd_mixture_pair(max(n_y, n_x), seed, k=4)
    r0, r1 = f32(rho0[:n_y, :n_x]), f32(rho1[:n_y, :n_x])
    r1 *= r0.sum() / r1.sum()
    f_ref, psi = oemd.setup(r0, r1, h)
    gpx, gpy = (f32(a) for a in grid.grad(psi, h))
    z = np.zeros_like(f_ref)
    st = (z, z.copy(), z.copy(), z.copy(), z.copy(), z.copy())
    for _ in range(steps):
        st = oemd.step(*st, gpx, gpy, h, tau, 1 / tau, norm)
    ux, uy = oemd.leray(f32(st[0]), f32(st[1]), h)
    return h, f_ref, gpx, gpy, (ux, uy) + tuple(f32(a) for a in st[2:])


@pytest.mark.parametrize("ny,nx", [(256, 256), (128, 256)])
def test_rof_pd_step_anisotropic(gpctx, ny, nx):
    from paper_1805_09453_amd._lib import GP_KIND_ROF, GP_NORM_ANISO
    I = f32(np.tile(synth.rof_scene(128, 21), (ny // 128, nx // 128)))
    lam, tau, h = 8.0, 0.02, 1.0
    st = (np.zeros_like(I),) + tuple(np.zeros_like(I) for _ in range(4))
    for _ in range(3):
        st = orof.step(*st, I, h, lam, tau, 1 / tau, grid.ANISO)
    st = tuple(f32(a) for a in st)
    ref = orof.step(*st, I, h, lam, tau, 1 / tau, grid.ANISO)
    announce(f"rof pd_step anisotropic {ny}x{nx}")
    s = gpctx.make_state(GP_KIND_ROF, dev(I), h, tau, lam=lam, u=dev(st[0]), p=dev(np.stack(st[1:3])),
                         pbar=dev(np.stack(st[3:5])), norm=GP_NORM_ANISO)
    gpctx.pd_step(s, 1)
    got = (host(s.u), host(s.p)[0], host(s.p)[1], host(s.pbar)[0], host(s.pbar)[1])
    errs = [rel(g, r) for g, r in zip(got, ref)]
    print("rel err (u, px, py, pbx, pby):", ["%.2e" % e for e in errs])
    assert max(errs) <= 1e-5
    g = gpctx.pd_gap(s)
    P = orof.primal(got[0], I, h, lam, grid.ANISO)
    assert abs(g["primal"] - P) <= 1e-6 * abs(P)


@pytest.mark.parametrize("ny,nx", [(128, 128), (64, 128)])
def test_emd_pd_step_anisotropic_and_rectangular(gpctx, ny, nx):
    from paper_1805_09453_amd._lib import GP_KIND_EMD, GP_NORM_ANISO, GP_NORM_ISO
    for norm, gnorm in ((GP_NORM_ANISO, grid.ANISO), (GP_NORM_ISO, grid.ISO)):
        tau = 0.3
        h, f_ref, gpx, gpy, st = emd_state(ny, nx, 5, tau, gnorm)
        ref = oemd.step(*st, gpx, gpy, h, tau, 1 / tau, gnorm)
        announce(f"emd pd_step {ny}x{nx} norm={norm}")
        s = gpctx.make_state(GP_KIND_EMD, dev(f_ref), h, tau, gpsi=dev(np.stack([gpx, gpy])),
                             u=dev(np.stack(st[0:2])), p=dev(np.stack(st[2:4])), pbar=dev(np.stack(st[4:6])),
                             norm=norm)
        gpctx.pd_step(s, 1)
        got = (host(s.u)[0], host(s.u)[1], host(s.p)[0], host(s.p)[1], host(s.pbar)[0], host(s.pbar)[1])
        errs = [rel(g, r) for g, r in zip(got, ref)]
        print("rel err (ux, uy, px, py, pbx, pby):", ["%.2e" % e for e in errs])
        assert max(errs) <= 1e-5
        g = gpctx.pd_gap(s)
        P = oemd.primal(got[0], got[1], gpx, gpy, h, gnorm)
        D = oemd.certificate(got[2], got[3], f_ref, h, gnorm)[0]
        assert abs(g["primal"] - P) <= 1e-6 * P and abs(g["dual"] - D) <= 2e-6 * P


@pytest.mark.parametrize("ny,nx,norm", [(64, 128, 0), (128, 64, 1), (64, 1024, 0)])
def test_emd_solve_rectangular_matches_oracle(gpctx, ny, nx, norm):
    """emd_solve (the single-variable form at sigma tau = 1) on rectangular grids,
    both norms, rows of the radix-8 length class: 9 iterations against the
    two-variable FP64 oracle."""
    from paper_1805_09453_amd import Options
    h = 1.0 / max(ny, nx)
    rho0, rho1 = synth.emd_mixture_pair(max(ny, nx), 31, k=4)
    r0, r1 = f32(rho0[:ny, :nx]), f32(rho1[:ny, :nx])
    r1 *= r0.sum() / r1.sum()
    r1 = f32(r1)
    announce(f"emd_solve {ny}x{nx} norm={norm}, 9 iterations")
    m, phi, rep = gpctx.emd_solve(dev(r0), dev(r1), h, Options(tau=0.3, tol=0.0, max_iter=9, check_every=9, norm=norm))
    ref = oemd.solve(r0, r1, h, tau=0.3, tol=0.0, max_iter=9, check_every=9, norm=norm)
    D, L, phit = oemd.certificate(ref.px, ref.py, ref.f, h, norm)
    mg = host(m)
    errs = [rel(mg[0], ref.m[0]), rel(mg[1], ref.m[1]), rel(host(phi), phit)]
    print(["%.2e" % e for e in errs], rep["primal"], ref.primal, rep["dual"], D)
    assert max(errs) <= 1e-5
    assert abs(rep["primal"] - ref.primal) <= 1e-6 * ref.primal and abs(rep["dual"] - D) <= 2e-6 * ref.primal


def test_emd_solve_anisotropic_value(gpctx):
    """64x64 two-Gaussian pair in the l1 grid norm: the converged GPU solve's
    certificate brackets the oracle's converged value (tests/golden, written by
    make_oracle_references.py from the oracle alone)."""
    import json
    import os

    from paper_1805_09453_amd import Options
    from paper_1805_09453_amd._lib import GP_NORM_ANISO
    with open(os.path.join(os.path.dirname(__file__), "golden", "oracle_references.json")) as fh:
        ref = json.load(fh)["emd_aniso_64"]
    n = 64
    rho0, rho1 = synth.emd_mixture_pair(n, 17, k=2)
    announce("emd_solve anisotropic 64x64")
    m, _, rep = gpctx.emd_solve(dev(rho0), dev(rho1), 1.0 / n,
                                Options(tau=0.3, tol=1e-6, max_iter=400000, check_every=50, norm=GP_NORM_ANISO))
    print(rep, ref)
    assert rep["converged"]
    # both are certified: the GPU bracket [D, P] and the oracle's overlap, and the values agree to 2e-6
    assert rep["dual"] <= ref["primal"] * (1 + 1e-6) and ref["dual"] <= rep["primal"] * (1 + 1e-6)
    assert abs(rep["primal"] - ref["primal"]) <= 2e-6 * ref["primal"]


def test_emd_identical_densities_is_zero_at_the_first_check(gpctx):
    """rho0 = rho1: f = 0, psi = 0, the zero flux is optimal, P = D = 0 at the first check."""
    import torch
    from paper_1805_09453_amd import Options
    n = 128
    rho, _ = synth.emd_mixture_pair(n, 23, k=4)
    announce("emd_solve identical densities")
    m, phi, rep = gpctx.emd_solve(dev(rho), dev(rho), 1.0 / n, Options(tau=0.3, tol=1e-6, max_iter=1000,
                                                                      check_every=10))
    print(rep)
    assert rep["converged"] and rep["iters"] == 10
    assert rep["primal"] == 0.0 and rep["dual"] == 0.0
    assert torch.count_nonzero(m).item() == 0


def test_rof_constant_image(gpctx):
    """I = c: u* = c, p* = 0, F* = 0; the solve approaches c from the zero start."""
    from paper_1805_09453_amd import Options
    n, c = 128, 0.3
    I = np.full((n, n), c)
    announce("rof_solve constant image")
    u, p, rep = gpctx.rof_solve(dev(I), 1.0, 8.0, Options(tau=0.01, tol=1e-7, max_iter=20000, check_every=10))
    uu = host(u)
    print(rep, np.abs(uu - c).max())
    assert np.abs(uu - c).max() <= 1e-5
    assert rep["primal"] <= 1e-6 * 0.5 * 8.0 * c * c * n * n  # 1e-6 of the zero start's objective


def test_solver_errors(gpctx):
    from paper_1805_09453_amd import GPError, Options
    from paper_1805_09453_amd._lib import GP_EINVAL, GP_EMASS
    n = 64
    I = np.zeros((n, n))
    I[3, 5] = np.nan
    with pytest.raises(GPError) as e:
        gpctx.rof_solve(dev(I), 1.0, 8.0, Options(tau=0.01))
    assert e.value.code == GP_EINVAL and "non-finite" in str(e.value)
    ok = dev(np.ones((n, n)))
    for bad in (Options(tau=0.5, sigma=4.0), Options(tau=0.01, max_iter=0), Options(tau=0.01, check_every=0),
                Options(tau=-1.0), Options(tau=0.01, tol=-1.0)):
        with pytest.raises(GPError) as e:
            gpctx.rof_solve(ok, 1.0, 8.0, bad)
        assert e.value.code == GP_EINVAL
    with pytest.raises(GPError) as e:
        gpctx.rof_solve(ok, 1.0, -8.0, Options(tau=0.01))
    assert e.value.code == GP_EINVAL
    r0, r1 = synth.emd_mixture_pair(n, 3, k=2)
    with pytest.raises(GPError) as e:
        gpctx.emd_solve(dev(r0), dev(r1 * 1.01), 1.0 / n, Options(tau=0.3))
    assert e.value.code == GP_EMASS
