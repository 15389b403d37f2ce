"""GPU parity of one G-prox iteration (pd_step), of the duality-gap evaluation
(pd_gap), of the EMD set-up, and of full solves, against the FP64 oracle."""
import json
import os

import numpy as np
import pytest

import synth
from conftest import announce, field_err
from oracle import emd as oemd
from oracle import grid
from oracle import rof as orof

pytestmark = pytest.mark.gpu
GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


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


# ---------------------------------------------------------------- ROF
ROF_STEP_CASES = [(64, 64, 1.0, 8.0, 0.01), (128, 256, 1.0 / 256, 20.0, 2.0), (512, 512, 1.0, 8.0, 0.05),
                  (4096, 4096, 1.0, 8.0, 0.01)]


@pytest.mark.parametrize("ny,nx,h,lam,tau", ROF_STEP_CASES)
def test_rof_pd_step_matches_oracle_step(gpctx, ny, nx, h, lam, tau):
    from paper_1805_09453_amd._lib import GP_KIND_ROF
    n = min(ny, nx)
    I = f32(synth.rof_scene(n, 11))
    I = f32(np.tile(I, (ny // n, nx // n)))
    u = np.zeros_like(I)
    px, py = np.zeros_like(I), np.zeros_like(I)
    pbx, pby = px.copy(), py.copy()
    sig = 1.0 / tau
    for _ in range(3 if ny < 4096 else 1):  # a non-trivial starting state
        u, px, py, pbx, pby = orof.step(u, px, py, pbx, pby, I, h, lam, tau, sig)
    u, px, py, pbx, pby = (f32(a) for a in (u, px, py, pbx, pby))
    ref = orof.step(u, px, py, pbx, pby, I, h, lam, tau, sig)
    announce(f"rof pd_step {ny}x{nx} h={h} lam={lam} tau={tau}")
    st = gpctx.make_state(GP_KIND_ROF, dev(I), h, tau, lam=lam, u=dev(u), p=dev(np.stack([px, py])),
                          pbar=dev(np.stack([pbx, pby])))
    gpctx.pd_step(st, 1)
    got = (host(st.u), host(st.p)[0], host(st.p)[1], host(st.pbar)[0], host(st.pbar)[1])
    errs = [rel(g, r) for g, r in zip(got, ref)]
    print("per-field rel err (u, px, py, pbx, pby):", ["%.2e" % e for e in errs])
    assert max(errs) <= 1e-5
    assert st.iter == 1


def test_rof_gap_matches_oracle_values(gpctx):
    from paper_1805_09453_amd._lib import GP_KIND_ROF
    I = f32(synth.rof_scene(256, 5))
    r = orof.solve(I, 1.0, 8.0, 0.01, tol=0.0, max_iter=40, check_every=40)
    u, px, py = f32(r.u), f32(r.px), f32(r.py)
    announce("rof pd_gap 256x256")
    st = gpctx.make_state(GP_KIND_ROF, dev(I), 1.0, 0.01, lam=8.0, u=dev(u), p=dev(np.stack([px, py])))
    g = gpctx.pd_gap(st)
    P, D = orof.primal(u, I, 1.0, 8.0), orof.dual(px, py, I, 1.0, 8.0)
    assert abs(g["primal"] - P) / abs(P) < 1e-6 and abs(g["dual"] - D) / abs(P) < 1e-6


def test_rof_solve_objective_parity_64px_scene(gpctx):
    """64x64 scene (3-6 shapes, sigma 0.1 noise, lambda 8, h 1): the GPU solve's
    objective, evaluated in FP64 on the downloaded u, is within 1e-5 of F*."""
    from paper_1805_09453_amd import Options
    I = synth.rof_scene(64, synth.config_seed(0))
    with open(os.path.join(GOLDEN, "oracle_references.json")) as fh:
        Fstar = json.load(fh)["rof_c0"]["primal"]
    announce("rof_solve 64x64 config-0 scene")
    u, p, rep = gpctx.rof_solve(dev(I), 1.0, 8.0, Options(tau=0.01, tol=1e-6, max_iter=20000, check_every=10))
    Fg = orof.primal(host(u), I, 1.0, 8.0)
    err = abs(Fg - Fstar) / Fstar
    print(f"iters {rep['iters']} gpu gap {rep['rel_gap']:.2e} objective error {err:.2e}")
    assert rep["converged"]
    assert err <= 1e-5
    # the reported gap is a certificate: recompute P and D in FP64 from the outputs
    P = orof.primal(host(u), I, 1.0, 8.0)
    D = orof.dual(host(p)[0], host(p)[1], I, 1.0, 8.0)
    assert abs(rep["primal"] - P) / P < 1e-6 and abs(rep["dual"] - D) / P < 1e-6
    assert D <= Fstar * (1 + 1e-9)


def test_rof_solve_disc_closed_form(gpctx):
    """Disc indicator, lambda = 20, h = 1/n (paper's ROF experiment, corrected closed form)."""
    from paper_1805_09453_amd import Options
    n, lam, rad = 256, 20.0, 0.25
    I = synth.disc_image(n, rad)
    announce("rof_solve disc 256x256")
    u, p, rep = gpctx.rof_solve(dev(I), 1.0 / n, lam, Options(tau=2.0, tol=1e-5, max_iter=20000, check_every=20))
    uu = host(u)
    X, Y = synth.cell_centres(n, n)
    d = np.hypot(X - 0.5, Y - 0.5)
    a = 1 - 2 / (lam * rad)
    b = 2 * np.pi * rad / (lam * (1 - np.pi * rad * rad))
    assert rep["converged"]
    assert abs(uu[d < rad - 0.1].mean() - a) < 0.01 and abs(uu[d > rad + 0.1].mean() - b) < 0.005
    assert abs(uu.mean() - I.mean()) < 1e-5


# ---------------------------------------------------------------- EMD
def test_emd_setup_matches_oracle(gpctx):
    n = 256
    rho0, rho1 = synth.emd_mixture_pair(n, synth.config_seed(1), k=4)
    r0, r1 = f32(rho0), f32(rho1)
    f_ref, psi = oemd.setup(r0, r1, 1.0 / n)
    gx, gy = grid.grad(psi, 1.0 / n)
    announce("emd_setup 256x256")
    f, gpsi = gpctx.emd_setup(dev(r0), dev(r1), 1.0 / n)
    ef, egx, egy = rel(host(f), f_ref), rel(host(gpsi)[0], gx), rel(host(gpsi)[1], gy)
    print(f"setup rel err f {ef:.2e} gpsi {egx:.2e} {egy:.2e}")
    assert max(ef, egx, egy) <= 1e-6


@pytest.mark.parametrize("n,tau", [(64, 0.25), (256, 1.0), (1024, 0.3)])
def test_emd_pd_step_matches_oracle_step(gpctx, n, tau):
    from paper_1805_09453_amd._lib import GP_KIND_EMD
    h = 1.0 / n
    rho0, rho1 = synth.emd_mixture_pair(n, 3, k=4)
    r0, r1 = f32(rho0), f32(rho1)
    f_ref, psi = oemd.setup(r0, r1, h)
    gpx, gpy = (f32(a) for a in grid.grad(psi, h))
    ux, uy = np.zeros_like(f_ref), np.zeros_like(f_ref)
    px, py = np.zeros_like(f_ref), np.zeros_like(f_ref)
    pbx, pby = px.copy(), py.copy()
    for _ in range(4):
        ux, uy, px, py, pbx, pby = oemd.step(ux, uy, px, py, pbx, pby, gpx, gpy, h, tau, 1 / tau)
    # the projected-form update equals the literal one on a divergence-free u
    ux, uy = oemd.leray(f32(ux), f32(uy), h)
    px, py, pbx, pby = (f32(a) for a in (px, py, pbx, pby))
    ref = oemd.step(ux, uy, px, py, pbx, pby, gpx, gpy, h, tau, 1 / tau)
    announce(f"emd pd_step {n}x{n} tau={tau}")
    st = gpctx.make_state(GP_KIND_EMD, dev(f_ref), h, tau, gpsi=dev(np.stack([gpx, gpy])),
                          u=dev(np.stack([ux, uy])), p=dev(np.stack([px, py])), pbar=dev(np.stack([pbx, pby])))
    gpctx.pd_step(st, 1)
    got = (host(st.u)[0], host(st.u)[1], host(st.p)[0], host(st.p)[1], host(st.pbar)[0], host(st.pbar)[1])
    errs = [rel(g, r) for g, r in zip(got, ref)]
    print("per-field rel err (ux, uy, px, py, pbx, pby):", ["%.2e" % e for e in errs])
    assert max(errs) <= 1e-5


def test_emd_gap_matches_oracle_values(gpctx):
    from paper_1805_09453_amd._lib import GP_KIND_EMD
    n = 128
    h = 1.0 / n
    rho0, rho1, _ = synth.translated_gaussian_pair(n)
    r = oemd.solve(f32(rho0), f32(rho1), h, tau=0.25, tol=0.0, max_iter=50, check_every=50)
    gpx, gpy = (f32(a) for a in grid.grad(r.psi, h))
    ux, uy, px, py = (f32(a) for a in (r.ux, r.uy, r.px, r.py))
    announce("emd pd_gap 128x128")
    st = gpctx.make_state(GP_KIND_EMD, dev(r.f), h, 0.25, gpsi=dev(np.stack([gpx, gpy])),
                          u=dev(np.stack([ux, uy])), p=dev(np.stack([px, py])))
    g = gpctx.pd_gap(st)
    P = oemd.primal(ux, uy, gpx, gpy, h)
    D = oemd.certificate(px, py, f32(r.f), h)[0]
    print(g, P, D)
    assert abs(g["primal"] - P) / P < 1e-6 and abs(g["dual"] - D) / P < 2e-6


def test_emd_solve_translated_pair(gpctx):
    """Gaussian translated by n/8 cells in x: EMD = shift / (1 + floor) exactly on the grid."""
    from paper_1805_09453_amd import Options
    n = 256
    rho0, rho1, s = synth.translated_gaussian_pair(n)
    exact = s / (1 + synth.scenes.DENSITY_FLOOR)
    announce("emd_solve translated pair 256x256")
    m, phi, rep = gpctx.emd_solve(dev(rho0), dev(rho1), 1.0 / n,
                                  Options(tau=0.25, tol=1e-4, max_iter=50000, check_every=50))
    f_ref, _ = oemd.setup(f32(rho0), f32(rho1), 1.0 / n)
    val, resid = oemd.flux_value(host(m)[0], host(m)[1], f_ref, 1.0 / n)
    print(rep, val, exact, resid)
    assert rep["converged"]
    assert rep["dual"] <= exact * (1 + 1e-6) and exact <= rep["primal"] * (1 + 1e-6)
    assert abs(val - exact) / exact <= 1e-4


def test_emd_solve_mixture_objective_parity(gpctx):
    """256x256 4-Gaussian mixtures: FP64 value of the re-projected GPU flux vs the oracle's F*."""
    from paper_1805_09453_amd import Options
    n = 256
    rho0, rho1 = synth.emd_mixture_pair(n, synth.config_seed(1), k=4)
    with open(os.path.join(GOLDEN, "oracle_references.json")) as fh:
        ref = json.load(fh)["emd_c1_mixture"]
    announce("emd_solve mixture 256x256")
    m, phi, rep = gpctx.emd_solve(dev(rho0), dev(rho1), 1.0 / n,
                                  Options(tau=0.3, tol=1e-5, max_iter=100000, check_every=100))
    f_ref, _ = oemd.setup(f32(rho0), f32(rho1), 1.0 / n)
    val, resid = oemd.flux_value(host(m)[0], host(m)[1], f_ref, 1.0 / n)
    err = abs(val - ref["primal"]) / ref["primal"]
    print(f"iters {rep['iters']} gap {rep['rel_gap']:.2e} objective error {err:.2e} div residual {resid:.2e}")
    assert err <= 1e-5
