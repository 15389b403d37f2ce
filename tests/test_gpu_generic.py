"""Grid sides that are not powers of two (every prime factor 2, 3, 5 or 7): the
mixed-radix DCT path against the FP64 oracle (the oracle's DCT is scipy's, for
any length): the screened Poisson solve, one G-prox iteration of each problem,
solver loops and a full solve."""
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


def dev(a, dtype=None):
    import torch
    return torch.tensor(np.ascontiguousarray(a), dtype=dtype or torch.float32, device="cuda")


def host(t):
    return t.cpu().double().numpy()


def scene(ny, nx, seed):
    """A noisy piecewise-constant ny x nx image (the 64^2 recipe on the larger side, cropped)."""
    return f32(synth.rof_scene(max(ny, nx), seed)[:ny, :nx])


def mixture(ny, nx, seed, k=4):
    r0, r1 = synth.emd_mixture_pair(max(ny, nx), seed, k=k)
    r0, r1 = f32(r0[:ny, :nx]), f32(r1[:ny, :nx])
    return r0, f32(r1 * (r0.sum() / r1.sum()))


SIZES = [(96, 96), (320, 320), (448, 448), (720, 720), (96, 160), (75, 105), (64, 1000)]


@pytest.mark.parametrize("ny,nx", SIZES)
@pytest.mark.parametrize("alpha", [0.0, 0.3])
def test_dct_poisson_generic_sizes(gpctx, ny, nx, alpha):
    import torch
    b = f32(np.random.default_rng(ny * 7 + nx).standard_normal((ny, nx)))
    h = 1.0 / max(ny, nx) if alpha == 0.0 else 1.0
    announce(f"dct_poisson {ny}x{nx} alpha {alpha}")
    x = host(gpctx.dct_poisson(dev(b), h=h, alpha=alpha))
    ref = grid.poisson_solve(b, h, alpha)
    err = field_err(x, ref)
    x64 = gpctx.dct_poisson_f64(dev(b, torch.float64), h=h, alpha=alpha).cpu().numpy()
    err64 = field_err(x64, ref)
    print(f"FP32 {err:.2e}  FP64 {err64:.2e}")
    assert err <= (1e-6 if max(ny, nx) <= 256 else 5e-6)
    assert err64 <= 1e-12


@pytest.mark.parametrize("ny,nx", SIZES[:5])
def test_rof_pd_step_generic_sizes(gpctx, ny, nx):
    from paper_1805_09453_amd._lib import GP_KIND_ROF
    h, lam, tau = 1.0, 8.0, 0.02
    I = scene(ny, nx, 21)
    u = np.zeros_like(I)
    px, py = np.zeros_like(I), np.zeros_like(I)
    pbx, pby = px.copy(), py.copy()
    for _ in range(3):
        u, px, py, pbx, pby = orof.step(u, px, py, pbx, pby, I, h, lam, tau, 1 / tau)
    u, px, py, pbx, pby = (f32(a) for a in (u, px, py, pbx, pby))
    ref = orof.step(u, px, py, pbx, pby, I, h, lam, tau, 1 / tau)
    announce(f"rof pd_step {ny}x{nx}")
    st = gpctx.make_state(GP_KIND_ROF, dev(I), h, tau, lam=lam, u=dev(u), p=dev(np.stack([px, py])),
                          pbar=dev(np.stack([pbx, pby])))
    gpctx.pd_step(st, 1)
    got = (host(st.u), host(st.p)[0], host(st.p)[1], host(st.pbar)[0], host(st.pbar)[1])
    errs = [field_err(g, r) for g, r in zip(got, ref)]
    print(["%.2e" % e for e in errs])
    assert max(errs) <= 1e-5
    g = gpctx.pd_gap(st)
    P, D = orof.primal(ref[0], I, h, lam), orof.dual(ref[1], ref[2], I, h, lam)
    assert abs(g["primal"] - P) <= 1e-6 * abs(P) and abs(g["dual"] - D) <= 1e-6 * abs(P)


@pytest.mark.parametrize("ny,nx", SIZES[:5])
def test_emd_pd_step_generic_sizes(gpctx, ny, nx):
    from paper_1805_09453_amd._lib import GP_KIND_EMD
    h, tau = 1.0 / max(ny, nx), 0.3
    r0, r1 = mixture(ny, nx, 5)
    f_ref, psi = oemd.setup(r0, r1, h)
    gpx, gpy = (f32(a) for a in grid.grad(psi, h))
    ux, uy = np.zeros_like(f_ref), np.zeros_like(f_ref)
    px, py = np.zeros_like(f_ref), np.zeros_like(f_ref)
    pbx, pby = px.copy(), py.copy()
    for _ in range(4):
        ux, uy, px, py, pbx, pby = oemd.step(ux, uy, px, py, pbx, pby, gpx, gpy, h, tau, 1 / tau)
    ux, uy = oemd.leray(f32(ux), f32(uy), h)
    px, py, pbx, pby = (f32(a) for a in (px, py, pbx, pby))
    ref = oemd.step(ux, uy, px, py, pbx, pby, gpx, gpy, h, tau, 1 / tau)
    announce(f"emd set-up and pd_step {ny}x{nx}")
    f, gpsi = gpctx.emd_setup(dev(r0), dev(r1), h)
    assert field_err(host(f), f_ref) <= 1e-6
    assert field_err(host(gpsi)[0], gpx) <= 1e-6 and field_err(host(gpsi)[1], gpy) <= 1e-6
    st = gpctx.make_state(GP_KIND_EMD, dev(f_ref), h, tau, gpsi=dev(np.stack([gpx, gpy])),
                          u=dev(np.stack([ux, uy])), p=dev(np.stack([px, py])), pbar=dev(np.stack([pbx, pby])))
    gpctx.pd_step(st, 1)
    got = (host(st.u)[0], host(st.u)[1], host(st.p)[0], host(st.p)[1], host(st.pbar)[0], host(st.pbar)[1])
    errs = [field_err(g, r) for g, r in zip(got, ref)]
    print(["%.2e" % e for e in errs])
    assert max(errs) <= 1e-5
    g = gpctx.pd_gap(st)
    P = oemd.primal(ref[0], ref[1], gpx, gpy, h)
    D = oemd.certificate(ref[2], ref[3], f32(f_ref), h)[0]
    assert abs(g["primal"] - P) <= 1e-6 * P and abs(g["dual"] - D) <= 2e-6 * P


def test_pd_step_alternating_states_and_parameters(gpctx):
    """pd_step on 7-smooth grids keeps the arguments of its launches in a device
    table that it rewrites when the state changes: two states of different sizes
    stepped in turn, and one of them with its step size changed between calls,
    each match the oracle's iterations."""
    from paper_1805_09453_amd._lib import GP_KIND_ROF
    h, lam = 1.0, 8.0
    cases = [(96, 160, 21), (75, 105, 22)]
    host_st, dev_st = [], []
    for ny, nx, seed in cases:
        I = scene(ny, nx, seed)
        z = np.zeros_like(I)
        host_st.append([I, z, z, z, z, z])  # I, u, px, py, pbx, pby
        dev_st.append(gpctx.make_state(GP_KIND_ROF, dev(I), h, 0.02, lam=lam, u=dev(z), p=dev(np.stack([z, z])),
                                       pbar=dev(np.stack([z, z]))))
    announce("pd_step on two 7-smooth states in turn, one with its tau changed")
    for rnd, tau in enumerate((0.02, 0.02, 0.05)):
        for k in (0, 1):
            I, u, px, py, pbx, pby = host_st[k]
            t = tau if k == 0 else 0.02
            dev_st[k].c.tau = t
            dev_st[k].c.sigma = 1.0 / t
            gpctx.pd_step(dev_st[k], 1)
            # the oracle's state rounded to FP32 before each step, as the GPU stores it
            u, px, py, pbx, pby = orof.step(*(f32(a) for a in (u, px, py, pbx, pby)), I, h, lam, t, 1 / t)
            host_st[k] = [I, u, px, py, pbx, pby]
            got = (host(dev_st[k].u), host(dev_st[k].p)[0], host(dev_st[k].p)[1])
            errs = [field_err(g_, r) for g_, r in zip(got, (u, px, py))]
            print(rnd, k, ["%.2e" % e for e in errs])
            assert max(errs) <= 1e-5


@pytest.mark.parametrize("ny,nx,norm", [(720, 720, 0), (96, 160, 1)])
def test_rof_solver_loop_generic_sizes(gpctx, ny, nx, norm):
    from paper_1805_09453_amd import Options
    K = 12
    I = scene(ny, nx, 33)
    announce(f"rof_solve {ny}x{nx} {K} iterations, norm {norm}")
    u, p, rep = gpctx.rof_solve(dev(I), 1.0, 8.0, Options(tau=0.01, tol=0.0, max_iter=K, check_every=K, norm=norm))
    ref = orof.solve(I, 1.0, 8.0, 0.01, tol=0.0, max_iter=K, check_every=K, norm=norm)
    errs = [field_err(host(u), ref.u), field_err(host(p)[0], ref.px), field_err(host(p)[1], ref.py)]
    print(["%.2e" % e for e in errs], rep["primal"], ref.primal, rep["dual"], ref.dual)
    assert rep["iters"] == K and max(errs) <= 1e-5
    assert abs(rep["primal"] - ref.primal) <= 1e-6 * abs(ref.primal)
    assert abs(rep["dual"] - ref.dual) <= 1e-6 * abs(ref.primal)


@pytest.mark.parametrize("ny,nx,sigma_tau,warm", [(320, 320, 1.0, False), (96, 160, 0.5, False), (448, 448, 1.0, True)])
def test_emd_solver_loop_generic_sizes(gpctx, ny, nx, sigma_tau, warm):
    from paper_1805_09453_amd import Options
    K, tau = 10, 0.3
    h = 1.0 / max(ny, nx)
    r0, r1 = mixture(ny, nx, 9)
    X, Y = synth.cell_centres(ny, nx)
    phi0 = f32(0.3 * np.sin(3 * X) * np.cos(2 * Y)) if warm else None
    announce(f"emd_solve {ny}x{nx} {K} iterations, sigma tau {sigma_tau}, warm {warm}")
    m, phi, rep = gpctx.emd_solve(dev(r0), dev(r1), h, Options(tau=tau, sigma=sigma_tau / tau, tol=0.0, max_iter=K,
                                                               check_every=K, warm_start=warm),
                                  phi=dev(phi0) if warm else None)
    ref = oemd.solve(r0, r1, h, tau=tau, sigma=sigma_tau / tau, tol=0.0, max_iter=K, check_every=K, phi0=phi0)
    D, L, phit = oemd.certificate(ref.px, ref.py, ref.f, h)
    mg = host(m)
    errs = [field_err(mg[0], ref.m[0]), field_err(mg[1], ref.m[1]), field_err(host(phi), phit)]
    print(["%.2e" % e for e in errs], rep["primal"], ref.primal, rep["dual"], D)
    assert rep["iters"] == K and max(errs) <= 1e-5
    assert abs(rep["primal"] - ref.primal) <= 1e-6 * ref.primal and abs(rep["dual"] - D) <= 2e-6 * ref.primal


def test_full_solves_reach_the_oracle_optimum_on_a_generic_grid(gpctx):
    """96 x 160: ROF to a 1e-6 gap and EMD to 1e-5, objective error against long oracle solves."""
    from paper_1805_09453_amd import Options
    ny, nx = 96, 160
    I = scene(ny, nx, 44)
    announce("rof_solve 96x160 to 1e-6")
    u, _, rep = gpctx.rof_solve(dev(I), 1.0, 8.0, Options(tau=0.01, tol=1e-6, max_iter=40000, check_every=10))
    ref = orof.solve(I, 1.0, 8.0, 0.01, tol=1e-9, max_iter=200000, check_every=100)
    err = abs(orof.primal(host(u), I, 1.0, 8.0) - ref.primal) / ref.primal
    print("ROF", rep["iters"], err)
    assert rep["converged"] and err <= 1e-5
    h = 1.0 / nx
    r0, r1 = mixture(ny, nx, 45)
    announce("emd_solve 96x160 to 1e-5")
    m, _, rep = gpctx.emd_solve(dev(r0), dev(r1), h, Options(tau=0.3, tol=1e-5, max_iter=100000, check_every=50))
    eref = oemd.solve(r0, r1, h, tau=0.3, tol=2e-6, max_iter=400000, check_every=200)
    f_ref, _ = oemd.setup(r0, r1, h)
    val, _ = oemd.flux_value(host(m)[0], host(m)[1], f_ref, h)
    print("EMD", rep["iters"], val, eref.primal, eref.dual)
    assert rep["converged"]
    assert abs(val - eref.primal) <= 1e-5 * eref.primal
    assert rep["dual"] <= eref.primal * (1 + 1e-6)


def test_unsupported_sides_and_options(gpctx):
    from paper_1805_09453_amd import GPError, Options
    from paper_1805_09453_amd._lib import GP_EUNSUPPORTED
    bad = dev(np.ones((64, 66)))   # 66 = 2 * 3 * 11
    with pytest.raises(GPError) as e:
        gpctx.dct_poisson(bad, h=1.0, alpha=1.0)
    assert e.value.code == GP_EUNSUPPORTED
    with pytest.raises(GPError) as e:
        gpctx.rof_solve(dev(np.ones((96, 96))), 1.0, 8.0, Options(tau=0.01, ergodic=True))
    assert e.value.code == GP_EUNSUPPORTED


def test_batch_with_generic_sides_equals_single_solves(gpctx):
    """A batch mixing non-power-of-two sides (square, rectangular, odd) with a
    power-of-two instance: every instance equals its single-instance solve bit for
    bit, and one ROF instance reaches the oracle's optimum."""
    from paper_1805_09453_amd import Options
    from paper_1805_09453_amd._lib import GP_KIND_EMD, GP_KIND_ROF

    def rof_p(ny, nx, seed, lam=8.0, tau=0.01):
        return {"kind": GP_KIND_ROF, "I": dev(scene(ny, nx, seed)), "h": 1.0, "lam": lam, "tau": tau}

    def emd_p(ny, nx, seed, tau=0.3):
        r0, r1 = mixture(ny, nx, seed)
        return {"kind": GP_KIND_EMD, "rho0": dev(r0), "rho1": dev(r1), "h": 1.0 / max(ny, nx), "tau": tau}

    probs = [rof_p(96, 96, 1), emd_p(75, 105, 2), rof_p(96, 160, 3), emd_p(96, 96, 4), rof_p(96, 96, 5),
             rof_p(64, 64, 6), emd_p(96, 96, 7), rof_p(320, 320, 8, lam=4.0, tau=0.02)]
    opts = Options(tau=1.0, tol=1e-4, max_iter=2000, check_every=10)
    announce(f"gp_batch_solve with non-power-of-two sides, {len(probs)} instances")
    outs, reps, rc = gpctx.batch_solve(probs, opts)
    for i, q in enumerate(probs):
        announce(f"single solve for batch instance {i}")
        o = Options(tau=q["tau"], tol=opts.tol, max_iter=opts.max_iter, check_every=10)
        if q["kind"] == GP_KIND_ROF:
            ref, _, rrep = gpctx.rof_solve(q["I"], q["h"], q["lam"], o)
        else:
            ref, _, rrep = gpctx.emd_solve(q["rho0"], q["rho1"], q["h"], o, want_phi=False)
        print(i, tuple(q[k].shape for k in ("I", "rho0") if k in q), reps[i]["iters"], rrep["iters"],
              reps[i]["rel_gap"], rrep["rel_gap"])
        assert reps[i]["iters"] == rrep["iters"] and reps[i]["converged"] == rrep["converged"]
        assert reps[i]["primal"] == rrep["primal"] and reps[i]["dual"] == rrep["dual"]
        np.testing.assert_array_equal(host(outs[i]), host(ref))
    assert len({r["iters"] for r in reps}) > 1
    # ROF 96 x 160 instance: objective within 1e-4 of the oracle's optimum at this tolerance
    I = host(probs[2]["I"])
    ref = orof.solve(I, 1.0, 8.0, 0.01, tol=1e-9, max_iter=200000, check_every=100)
    err = abs(orof.primal(host(outs[2]), I, 1.0, 8.0) - ref.primal) / ref.primal
    print("oracle objective error", err)
    assert err <= 1e-4


PLANS_720 = [[5, 3, 3, 8, 2], [8, 2, 5, 3, 3], [5, 3, 3, 4, 4], [4, 4, 5, 3, 3], [2, 3, 2, 5, 2, 3, 2]]


@pytest.mark.parametrize("plan", PLANS_720)
def test_every_radix_plan_computes_the_same_solve(plan):
    """720 = 2^4 3^2 5: the candidate plans the tuner times and one it never
    picks (radix 2 and 3 passes interleaved) all give the oracle's solve in FP32
    and FP64, and the plan set is the plan used."""
    import torch
    from paper_1805_09453_amd import Context
    n = 720
    b = f32(np.random.default_rng(5).standard_normal((n, n)))
    ref = grid.poisson_solve(b, 1.0, 0.3)
    with Context(n, n) as ctx:
        ctx.set_radix_plan(False, n, plan)
        ctx.set_radix_plan(True, n, plan)
        assert ctx.get_radix_plan(False, n) == plan and ctx.get_radix_plan(True, n) == plan
        announce(f"dct_poisson {n}x{n} with radix plan {plan}")
        err = field_err(host(ctx.dct_poisson(dev(b), h=1.0, alpha=0.3)), ref)
        err64 = field_err(ctx.dct_poisson_f64(dev(b, torch.float64), h=1.0, alpha=0.3).cpu().numpy(), ref)
        print(plan, f"FP32 {err:.2e}  FP64 {err64:.2e}")
        assert err <= 5e-6 and err64 <= 1e-12
        assert ctx.get_radix_plan(False, n) == plan


def test_radix_plan_tuned_on_first_use_and_validated():
    from paper_1805_09453_amd import Context, GPError
    n = 720
    with Context(n, n) as ctx:
        default = ctx.get_radix_plan(False, n)
        assert default == [5, 3, 3, 8, 2]
        ctx.dct_poisson(dev(np.ones((n, n))), h=1.0, alpha=0.3)   # measures the FP32 candidates
        plan = ctx.get_radix_plan(False, n)
        print("tuned FP32 plan for 720:", plan)
        assert plan in PLANS_720[:4] and int(np.prod(plan)) == n
        for bad in ([6, 120], [8, 2, 5, 3, 2], [2] * 17, []):
            with pytest.raises(GPError):
                ctx.set_radix_plan(False, n, bad)
        with pytest.raises(GPError):
            ctx.get_radix_plan(False, 512)   # powers of two have their fixed schedule
        with pytest.raises(GPError):
            ctx.get_radix_plan(False, 110)   # 11 is not a supported factor


def test_radix_plan_set_between_solves_is_used():
    """A plan set between two solves of the same size on one context is the plan
    the second solve runs (the single-solve launch tables are rebuilt): its result
    equals, bit for bit, that of a fresh context given the same plan."""
    import torch
    from paper_1805_09453_amd import Context, Options
    n = 720
    I = dev(scene(n, n, 11))
    opts = Options(tau=0.01, tol=0.0, max_iter=30, check_every=30)
    plan_a, plan_b = PLANS_720[0], PLANS_720[3]
    announce(f"rof_solve {n}x{n}: plan {plan_a}, then {plan_b} on the same context")
    with Context(n, n) as ctx:
        u = torch.empty_like(I)
        p = torch.empty((2, n, n), device="cuda")
        ctx.set_radix_plan(False, n, plan_a)
        ctx.rof_solve(I, 1.0, 8.0, opts, u=u, p=p)
        ua = u.clone()
        ctx.set_radix_plan(False, n, plan_b)
        ctx.rof_solve(I, 1.0, 8.0, opts, u=u, p=p)
        ub = u.clone()
    with Context(n, n) as ctx:
        ctx.set_radix_plan(False, n, plan_b)
        uc, _, _ = ctx.rof_solve(I, 1.0, 8.0, opts)
    print("plan a vs b max diff", float((ua - ub).abs().max()))
    assert torch.equal(ub, uc)
