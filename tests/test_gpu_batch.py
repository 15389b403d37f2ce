"""Batched solves (gp_batch_solve): every instance of a mixed batch must equal
the matching single-instance solve bit for bit (the iteration of Algorithm 2 is
per instance; stacking only changes which launch runs it), and instances are
checked against the FP64 oracle through the single-instance parity."""
import json
import os

import numpy as np
import pytest

import synth
from conftest import announce
from oracle import emd as oemd
from oracle import rof as orof

pytestmark = pytest.mark.gpu
GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def dev(a):
    import torch
    return torch.tensor(np.ascontiguousarray(a, dtype=np.float32), device="cuda")


def host(t):
    return t.cpu().double().numpy()


def rof_problem(n, seed, lam, tau, h=1.0):
    from paper_1805_09453_amd._lib import GP_KIND_ROF
    return {"kind": GP_KIND_ROF, "I": dev(synth.rof_scene(n, seed)), "h": h, "lam": lam, "tau": tau}


def emd_problem(n, seed, tau, k=4):
    from paper_1805_09453_amd._lib import GP_KIND_EMD
    r0, r1 = synth.emd_mixture_pair(n, seed, k=k)
    return {"kind": GP_KIND_EMD, "rho0": dev(r0), "rho1": dev(r1), "h": 1.0 / n, "tau": tau}


def single(ctx, q, opts):
    from paper_1805_09453_amd._lib import GP_KIND_ROF
    if q["kind"] == GP_KIND_ROF:
        u, _, rep = ctx.rof_solve(q["I"], q["h"], q["lam"], opts)
        return u, rep
    m, _, rep = ctx.emd_solve(q["rho0"], q["rho1"], q["h"], opts, want_phi=False)
    return m, rep


def test_batch_mixed_equals_single_solves(gpctx):
    """Two ROF sizes, two lambdas, two EMD sizes, interleaved: outputs, iteration
    counts and gaps equal the single-instance solves exactly."""
    from paper_1805_09453_amd import Options
    probs = [rof_problem(128, 1, 8.0, 0.01), emd_problem(64, 2, 0.3), rof_problem(64, 3, 8.0, 0.01),
             rof_problem(128, 4, 8.0, 0.01), rof_problem(64, 5, 4.0, 0.02), emd_problem(128, 6, 0.3),
             emd_problem(64, 7, 0.3), rof_problem(64, 8, 8.0, 0.01)]
    opts = Options(tau=1.0, tol=1e-4, max_iter=600, check_every=10)
    announce(f"gp_batch_solve mixed batch of {len(probs)}")
    outs, reps, rc = gpctx.batch_solve(probs, opts)
    for i, q in enumerate(probs):
        announce(f"single solve for batch instance {i}")
        ref, rrep = single(gpctx, q, Options(tau=q["tau"], tol=opts.tol, max_iter=opts.max_iter, check_every=10))
        print(i, reps[i]["iters"], rrep["iters"], reps[i]["rel_gap"], rrep["rel_gap"])
        assert reps[i]["iters"] == rrep["iters"]
        assert reps[i]["converged"] == rrep["converged"]
        assert reps[i]["rel_gap"] == rrep["rel_gap"]
        assert reps[i]["primal"] == rrep["primal"] and reps[i]["dual"] == rrep["dual"]
        np.testing.assert_array_equal(host(outs[i]), host(ref))
    # the instances did not all stop together (retirement was exercised)
    assert len({r["iters"] for r in reps}) > 1


def test_batch_rof_instance_matches_oracle_optimum(gpctx):
    """The 64x64 config-0 scene inside a batch of 16: objective within 1e-5 of
    the oracle's F*, and the batch's own gap is a valid certificate."""
    from paper_1805_09453_amd import Options
    from paper_1805_09453_amd._lib import GP_KIND_ROF
    I0 = synth.rof_scene(64, synth.config_seed(0))
    with open(os.path.join(GOLDEN, "oracle_references.json")) as fh:
        Fstar = json.load(fh)["rof_c0"]["primal"]
    probs = [{"kind": GP_KIND_ROF, "I": dev(I0), "h": 1.0, "lam": 8.0, "tau": 0.01}]
    probs += [rof_problem(64, 100 + s, 8.0, 0.01) for s in range(15)]
    announce("gp_batch_solve 16 x ROF 64x64")
    outs, reps, rc = gpctx.batch_solve(probs, Options(tau=0.01, tol=1e-6, max_iter=20000, check_every=10))
    assert all(r["converged"] for r in reps)
    Fg = orof.primal(host(outs[0]), I0, 1.0, 8.0)
    assert abs(Fg - Fstar) / Fstar <= 1e-5
    for i, q in enumerate(probs):
        P = orof.primal(host(outs[i]), host(q["I"]), 1.0, 8.0)
        assert abs(reps[i]["primal"] - P) / P < 1e-6


def test_batch_emd_translated_pairs_exact_values(gpctx):
    """Translated Gaussians (exact EMD = shift / (1 + floor)) of two sizes in one batch."""
    from paper_1805_09453_amd import Options
    from paper_1805_09453_amd._lib import GP_KIND_EMD
    probs, exact = [], []
    for n in (64, 128, 128):
        r0, r1, s = synth.translated_gaussian_pair(n)
        probs.append({"kind": GP_KIND_EMD, "rho0": dev(r0), "rho1": dev(r1), "h": 1.0 / n, "tau": 0.25})
        exact.append(s / (1 + synth.scenes.DENSITY_FLOOR))
    announce("gp_batch_solve 3 x EMD translated pairs")
    outs, reps, rc = gpctx.batch_solve(probs, Options(tau=0.25, tol=1e-4, max_iter=50000, check_every=50))
    for i, q in enumerate(probs):
        n = q["rho0"].shape[0]
        f_ref, _ = oemd.setup(host(q["rho0"]), host(q["rho1"]), 1.0 / n)
        val, _ = oemd.flux_value(host(outs[i])[0], host(outs[i])[1], f_ref, 1.0 / n)
        print(n, reps[i], val, exact[i])
        assert reps[i]["converged"]
        assert reps[i]["dual"] <= exact[i] * (1 + 1e-6) <= reps[i]["primal"] * (1 + 2e-6)
        assert abs(val - exact[i]) / exact[i] <= 2e-4


def test_batch_max_iter_and_errors(gpctx):
    from paper_1805_09453_amd import GPError, Options
    from paper_1805_09453_amd._lib import GP_EMASS, GP_ENOTCONV, GP_EUNSUPPORTED, GP_KIND_EMD
    probs = [rof_problem(64, 1, 8.0, 0.01), rof_problem(64, 2, 8.0, 0.01)]
    announce("gp_batch_solve max_iter 20")
    outs, reps, rc = gpctx.batch_solve(probs, Options(tau=0.01, tol=0.0, max_iter=20, check_every=10))
    assert rc == GP_ENOTCONV and all(r["iters"] == 20 and not r["converged"] for r in reps)
    # an odd check_every: chunks of C = 6 iterations, the first check at or after max_iter = 20 is 24
    announce("gp_batch_solve max_iter 20, check_every 5")
    outs, reps, rc = gpctx.batch_solve(probs, Options(tau=0.01, tol=0.0, max_iter=20, check_every=5))
    assert rc == GP_ENOTCONV and all(r["iters"] == 24 and not r["converged"] for r in reps)
    # the batch starts from zero: a warm start is refused, and so is a non-finite image
    from paper_1805_09453_amd._lib import GP_EINVAL
    with pytest.raises(GPError) as e:
        gpctx.batch_solve(probs, Options(tau=0.01, warm_start=True))
    assert e.value.code == GP_EINVAL
    nan = rof_problem(64, 4, 8.0, 0.01)
    nan["I"][7, 9] = float("nan")
    with pytest.raises(GPError) as e:
        gpctx.batch_solve([probs[0], nan], Options(tau=0.01))
    assert e.value.code == GP_EINVAL and "instance 1" in str(e.value)
    bad = emd_problem(64, 3, 0.3)
    bad["rho1"] = bad["rho1"] * 1.01
    announce("gp_batch_solve mass mismatch")
    with pytest.raises(GPError) as e:
        gpctx.batch_solve([probs[0], bad], Options(tau=0.3))
    assert e.value.code == GP_EMASS and "instance 1" in str(e.value)
    odd = {"kind": GP_KIND_EMD, "rho0": dev(np.ones((88, 88))), "rho1": dev(np.ones((88, 88))), "h": 1.0,
           "tau": 0.3}
    with pytest.raises(GPError) as e:
        gpctx.batch_solve([odd], Options(tau=0.3))
    assert e.value.code == GP_EUNSUPPORTED


def test_batch_emd_potential_output_equals_single_solve(gpctx):
    """The optional per-instance potential (the scaled certificate of the final
    dual) equals emd_solve's phi, also for instances that retire early while
    others keep running."""
    import torch
    from paper_1805_09453_amd import Options
    probs = [emd_problem(64, 21, 0.3), emd_problem(64, 22, 0.3, k=8), emd_problem(128, 23, 0.3)]
    for q in probs:
        q["phi"] = torch.empty_like(q["rho0"])
    opts = Options(tau=0.3, tol=1e-4, max_iter=4000, check_every=20)
    announce("gp_batch_solve EMD potentials")
    outs, reps, _ = gpctx.batch_solve(probs, opts)
    for i, q in enumerate(probs):
        m, phi, rep = gpctx.emd_solve(q["rho0"], q["rho1"], q["h"], opts)
        print(i, reps[i]["iters"], rep["iters"])
        assert reps[i]["iters"] == rep["iters"]
        assert torch.equal(outs[i], m) and torch.equal(q["phi"], phi)


def test_launch_shapes_do_not_change_results(gpctx):
    """Every FFT group computes the same arithmetic whatever the number of groups
    per workgroup or the tile width of the intermediate: solves under other
    row / column / tile shapes are bit-identical."""
    from paper_1805_09453_amd import GPError, Options
    I = dev(synth.rof_scene(256, 31))
    r0, r1 = synth.emd_mixture_pair(128, 32, k=4)
    r0, r1 = dev(r0), dev(r1)
    o_rof = Options(tau=0.01, tol=0.0, max_iter=60, check_every=20)
    o_emd = Options(tau=0.3, tol=0.0, max_iter=60, check_every=20)
    saved = [gpctx.get_shape(False, 256), gpctx.get_shape(True, 128)]
    announce("shape variants ROF 256x256 / EMD 128x128")
    u0, p0, rep0 = gpctx.rof_solve(I, 1.0, 8.0, o_rof)
    m0, phi0, rpe0 = gpctx.emd_solve(r0, r1, 1.0 / 128, o_emd)
    try:
        for rg, cg, tw in ((8, 2, 4), (32, 4, 64), (16, 32, 2), (16, 1, 32)):
            gpctx.set_shape(False, 256, rg, cg, tw)
            gpctx.set_shape(True, 128, 16, min(cg, 16), tw)
            print("shapes", gpctx.get_shape(False, 256), gpctx.get_shape(True, 128))
            u, p, rep = gpctx.rof_solve(I, 1.0, 8.0, o_rof)
            m, phi, rpe = gpctx.emd_solve(r0, r1, 1.0 / 128, o_emd)
            assert rep["primal"] == rep0["primal"] and rep["dual"] == rep0["dual"]
            np.testing.assert_array_equal(host(u), host(u0))
            np.testing.assert_array_equal(host(m), host(m0))
            np.testing.assert_array_equal(host(phi), host(phi0))
        with pytest.raises(GPError):
            gpctx.set_shape(False, 256, 3, 0)   # not a whole number of waves
        with pytest.raises(GPError):
            gpctx.set_shape(False, 256, 0, 3)   # not a power of two
        with pytest.raises(GPError):
            gpctx.set_shape(False, 256, 0, 0, 12)  # tile width not a power of two
    finally:
        gpctx.set_shape(False, 256, *saved[0])
        gpctx.set_shape(True, 128, *saved[1])


@pytest.mark.parametrize("n", [256, 512])
def test_launch_shapes_do_not_change_results_16_values_per_thread(gpctx, n):
    """Lengths 256 and 512 hold 16 values per thread, so a slot's spectrum indices
    are only N/8 = 32 or 64 apart, at or below the widest strip of the tiled
    intermediate: ROF (FP32) and EMD (FP64) solves under the extreme and middle
    row / column / tile settings are bit-identical to the default ones."""
    from paper_1805_09453_amd import Options
    I = dev(synth.rof_scene(n, 41))
    r0, r1 = synth.emd_mixture_pair(n, 42, k=4)
    r0, r1 = dev(r0), dev(r1)
    o_rof = Options(tau=0.01, tol=0.0, max_iter=40, check_every=20)
    o_emd = Options(tau=0.3, tol=0.0, max_iter=40, check_every=20)
    saved = [gpctx.get_shape(False, n), gpctx.get_shape(True, n)]
    announce(f"shape variants ROF and EMD {n}x{n}")
    u0, _, rep0 = gpctx.rof_solve(I, 1.0, 8.0, o_rof)
    m0, phi0, rpe0 = gpctx.emd_solve(r0, r1, 1.0 / n, o_emd)
    # (row groups, column groups, tile width): FP32 first, then FP64
    shapes = {256: [((4, 1, 2), (4, 1, 2)), ((32, 32, 64), (28, 32, 64)), ((8, 4, 16), (8, 4, 16))],
              512: [((2, 1, 2), (2, 1, 2)), ((16, 16, 64), (14, 16, 64)), ((4, 8, 16), (4, 8, 16))]}[n]
    try:
        for s32, s64 in shapes:
            gpctx.set_shape(False, n, *s32)
            gpctx.set_shape(True, n, *s64)
            print("shapes", gpctx.get_shape(False, n), gpctx.get_shape(True, n))
            u, _, rep = gpctx.rof_solve(I, 1.0, 8.0, o_rof)
            m, phi, rpe = gpctx.emd_solve(r0, r1, 1.0 / n, o_emd)
            assert rep["primal"] == rep0["primal"] and rep["dual"] == rep0["dual"]
            assert rpe["primal"] == rpe0["primal"] and rpe["dual"] == rpe0["dual"]
            np.testing.assert_array_equal(host(u), host(u0))
            np.testing.assert_array_equal(host(m), host(m0))
            np.testing.assert_array_equal(host(phi), host(phi0))
    finally:
        gpctx.set_shape(False, n, *saved[0])
        gpctx.set_shape(True, n, *saved[1])


def test_batch_rectangular_anisotropic_equals_single_solves(gpctx):
    """Rectangular instances (wide and tall, rows of the radix-8 and radix-16
    length classes) under the anisotropic norm: each instance of the batch
    equals its single-instance solve bit for bit, as for square grids."""
    from paper_1805_09453_amd import Options
    from paper_1805_09453_amd._lib import GP_KIND_EMD, GP_KIND_ROF, GP_NORM_ANISO

    def rof_rect(ny, nx, seed, lam, tau):
        I = synth.rof_scene(max(ny, nx), seed)[:ny, :nx]
        return {"kind": GP_KIND_ROF, "I": dev(I), "h": 1.0, "lam": lam, "tau": tau}

    def emd_rect(ny, nx, seed, tau):
        r0, r1 = synth.emd_mixture_pair(max(ny, nx), seed, k=4)
        r0 = np.asarray(r0[:ny, :nx], dtype=np.float32).astype(np.float64)
        r1 = np.asarray(r1[:ny, :nx], dtype=np.float32).astype(np.float64)
        r1 *= r0.sum() / r1.sum()
        return {"kind": GP_KIND_EMD, "rho0": dev(r0), "rho1": dev(r1), "h": 1.0 / max(ny, nx), "tau": tau}

    probs = [rof_rect(64, 128, 11, 8.0, 0.01), emd_rect(128, 64, 12, 0.3), rof_rect(128, 64, 13, 8.0, 0.01),
             emd_rect(64, 1024, 14, 0.3), rof_rect(64, 128, 15, 8.0, 0.01), emd_rect(128, 64, 16, 0.3)]
    opts = Options(tau=1.0, tol=1e-4, max_iter=400, check_every=10, norm=GP_NORM_ANISO)
    announce(f"gp_batch_solve rectangular anisotropic batch of {len(probs)}")
    outs, reps, rc = gpctx.batch_solve(probs, opts)
    for i, q in enumerate(probs):
        announce(f"single solve for rectangular batch instance {i}")
        ref, rrep = single(gpctx, q, Options(tau=q["tau"], tol=opts.tol, max_iter=opts.max_iter, check_every=10,
                                             norm=GP_NORM_ANISO))
        print(i, reps[i]["iters"], rrep["iters"], reps[i]["rel_gap"], rrep["rel_gap"])
        assert reps[i]["iters"] == rrep["iters"] and reps[i]["converged"] == rrep["converged"]
        assert reps[i]["rel_gap"] == rrep["rel_gap"]
        assert reps[i]["primal"] == rrep["primal"] and reps[i]["dual"] == rrep["dual"]
        np.testing.assert_array_equal(host(outs[i]), host(ref))


def test_batch_1024_instances_match_oracle_optimum(gpctx):
    """The first ROF and the first EMD 1024^2 instance of the 512-instance mixed
    batch (power-of-two sides), solved inside a batch with the six instances that
    precede the first of them, to a 1e-5 relative gap: the FP64 objective of each
    downloaded result lies within 1e-5 of the oracle's certified optimum."""
    from paper_1805_09453_amd import Options
    from paper_1805_09453_amd._lib import GP_KIND_EMD, GP_KIND_ROF
    with open(os.path.join(GOLDEN, "oracle_references.json")) as fh:
        refs = json.load(fh)["batch_1024"]["cases"]
    insts = synth.batch_instances(512)
    first = min(refs["rof"]["index"], refs["emd"]["index"])
    pick = sorted(set(range(max(0, first - 6), first)) | {refs["rof"]["index"], refs["emd"]["index"]})
    probs, xs = [], []
    for i in pick:
        q = insts[i]
        x = synth.batch_instance_inputs(q)
        xs.append(x)
        if q["kind"] == "rof":
            probs.append({"kind": GP_KIND_ROF, "I": dev(x["image"]), "h": 1.0, "lam": 8.0, "tau": 0.01})
        else:
            probs.append({"kind": GP_KIND_EMD, "rho0": dev(x["rho0"]), "rho1": dev(x["rho1"]),
                          "h": 1.0 / q["n"], "tau": 0.3})
    announce(f"gp_batch_solve of instances {pick} of the 512-instance batch to 1e-5")
    outs, reps, rc = gpctx.batch_solve(probs, Options(tau=1.0, tol=1e-5, max_iter=40000, check_every=20))
    assert all(r["converged"] for r in reps)
    for kind in ("rof", "emd"):
        ref = refs[kind]
        j = pick.index(ref["index"])
        q, x = insts[ref["index"]], xs[j]
        assert q["kind"] == kind and q["n"] == 1024 and q["seed"] == ref["seed"]
        if kind == "rof":
            I32 = np.asarray(x["image"], np.float32).astype(np.float64)
            val = orof.primal(host(outs[j]), I32, 1.0, 8.0)
            assert val >= ref["dual"] * (1 - 1e-12)
        else:
            r0, r1 = (np.asarray(x[k], np.float32).astype(np.float64) for k in ("rho0", "rho1"))
            f_ref, _ = oemd.setup(r0, r1, 1.0 / 1024)
            val, _ = oemd.flux_value(host(outs[j])[0], host(outs[j])[1], f_ref, 1.0 / 1024)
            assert val >= ref["dual"] * (1 - 1e-6)
        err = abs(val - ref["primal"]) / ref["primal"]
        print(kind, "iters", reps[j]["iters"], "gap %.2e" % reps[j]["rel_gap"], "FP64 value", val,
              "oracle", ref["primal"], "err %.2e" % err)
        assert err <= 1e-5
