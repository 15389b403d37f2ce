"""Writes oracle_references.json: long FP64 oracle runs that serve as the
ground-truth objective F* for the GPU parity tests (the paper's own protocol in
section 4 computes a ground truth by a long G-prox run certified by the gap).

Calls only oracle/ and synth/ (no GPU code).  Usage:
    python tests/golden/make_oracle_references.py [name ...]
"""
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import synth  # noqa: E402
from oracle import emd, grid, rof  # noqa: E402

OUT = os.path.join(HERE, "oracle_references.json")


def rof_c0():
    I = synth.rof_scene(64, synth.config_seed(0))
    r = rof.solve(I, 1.0, 8.0, 0.005, tol=1e-10, max_iter=200000, check_every=100)
    return dict(workload="ROF 64x64, 3-6 shapes + N(0,0.1^2), lambda=8, h=1, seed config 0",
                tau=0.005, iters=r.iters, primal=r.primal, dual=r.dual, rel_gap=r.rel_gap)


def emd_c1_mixture():
    n = 256
    rho0, rho1 = synth.emd_mixture_pair(n, synth.config_seed(1), k=4)
    r = emd.solve(rho0, rho1, 1.0 / n, tau=0.3, tol=2e-6, max_iter=150000, check_every=500)
    return dict(workload="EMD 256x256, 4-Gaussian mixtures with 1e-3 floor, h=1/256, seed config 1",
                tau=0.3, iters=r.iters, primal=r.primal, dual=r.dual, rel_gap=r.rel_gap)


def emd_aniso_64():
    import numpy as np

    from oracle import grid
    n = 64
    rho0, rho1 = synth.emd_mixture_pair(n, 17, k=2)
    # the densities as the GPU receives them (FP32)
    rho0, rho1 = (np.asarray(a, np.float32).astype(np.float64) for a in (rho0, rho1))
    r = emd.solve(rho0, rho1, 1.0 / n, tau=0.3, tol=1e-7, max_iter=400000, check_every=50, norm=grid.ANISO)
    return dict(workload="EMD 64x64, 2-Gaussian mixtures (seed 17) rounded to FP32, l1 grid norm, h=1/64",
                tau=0.3, iters=r.iters, primal=r.primal, dual=r.dual, rel_gap=r.rel_gap)


def _save(name, res):
    # re-read before writing: several jobs may run in parallel processes
    data = json.load(open(OUT)) if os.path.exists(OUT) else {}
    data[name] = res
    with open(OUT, "w") as fh:
        json.dump(data, fh, indent=2)


def _checkpoints(name, workload, tau, marks, t0):
    """Callback that stores (P, D) the first time the relative gap falls below
    each value of ``marks`` (entries name@mark), so that a long run leaves usable
    brackets of F* before it ends."""
    left = sorted(marks, reverse=True)

    def cb(it, P, D, g):
        print(" ", name, it, P, D, g, flush=True)
        while left and g <= left[0]:
            m = left.pop(0)
            _save(f"{name}@{m:g}", dict(workload=workload, tau=tau, iters=it, primal=P, dual=D, rel_gap=g,
                                         oracle_seconds=round(time.time() - t0, 1)))
    return cb


ROF_C2_WORKLOAD = "ROF 4096x4096, 50 shapes + N(0,0.1^2), lambda=8, h=1, seed config 2, image rounded to FP32"


def rof_c2_4096():
    """F* of the 4096^2 ROF workload (50 shapes, lambda 8, h 1) on the image as the
    GPU receives it (FP32), to a relative gap of 1e-7 (brackets stored on the way
    at 1e-5 and 1e-6)."""
    import numpy as np
    I = synth.rof_scene(4096, synth.config_seed(2), n_shapes=50, size_range=(0.02, 0.15))
    I = np.asarray(I, np.float32).astype(np.float64)
    cb = _checkpoints("rof_c2_4096", ROF_C2_WORKLOAD, 0.01, (1e-5, 1e-6), time.time())
    r = rof.solve(I, 1.0, 8.0, 0.01, tol=1e-7, max_iter=100000, check_every=25, callback=cb)
    return dict(workload=ROF_C2_WORKLOAD, tau=0.01, iters=r.iters, primal=r.primal, dual=r.dual, rel_gap=r.rel_gap)


EMD_C2_WORKLOAD = ("EMD 1024x1024, 16-Gaussian mixtures with 1e-3 floor, h=1/1024, seed config 2 instance 1, "
                   "densities rounded to FP32")


def emd_c2_1024():
    """Bracket [D, P] of F* for a 1024^2 pair of 16-Gaussian mixtures (the 4096^2
    recipe at 1024^2), densities rounded to FP32, to a relative gap of 1e-5
    (brackets stored on the way at 1e-4 and 3e-5)."""
    import numpy as np
    n = 1024
    rho0, rho1 = synth.emd_mixture_pair(n, synth.config_seed(2, 1), k=16)
    rho0, rho1 = (np.asarray(a, np.float32).astype(np.float64) for a in (rho0, rho1))
    cb = _checkpoints("emd_c2_1024", EMD_C2_WORKLOAD, 0.3, (1e-4, 3e-5), time.time())
    r = emd.solve(rho0, rho1, 1.0 / n, tau=0.3, tol=1e-5, max_iter=400000, check_every=250, callback=cb)
    return dict(workload=EMD_C2_WORKLOAD, tau=0.3, iters=r.iters, primal=r.primal, dual=r.dual, rel_gap=r.rel_gap)


def _count_to_eps(step, value, fstar, eps, max_iter):
    """The section 4 protocol: iterations from the zero start until F(u_n) - F* < eps
    (F evaluated after every iteration); None when max_iter is reached first."""
    for it in range(1, max_iter + 1):
        step()
        if value() - fstar < eps:
            return it
    return None


def paper_protocol_128():
    """The section 4 protocol run by the oracle at 128^2 (h = 1/128): ground truth
    F* certified by the gap to well below eps/10, the step size of each table's
    rule and the oracle's own iteration count to F(u_n) - F* < eps.  Inputs as the
    GPU receives them (FP32)."""
    import numpy as np
    n, h = 128, 1.0 / 128
    out = {}
    I = np.asarray(synth.disc_image(n, 0.25), np.float32).astype(np.float64)
    for lam in (10.0, 20.0):
        ref = rof.solve(I, h, lam, rof.step_rule_tau(I, h, lam, 1e-3), tol=1e-9, max_iter=400000, check_every=100)
        cases = [(1e-2, False), (1e-3, False)] + ([(1e-2, True)] if lam == 20.0 else [])
        for eps, gi in cases:
            tau = (np.sqrt(lam) * rof.tv_norm(I, h) / np.sqrt(eps)) if gi else rof.step_rule_tau(I, h, lam, eps)
            st = dict(u=np.zeros_like(I), px=np.zeros_like(I), py=np.zeros_like(I))
            st["pbx"], st["pby"] = st["px"].copy(), st["py"].copy()

            def step():
                st["u"], st["px"], st["py"], st["pbx"], st["pby"] = rof.step(
                    st["u"], st["px"], st["py"], st["pbx"], st["pby"], I, h, lam, tau, 1.0 / tau)
            it = _count_to_eps(step, lambda: rof.primal(st["u"], I, h, lam), ref.primal, eps, 5000)
            out[f"rof_lam{lam:g}_eps{eps:g}{'_gi' if gi else ''}"] = dict(
                table=1 if lam == 10.0 else (3 if gi else 2), lam=lam, eps=eps, grid_independent=gi, tau=tau,
                fstar=ref.primal, fstar_gap=ref.primal - ref.dual, iters=it)
    for kind in ("discs", "deltas"):
        r0, r1 = synth.uniform_disc_pair(n) if kind == "discs" else synth.delta_pair(n)
        r0, r1 = (np.asarray(a, np.float32).astype(np.float64) for a in (r0, r1))
        tau_ref = 1.0 if kind == "discs" else emd.step_rule_tau_singular(1e-3, n)
        ref = emd.solve(r0, r1, h, tau=tau_ref, tol=2e-6 if kind == "discs" else 1e-4, max_iter=400000,
                        check_every=100)
        cases = [(1e-3, 1.0, 6)] if kind == "discs" else [(1e-2, emd.step_rule_tau_singular(1e-2, n), 7),
                                                          (1e-2, 1.0, 8)]
        for eps, tau, table in cases:
            f, psi = emd.setup(r0, r1, h)
            gpx, gpy = grid.grad(psi, h)
            z = np.zeros_like(f)
            st = dict(ux=z.copy(), uy=z.copy(), px=z.copy(), py=z.copy(), pbx=z.copy(), pby=z.copy())

            def step():
                (st["ux"], st["uy"], st["px"], st["py"], st["pbx"], st["pby"]) = emd.step(
                    st["ux"], st["uy"], st["px"], st["py"], st["pbx"], st["pby"], gpx, gpy, h, tau, 1.0 / tau)
            it = _count_to_eps(step, lambda: emd.primal(st["ux"], st["uy"], gpx, gpy, h), ref.primal, eps, 5000)
            out[f"emd_{kind}_eps{eps:g}_table{table}"] = dict(table=table, pair=kind, eps=eps, tau=tau,
                                                              fstar=ref.primal, fstar_gap=ref.primal - ref.dual,
                                                              iters=it)
    for k, v in out.items():
        print(" ", k, v, flush=True)
    return dict(workload="section 4 protocol at 128x128, h = 1/128 (disc ROF; uniform-disc and Dirac EMD pairs)",
                cases=out)


def emd_ws_512():
    """Bracket of F* for held-out warm-start pair 0 (512^2, config 4 recipe),
    densities rounded to FP32, to a relative gap of 1e-5."""
    import numpy as np
    n, s = 512, 0
    seed = synth.config_seed(4, 900_000 + s)
    k = int(np.random.default_rng(seed).integers(4, 17))
    rho0, rho1 = (np.asarray(a, np.float32).astype(np.float64) for a in synth.emd_mixture_pair(n, seed, k=k))
    r = emd.solve(rho0, rho1, 1.0 / n, tau=0.3, tol=1e-5, max_iter=400000, check_every=250,
                  callback=lambda it, P, D, g: print("  emd_ws_512", it, P, D, g, flush=True))
    return dict(workload=f"EMD 512x512 held-out warm-start pair {s} ({k}-Gaussian mixtures), h=1/512, FP32 densities",
                held_out=s, tau=0.3, iters=r.iters, primal=r.primal, dual=r.dual, rel_gap=r.rel_gap)


def batch_1024():
    """F* of the first ROF and the first EMD 1024^2 instance of the 512-instance
    mixed batch (inputs rounded to FP32): ROF to a relative gap of 1e-7, EMD to 1e-5."""
    import numpy as np
    insts = synth.batch_instances(512)
    out = {}
    for kind in ("rof", "emd"):
        i = next(j for j, q in enumerate(insts) if q["kind"] == kind and q["n"] == 1024)
        x = synth.batch_instance_inputs(insts[i])
        if kind == "rof":
            I = np.asarray(x["image"], np.float32).astype(np.float64)
            r = rof.solve(I, 1.0, 8.0, 0.01, tol=1e-7, max_iter=200000, check_every=50)
            out[kind] = dict(index=i, seed=insts[i]["seed"], tau=0.01, lam=8.0, h=1.0, iters=r.iters,
                             primal=r.primal, dual=r.dual, rel_gap=r.rel_gap)
        else:
            r0, r1 = (np.asarray(x[k], np.float32).astype(np.float64) for k in ("rho0", "rho1"))
            r = emd.solve(r0, r1, 1.0 / 1024, tau=0.3, tol=1e-5, max_iter=400000, check_every=250)
            out[kind] = dict(index=i, seed=insts[i]["seed"], tau=0.3, h=1.0 / 1024, iters=r.iters,
                             primal=r.primal, dual=r.dual, rel_gap=r.rel_gap)
        print(" ", kind, out[kind], flush=True)
    return dict(workload="first ROF and first EMD 1024x1024 instance of synth.batch_instances(512), FP32 inputs",
                cases=out)


JOBS = {"rof_c0": rof_c0, "emd_c1_mixture": emd_c1_mixture, "emd_aniso_64": emd_aniso_64,
        "rof_c2_4096": rof_c2_4096, "emd_c2_1024": emd_c2_1024, "paper_protocol_128": paper_protocol_128,
        "emd_ws_512": emd_ws_512, "batch_1024": batch_1024}

if __name__ == "__main__":
    import scipy.fft
    names = sys.argv[1:] or list(JOBS)
    for nm in names:
        t = time.time()
        # threads only split the independent 1-D transforms of the oracle's DCTs
        with scipy.fft.set_workers(int(os.environ.get("ORACLE_FFT_WORKERS", "1"))):
            res = JOBS[nm]()
        res["oracle_seconds"] = round(time.time() - t, 1)
        print(nm, res, flush=True)
        _save(nm, res)
