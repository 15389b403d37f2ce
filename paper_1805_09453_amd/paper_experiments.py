"""The paper's own experiments (section 4) on the GPU.

    python -m paper_1805_09453_amd.paper_experiments [--sizes 512 1024 2048 4096] [--out results.json]

Workloads (analytic inputs, section 4):
  ROF   indicator of the disc of radius 1/4 centred in [0,1]^2, h = 1/n,
        lambda = 10 and 20, step rule tau = min(sqrt(lambda) |I|_TV / sqrt(eps),
        |grad I|_L2) (section 4.1), and for lambda = 20 also the grid-independent
        tau = sqrt(lambda) |I|_TV / sqrt(eps); sigma = 1/tau;
  EMD   unit-mass uniform discs of radius 1/4 centred at (3/8, 3/8) and
        (5/8, 5/8), tau = sigma = 1 (section 4.2); and unit Dirac masses in the
        cells holding those points, tau = min(sqrt(1/(eps |log eps|)), 2 M^(1/4))
        with M the side length n, and tau = sigma = 1.
Protocol (section 4): from the zero start, iterate until F(u_n) - F* < eps for
the n-th iterate (F evaluated after every iteration).  F* is the primal value
of a long plain solve whose duality gap certifies it to eps/10.  For the EMD
pairs (translations by (1/4, 1/4), a whole number of cells) the continuum value
1/sqrt(8) is a lower bound on the grid too (the potential (x + y)/sqrt(2) is
1-Lipschitz for the grid's differences); the grid optimum lies above it (by
~1e-6 for the discs, by more for the Dirac masses, whose flux cannot spread
over both axes), so the certified value is used.
The wall time of each count is measured separately by re-running that many
iterations of the fused solver loop (no per-iteration evaluation).

Every iteration and every evaluation runs in libgprox; this module only
schedules calls and compares numbers.
"""
import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import synth  # noqa: E402

EMD_EXACT = 1.0 / math.sqrt(8.0)


def rof_tau_rule(ctx, Id, h, lam, eps, grid_independent=False):
    """Section 4.1 step size in unit-square units, computed by the library
    (rof_step_rule): min(sqrt(lam) |I|_TV / sqrt(eps), |grad I|_L2), or the first
    term alone for the grid-independent choice."""
    r = ctx.rof_step_rule(Id, h, lam, eps)
    return r["tau_continuum"] if grid_independent else r["tau"]


def emd_delta_tau(eps, n):
    """Section 4.2 rule for the Dirac pairs (library: emd_step_rule_singular), M = n."""
    from .api import emd_step_rule_singular
    return emd_step_rule_singular(eps, n)


def _sync():
    import torch
    torch.cuda.synchronize()


def count_to_eps(ctx, st, fstar, eps, max_iter):
    """Iterations until F(u_n) - F* < eps (one pd_step and one pd_gap per iteration);
    None when max_iter is reached first."""
    for it in range(1, max_iter + 1):
        ctx.pd_step(st, 1)
        if ctx.pd_gap(st)["primal"] - fstar < eps:
            return it
    return None


_FSTAR = {}


def rof_ground_truth(ctx, Id, n, lam):
    """F* for the disc at (n, lam): primal value of a plain solve to a relative gap
    of 1e-6 (absolute gap ~1e-6 here, far below eps/10); cached per (n, lam)."""
    from . import Options
    if (n, lam) not in _FSTAR:
        tau = rof_tau_rule(ctx, Id, 1.0 / n, lam, 1e-3)
        _, _, ref = ctx.rof_solve(Id, 1.0 / n, lam, Options(tau=tau, tol=1e-6, max_iter=50000, check_every=50))
        _FSTAR[(n, lam)] = ref
    return _FSTAR[(n, lam)]


def rof_case(ctx, n, lam, eps, grid_independent, max_iter, ground_truth=None):
    """Table 1-3 protocol at side n.  ground_truth: optional (F*, certified gap) from
    elsewhere (the tests pass the FP64 oracle's); by default a long library solve."""
    import torch

    from . import Options
    from ._lib import GP_KIND_ROF
    h = 1.0 / n
    I = synth.disc_image(n, 0.25)
    Id = torch.tensor(I, dtype=torch.float32, device="cuda")
    tau = rof_tau_rule(ctx, Id, h, lam, eps, grid_independent)
    if ground_truth is None:
        ref = rof_ground_truth(ctx, Id, n, lam)
        ground_truth = (ref["primal"], ref["primal"] - ref["dual"])
    fstar, fgap = ground_truth
    certified = fgap <= 0.1 * eps
    st = ctx.make_state(GP_KIND_ROF, Id, h, tau, lam=lam)  # sigma = 1/tau
    it = count_to_eps(ctx, st, fstar, eps, max_iter)
    secs = None
    if it:
        _sync()
        t0 = time.perf_counter()
        ctx.rof_solve(Id, h, lam, Options(tau=tau, tol=0.0, max_iter=it, check_every=it))
        _sync()
        secs = time.perf_counter() - t0
    return {"n": n, "lambda": lam, "eps": eps, "tau": tau, "grid_independent_tau": grid_independent,
            "fstar": fstar, "fstar_gap": fgap, "fstar_certified": bool(certified), "iters": it, "seconds": secs}


def emd_ground_truth(ctx, R0, R1, n, kind):
    """F* for an EMD pair: primal value of a plain solve to a relative gap of
    2e-5 (absolute ~7e-6 < 1e-4 / 10); cached per (n, pair)."""
    from . import Options
    if (n, kind) not in _FSTAR:
        tau = 1.0 if kind == "discs" else emd_delta_tau(1e-3, n)
        _, _, ref = ctx.emd_solve(R0, R1, 1.0 / n, Options(tau=tau, tol=2e-5, max_iter=200000, check_every=100),
                                  want_phi=False)
        _FSTAR[(n, kind)] = ref
    return _FSTAR[(n, kind)]


def emd_case(ctx, n, kind, eps, tau, max_iter, ground_truth=None):
    """Table 6-8 protocol at side n (kind "discs" or "deltas").  ground_truth:
    optional (F*, certified gap) from elsewhere; by default a long library solve."""
    import torch

    from . import Options
    from ._lib import GP_KIND_EMD
    h = 1.0 / n
    r0, r1 = synth.uniform_disc_pair(n) if kind == "discs" else synth.delta_pair(n)
    R0 = torch.tensor(r0, dtype=torch.float32, device="cuda")
    R1 = torch.tensor(r1, dtype=torch.float32, device="cuda")
    if ground_truth is None:
        ref = emd_ground_truth(ctx, R0, R1, n, kind)  # (also tunes the launch shapes outside the timings)
        ground_truth = (ref["primal"], ref["primal"] - ref["dual"])
    fstar, fgap = ground_truth
    certified = fgap <= 0.1 * eps
    f, gpsi = ctx.emd_setup(R0, R1, h)
    st = ctx.make_state(GP_KIND_EMD, f, h, tau, gpsi=gpsi)  # sigma = 1/tau
    it = count_to_eps(ctx, st, fstar, eps, max_iter)
    secs = None
    if it:
        _sync()
        t0 = time.perf_counter()
        ctx.emd_solve(R0, R1, h, Options(tau=tau, tol=0.0, max_iter=it, check_every=it), want_phi=False)
        _sync()
        secs = time.perf_counter() - t0
    return {"n": n, "pair": kind, "eps": eps, "tau": tau, "fstar": fstar, "fstar_gap": fgap,
            "fstar_certified": bool(certified), "fstar_minus_continuum": fstar - EMD_EXACT, "iters": it,
            "seconds": secs}


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--sizes", type=int, nargs="+", default=[512, 1024, 2048, 4096])
    ap.add_argument("--max-iter", type=int, default=5000)
    ap.add_argument("--out")
    a = ap.parse_args(argv)
    from . import Context
    ctx = Context(max(a.sizes), max(a.sizes))
    rows = []

    def log(r):
        rows.append(r)
        print(json.dumps(r), flush=True)

    for n in a.sizes:
        for lam, gi in ((10.0, False), (20.0, False), (20.0, True)):
            for eps in (1e-2, 1e-3):
                log(dict(rof_case(ctx, n, lam, eps, gi, a.max_iter), table={(10.0, False): 1, (20.0, False): 2,
                                                                              (20.0, True): 3}[(lam, gi)]))
        for eps in (1e-3, 1e-4):
            log(dict(emd_case(ctx, n, "discs", eps, 1.0, a.max_iter), table=6))
        for eps in (1e-2, 1e-3, 1e-4):
            log(dict(emd_case(ctx, n, "deltas", eps, emd_delta_tau(eps, n), a.max_iter), table=7))
        for eps in (1e-2, 1e-3):
            log(dict(emd_case(ctx, n, "deltas", eps, 1.0, a.max_iter), table=8))
    ctx.close()
    if a.out:
        with open(a.out, "w") as fh:
            json.dump(rows, fh, indent=1)


if __name__ == "__main__":
    main()
