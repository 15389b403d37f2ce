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
from oracle import emd, rof  # noqa: E402

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


JOBS = {"rof_c0": rof_c0, "emd_c1_mixture": emd_c1_mixture, "emd_aniso_64": emd_aniso_64}

if __name__ == "__main__":
    names = sys.argv[1:] or list(JOBS)
    data = json.load(open(OUT)) if os.path.exists(OUT) else {}
    for nm in names:
        t = time.time()
        data[nm] = JOBS[nm]()
        data[nm]["oracle_seconds"] = round(time.time() - t, 1)
        print(nm, data[nm], flush=True)
        with open(OUT, "w") as fh:
            json.dump(data, fh, indent=2)
