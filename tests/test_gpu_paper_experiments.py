"""The section-4 experiment protocol against the FP64 oracle at 128^2.

The oracle ran the same protocol (tests/golden/make_oracle_references.py,
job paper_protocol_128): F* from a long oracle solve whose gap certifies it to
far below eps/10, each table's step rule evaluated by the oracle, and the
oracle's own iteration count from the zero start until F(u_n) - F* < eps.  The
library's protocol (paper_experiments.py: the device step rule, pd_step and
pd_gap after every iteration) is given that F* and must reach eps at the same
iteration, up to one iteration where FP32 rounding meets the threshold."""
import json
import os

import numpy as np
import pytest

import synth
from conftest import announce
from oracle import emd as oemd
from oracle import grid
from oracle import rof as orof

pytestmark = pytest.mark.gpu
GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "oracle_references.json")


def cases():
    return json.load(open(GOLDEN))["paper_protocol_128"]["cases"]


def dev(a):
    import torch
    return torch.tensor(np.ascontiguousarray(a, dtype=np.float32), device="cuda")


@pytest.mark.parametrize("name", ["rof_lam10_eps0.01", "rof_lam10_eps0.001", "rof_lam20_eps0.01",
                                  "rof_lam20_eps0.001", "rof_lam20_eps0.01_gi"])
def test_rof_disc_protocol_matches_oracle(gpctx, name):
    from paper_1805_09453_amd import paper_experiments as pe
    c = cases()[name]
    assert c["fstar_gap"] <= 0.01 * c["eps"]  # the ground truth is certified (far below eps/10)
    announce(f"paper protocol vs oracle: {name} (128x128)")
    r = pe.rof_case(gpctx, 128, c["lam"], c["eps"], c["grid_independent"], 2 * c["iters"] + 20,
                    ground_truth=(c["fstar"], c["fstar_gap"]))
    print(r, "oracle iters", c["iters"])
    assert r["tau"] == pytest.approx(c["tau"], rel=1e-6)  # device step rule = oracle's rule
    assert r["fstar_certified"]
    assert r["iters"] is not None and abs(r["iters"] - c["iters"]) <= 1


@pytest.mark.parametrize("name", ["emd_discs_eps0.001_table6", "emd_deltas_eps0.01_table7",
                                  "emd_deltas_eps0.01_table8"])
def test_emd_protocol_matches_oracle(gpctx, name):
    from paper_1805_09453_amd import paper_experiments as pe
    c = cases()[name]
    assert c["fstar_gap"] <= 0.1 * c["eps"]
    tau = pe.emd_delta_tau(c["eps"], 128) if c["table"] == 7 else 1.0
    assert tau == pytest.approx(c["tau"], rel=1e-14)
    announce(f"paper protocol vs oracle: {name} (128x128)")
    r = pe.emd_case(gpctx, 128, c["pair"], c["eps"], tau, 2 * c["iters"] + 20,
                    ground_truth=(c["fstar"], c["fstar_gap"]))
    print(r, "oracle iters", c["iters"])
    assert r["fstar_certified"]
    # the translated pairs: the certified grid value lies on or above 1/sqrt(8) (a lower bound on the grid)
    assert r["fstar_minus_continuum"] > -1e-6
    assert r["iters"] is not None and abs(r["iters"] - c["iters"]) <= 1


@pytest.mark.parametrize("n, h, lam, eps, norm", [
    (128, 1.0 / 128, 10.0, 1e-2, grid.ISO), (512, 1.0 / 512, 20.0, 1e-3, grid.ISO),
    (256, 1.0 / 256, 20.0, 1e-3, grid.ANISO), (4096, 1.0, 8.0, 1e-5, grid.ISO)])
def test_rof_step_rule_matches_oracle(gpctx, n, h, lam, eps, norm):
    """rof_step_rule (device FP64 sums) against the oracle's tv_norm, step_rule_tau and
    tv_bound: the disc image at h = 1/n and the 4096^2 noisy scene at h = 1."""
    I = (synth.disc_image(n, 0.25) if n < 4096 else
         synth.rof_scene(n, synth.config_seed(2), n_shapes=50, size_range=(0.02, 0.15)))
    I = np.asarray(I, np.float32).astype(np.float64)
    announce(f"rof_step_rule {n}x{n}, h {h:g}, lambda {lam:g}, eps {eps:g}, norm {norm}")
    r = gpctx.rof_step_rule(dev(I), h, lam, eps, norm=norm)
    tv = orof.tv_norm(I, h, norm)
    gx, gy = grid.grad(I, h)
    gl2 = float(np.sqrt(h * h * np.sum(gx * gx + gy * gy)))
    print(r, tv, gl2)
    assert r["tv"] == pytest.approx(tv, rel=1e-12)
    assert r["grad_l2"] == pytest.approx(gl2, rel=1e-12)
    assert r["tau_continuum"] == pytest.approx(np.sqrt(lam) * tv / np.sqrt(eps), rel=1e-12)
    if norm == grid.ISO:
        assert r["tau"] == pytest.approx(orof.step_rule_tau(I, h, lam, eps), rel=1e-12)
        assert r["tv_bound"] == pytest.approx(orof.tv_bound(I, h, lam), rel=1e-12)


def test_step_rule_rejects_bad_input(gpctx):
    from paper_1805_09453_amd import GPError
    I = np.zeros((64, 64))
    I[3, 5] = np.nan
    with pytest.raises(GPError):
        gpctx.rof_step_rule(dev(I), 1.0, 8.0, 1e-3)
    with pytest.raises(GPError):
        gpctx.rof_step_rule(dev(np.zeros((64, 64))), 1.0, 8.0, 0.0)


def test_emd_rule_is_the_oracles():
    from paper_1805_09453_amd import emd_step_rule_singular
    for eps in (1e-2, 1e-3, 1e-4):
        for n in (512, 1024, 2048, 4096):
            assert emd_step_rule_singular(eps, n) == pytest.approx(oemd.step_rule_tau_singular(eps, n), rel=1e-14)
