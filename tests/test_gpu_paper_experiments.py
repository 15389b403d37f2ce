"""The section-4 experiment protocol on small grids: iterate until
F(u_n) - F* < eps, with F* a gap-certified long solve (ROF disc, EMD pairs,
the latter checked against the continuum value 1/sqrt(8), a lower bound)."""
import math

import pytest

from conftest import announce

pytestmark = pytest.mark.gpu


def test_emd_disc_protocol_reaches_eps_and_brackets_the_closed_form(gpctx):
    from paper_1805_09453_amd import paper_experiments as pe
    announce("paper protocol: EMD uniform discs 128x128, eps 1e-3")
    r = pe.emd_case(gpctx, 128, "discs", 1e-3, 1.0, 2000)
    print(r)
    assert r["iters"] is not None and r["iters"] < 2000
    # the certified grid value lies on or above the continuum one (a lower bound on the grid)
    assert r["fstar_certified"] and -1e-6 <= r["fstar_minus_continuum"] < 1e-3


def test_emd_delta_rule_and_rof_disc_protocol(gpctx):
    from paper_1805_09453_amd import paper_experiments as pe
    tau = pe.emd_delta_tau(1e-2, 128)
    assert abs(tau - min(math.sqrt(1 / (1e-2 * math.log(100))), 2 * 128 ** 0.25)) < 1e-12
    announce("paper protocol: EMD deltas 128x128, eps 1e-2")
    r = pe.emd_case(gpctx, 128, "deltas", 1e-2, tau, 2000)
    print(r)
    assert r["iters"] is not None and r["fstar_certified"] and r["fstar_minus_continuum"] > -1e-6
    announce("paper protocol: ROF disc 128x128, lambda 10, eps 1e-2")
    r = pe.rof_case(gpctx, 128, 10.0, 1e-2, False, 2000)
    print(r)
    assert r["fstar_certified"] and r["iters"] is not None
