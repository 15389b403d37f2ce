"""The allocation-free entry point dct_poisson_noalloc against dct_poisson (the
entry point it varies) and the FP64 oracle: two calls in a row, the second on a
smaller grid (the shared workspace keeps the first call's contents), in place
and out of place, and the size limit."""
import numpy as np
import pytest

from conftest import announce, field_err
from oracle import grid

pytestmark = pytest.mark.gpu


def field(ny, nx, seed):
    return np.random.default_rng(seed).standard_normal((ny, nx)).astype(np.float32).astype(np.float64)


@pytest.mark.parametrize("first, second", [((1024, 1024, 1.0, 0.04), (256, 128, 1.0 / 256, 0.0)),
                                           ((256, 4096, 0.5, 0.0), (64, 64, 1.0, 2.0))])
def test_noalloc_matches_dct_poisson_on_two_calls(gpctx, first, second):
    import torch
    from paper_1805_09453_amd import dct_poisson_noalloc
    for k, (ny, nx, h, alpha) in enumerate((first, second)):
        b = field(ny, nx, 100 * k + ny)
        bd = torch.tensor(b, dtype=torch.float32, device="cuda")
        announce(f"dct_poisson_noalloc call {k + 1}: {ny}x{nx} h={h} alpha={alpha}")
        x_na = dct_poisson_noalloc(bd, h=h, alpha=alpha)
        x_ref = gpctx.dct_poisson(bd, h=h, alpha=alpha)
        torch.cuda.synchronize()
        xo = grid.poisson_solve(b, h, alpha)
        e_entry = field_err(x_na.cpu().double().numpy(), x_ref.cpu().double().numpy())
        e_oracle = field_err(x_na.cpu().double().numpy(), xo)
        same = torch.equal(x_na, x_ref)
        print(f"vs dct_poisson {e_entry:.2e} (bit-identical: {same}), vs oracle {e_oracle:.2e}")
        assert e_entry <= 1e-6
        assert e_oracle <= (1e-6 if max(ny, nx) <= 256 else 5e-6)
        # in place gives the same values
        xi = bd.clone()
        dct_poisson_noalloc(xi, x=xi, h=h, alpha=alpha)
        assert torch.equal(xi, x_na)


def test_noalloc_limits_and_errors():
    import torch
    from paper_1805_09453_amd import GPError, _lib, dct_poisson_noalloc
    big = torch.zeros((2048, 1024), dtype=torch.float32, device="cuda")
    announce("dct_poisson_noalloc size limit")
    with pytest.raises(GPError) as e:
        dct_poisson_noalloc(big)
    assert e.value.code == _lib.GP_EUNSUPPORTED and "at most" in str(e.value)
    odd = torch.zeros((96, 64), dtype=torch.float32, device="cuda")
    with pytest.raises(GPError) as e:
        dct_poisson_noalloc(odd)
    assert e.value.code == _lib.GP_EUNSUPPORTED
    ok = torch.zeros((64, 64), dtype=torch.float32, device="cuda")
    with pytest.raises(GPError) as e:
        dct_poisson_noalloc(ok, alpha=-1.0)
    assert e.value.code == _lib.GP_EINVAL
    lib = _lib.load()
    assert lib.dct_poisson_noalloc(None, None, 64, 64, 1.0, 0.0, None) == _lib.GP_EINVAL
    assert b"NULL" in lib.gp_last_error(None)
