"""CPU checks of the C ABI: the library builds/loads, exports every function
include/gprox.h declares, and rejects bad arguments before touching a GPU."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "gprox.h")


@pytest.fixture(scope="module")
def lib():
    from paper_1805_09453_amd import build as B
    if not os.path.exists(B.LIB):
        B.build()
    from paper_1805_09453_amd import _lib
    return _lib.load()


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?(?:long\s+long|\w+)\**\s+\**(\w+)\s*\(", src, flags=re.M)
    return sorted(set(names))


def test_header_declares_the_entry_points():
    names = declared_functions()
    for required in ("gp_create", "gp_destroy", "dct_poisson", "rof_solve", "emd_solve", "pd_step", "pd_gap",
                     "gp_strerror"):
        assert required in names


def test_library_exports_every_declared_symbol(lib):
    for name in declared_functions():
        assert hasattr(lib, name), f"libgprox.so does not export {name}"


def test_python_binding_covers_every_symbol():
    from paper_1805_09453_amd import _lib
    assert set(declared_functions()) == set(_lib._SIGS)


def test_strerror_and_null_arguments(lib):
    assert lib.gp_strerror(0) == b"ok"
    assert b"invalid" in lib.gp_strerror(-1)
    assert lib.gp_strerror(12345) == b"unknown error code"
    # NULL out-pointer and NULL contexts are rejected on the host
    assert lib.gp_create(None, 64, 64, None) == -1
    assert lib.gp_destroy(None) == 0
    assert lib.dct_poisson(None, None, None, 64, 64, 1.0, 0.0) == -1
    assert lib.pd_step(None, None, 1) == -1
    assert lib.pd_gap(None, None, None) == -1
    assert lib.rof_solve(None, None, None, None, 64, 64, 1.0, 8.0, None, None) == -1
    assert lib.dct_poisson3(None, None, None, 64, 64, 64, 1.0, 0.0) == -1
    assert lib.dct_poisson3_f64(None, None, None, 64, 64, 64, 1.0, 0.0) == -1
    assert lib.rof3_solve(None, None, None, None, 64, 64, 64, 1.0, 8.0, None, None) == -1
    assert lib.emd3_solve(None, None, None, None, None, 64, 64, 64, 1.0, None, None) == -1
    assert lib.gp_get_radix_plan(None, 0, 720, None, None) == -1
    assert lib.gp_set_radix_plan(None, 0, 720, None, 0) == -1
    assert lib.ws_train_step(None, None, None, None, None, 1, 1.0, 1e-3, None) == -1
    assert lib.ws_load_params(None, None, b"weights.f32") == -1
    assert lib.ws_save_params(None, None, b"weights.f32") == -1


def test_warm_start_blob_size_matches_the_oracle_network(lib):
    from oracle import unet
    assert lib.ws_param_count() == unet.n_params() == 1925313
    assert lib.ws_create(None, None, 1, 64, 64) == -1
    assert lib.ws_destroy(None) == 0
    assert lib.ws_emd_solve(None, None, None, None, None, None, 64, 64, 1.0, None, None, None) == -1
    assert lib.gp_batch_solve(None, None, 1, None, None) == -1


def test_unsupported_sizes_rejected_before_allocation(lib):
    h = ctypes.c_void_p()
    assert lib.gp_create(ctypes.byref(h), 110, 64, None) == -5  # 110 = 2 * 5 * 11
    assert lib.gp_create(ctypes.byref(h), 64, 8192, None) == -5
    assert not h.value


def test_python_layer_refuses_without_gpu():
    import torch
    if torch.cuda.is_available():
        pytest.skip("GPU present")
    from paper_1805_09453_amd import Context, GPError
    with pytest.raises(GPError):
        Context(64, 64)


def test_product_path_is_independent_of_the_oracle():
    """The package (binding, build, experiment and training drivers, HIP sources)
    neither imports nor includes anything from oracle/, and importing it in a
    fresh interpreter loads no oracle module: every solve runs in the HIP
    library, so the GPU parity tests compare two independent implementations."""
    import subprocess
    import sys
    pkg = os.path.join(ROOT, "paper_1805_09453_amd")
    pat = re.compile(r"^\s*(?:from\s+oracle\b|import\s+oracle\b|#\s*include\s*[<\"][^>\"]*oracle)", re.M)
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".hip", ".hpp", ".inc", ".h")):
                path = os.path.join(dirpath, f)
                assert not pat.search(open(path).read()), f"{path} reaches into oracle/"
    code = ("import sys; sys.path.insert(0, %r); import paper_1805_09453_amd, paper_1805_09453_amd.api; "
            "print(sorted(m for m in sys.modules if m == 'oracle' or m.startswith('oracle.')))" % ROOT)
    out = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, timeout=300)
    assert out.returncode == 0, out.stderr
    assert out.stdout.strip().splitlines()[-1] == "[]"


def test_singular_emd_rule_is_the_oracles(lib):
    """Host arithmetic of emd_step_rule_singular (section 4.2) against the pinned
    oracle helper, and its argument checks."""
    from oracle import emd
    for eps in (1e-2, 1e-3, 1e-4, 0.5):
        for m in (16, 128, 512, 4096):
            assert lib.emd_step_rule_singular(eps, m) == pytest.approx(emd.step_rule_tau_singular(eps, m),
                                                                       rel=1e-14)
    for eps, m in ((0.0, 64), (1.0, 64), (-1e-3, 64), (1e-3, 0.0)):
        assert lib.emd_step_rule_singular(eps, m) == -1.0
    assert lib.rof_step_rule(None, None, 64, 64, 1.0, 8.0, 1e-3, 0, None) == -1
