"""Host-side logic that needs no GPU: the rocprofv3 summariser's kernel-name
shortening and its steady-state counter figure."""
from paper_1805_09453_amd import profsum


def test_short_names():
    assert profsum.short("void gp::k_rof_A<4096>(float const*, float*)") == "k_rof_A<4096>"
    assert profsum.short("void gp::k_cols_solve<4096, HIP_vector_type<double, 2u> >(double*, int)") == \
        "k_cols_solve<4096, f64>"
    # kernels in an anonymous namespace, demangled or left mangled by the profiler
    assert profsum.short("void (anonymous namespace)::k_conv<0, 32>((anonymous namespace)::ConvArgs)") == \
        "k_conv<0, 32>"
    assert profsum.short("_ZN12_GLOBAL__N_110k_head_bwdEPKDF16bPKfS3_mPDF16bPfS5_") == "k_head_bwd"


def test_counter_figure_is_the_late_median():
    """Early dispatches (tuner launches in their entry mode, fewer stores) must not
    pull the figure down: the median over the later half of the dispatches is used,
    and the copy calibration is the largest copy dispatch."""
    rows = []
    did = 0
    for v in [70000.0, 69000.0, 90000.0, 71000.0, 209000.0, 208000.0, 210000.0, 77000.0, 209500.0, 208500.0]:
        did += 1
        rows.append({"Kernel_Name": "void gp::k_rof_A<4096>(float const*)", "Counter_Value": str(v),
                     "Dispatch_Id": str(did)})
    for v in [12.0, 262144.0, 40.0]:
        did += 1
        rows.append({"Kernel_Name": "__amd_rocclr_copyBuffer", "Counter_Value": str(v), "Dispatch_Id": str(did)})
    per, copy = profsum.counter_means(rows)
    assert copy == 262144.0
    # later half: 208000, 210000, 77000, 209500, 208500 -> median 208500
    assert per["k_rof_A<4096>"] == 208500.0


def test_training_symmetries():
    """The 16 training symmetries: distinct on a generic pair, reflections are
    involutions, and the density exchange negates the potential."""
    import torch

    from paper_1805_09453_amd.warmstart_train import symmetry
    g = torch.Generator().manual_seed(0)
    a, c, t = (torch.rand((2, 8, 8), generator=g) for _ in range(3))
    seen = set()
    for code in range(16):
        x = symmetry(a, c, t, code)
        seen.add(tuple(round(float(v), 6) for v in torch.cat([y.flatten() for y in x])[:24]))
    assert len(seen) == 16
    for code in (1, 2, 4, 8):
        x = symmetry(*symmetry(a, c, t, code), code)
        assert all(torch.equal(p, q) for p, q in zip(x, (a, c, t)))
    sa, sc, st = symmetry(a, c, t, 8)
    assert torch.equal(sa, c) and torch.equal(sc, a) and torch.equal(st, -t)
