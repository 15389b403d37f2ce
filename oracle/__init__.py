"""FP64 CPU oracle for G-prox PDHG (Jacobs, Leger, Li, Osher, arXiv 1805.09453).

TEST INFRASTRUCTURE ONLY.  This package is the slow, plain, obviously correct
reference that the GPU library is checked against.  It may be imported only by
the test suite, by the package entry's smoke check and by the benchmark's CPU
baseline leg; the product path never calls it.  It shares no code with the
HIP library: the only common dependency is the ``synth`` input generators.

Contents
--------
grid  : the discrete operators (forward-difference gradient, divergence as its
        negative adjoint, Neumann Laplacian diagonalised by the DCT-II, the
        pointwise projection onto the unit ball) and the screened Poisson solve.
rof   : the ROF functional (section 3.1, eq. for F_lambda), its dual, and the
        G-prox PDHG iteration for it (Algorithm 2 with the updates of 3.1).
emd   : the Beckmann/L1 EMD problem (section 3.2), the Hodge split, the
        G-prox PDHG iteration (updates of 3.2), the primal value and a dual
        certificate.
grid3 : the d = 3 case: operators on nz x ny x nx grids (7-point Laplacian,
        3-D DCT-II), the ROF and EMD iterations, values and certificates.
unet  : the learned warm start's network (a U-Net predicting the dual
        potential), its parameter gradients, loss, Adam step and the
        resolution changes used at 4096^2.  Not part of the paper.

Every function is FP64 NumPy/SciPy; scipy.fft's orthonormal DCT is used as a
library primitive for the Laplace inversion (section 4 and appendix A: the
inversion is done by FFT after even reflection, which is the DCT-II).

Parity status: every function is pinned by a CPU test (tests/test_oracle_*.py)
to something other than itself: adjointness, dense linear solves, BVLS, linear
programs and network flow, closed forms and invariants.  The step-size helpers
(rof.tv_norm, rof.step_rule_tau, rof.tv_bound, emd.step_rule_tau_singular) are
pinned in tests/test_oracle_step_rules.py by values worked out by hand on
images with closed-form differences and by the paper's own statements about
which term of the section 4.2 rule binds on its grids.  The small helpers
(rel_gap, pointwise_norm, dual_norm_max, reflect, the network's ReLU and 1x1
head with their backward passes) are pinned directly in
tests/test_oracle_helpers.py by hand values and finite differences, besides
their coverage through the solvers that call them.  No function here is
"parity unpinned".
"""
from . import grid, rof, emd, unet  # noqa: F401
