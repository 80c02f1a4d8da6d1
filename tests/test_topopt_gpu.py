"""End-to-end topology-optimisation loop on a small gold-gap problem (GPU):
filter, projection, forward and adjoint solves, chain rule and beta
continuation in the library's kernels, host-side ascent step.  Qualitative:
the objective must grow and the design stay in [0, 1]."""
import numpy as np
import pytest

from paper_2305_00234_amd import inputs as I
from tests.gpu_util import require_gpu, say

pytestmark = pytest.mark.gpu


def test_topopt_loop_increases_objective():
    require_gpu()
    from paper_2305_00234_amd.topopt import optimize
    w = I.drude_dipole_32(steps=300, n=32, npml=6)
    w.shape = (30, 27, 33)
    w.mat2 = (I.GOLD_TABLE1,) * 3
    w.design_lo = (10, 9, 11)
    w.rho = np.full((9, 8, 10), 0.5, dtype=np.float32)
    w.dipole_cell = (7, 13, 15)
    w.gap_lo, w.gap_dims = (14, 12, 15), (2, 2, 2)
    rho, hist = optimize(w, iterations=8, radius=1.5, beta0=2.0, beta_every=4, move=0.1)
    for h in hist:
        say("iteration", h.index, "F", h.objective, "beta", h.beta, "M_nd %", round(h.nondiscreteness, 2),
            "max step", round(h.max_step, 3))
    F = [h.objective for h in hist]
    assert np.all(np.isfinite(F)) and F[-1] > 1.05 * F[0]
    assert [h.beta for h in hist] == [2.0] * 4 + [4.0] * 4
    assert rho.min() >= 0.0 and rho.max() <= 1.0


def test_topopt_loop_per_edge_variables():
    """The same loop over one density per E edge (the paper's layout) with
    the staggered-position filter: the objective grows and the design stays
    in [0, 1]."""
    require_gpu()
    from paper_2305_00234_amd.lib import edge_count
    from paper_2305_00234_amd.topopt import optimize
    w = I.drude_dipole_32(steps=300, n=32, npml=6)
    w.shape = (30, 27, 33)
    w.mat2 = (I.GOLD_TABLE1,) * 3
    w.design_lo = (10, 9, 11)
    w.rho = np.full((9, 8, 10), 0.5, dtype=np.float32)
    w.dipole_cell = (7, 13, 15)
    w.gap_lo, w.gap_dims = (14, 12, 15), (2, 2, 2)
    rho, hist = optimize(w, iterations=6, radius=1.5, beta0=2.0, beta_every=3, move=0.1, per_edge=True)
    for h in hist:
        say("edge iteration", h.index, "F", h.objective, "beta", h.beta, "M_nd %", round(h.nondiscreteness, 2))
    F = [h.objective for h in hist]
    assert rho.size == edge_count(w.design_dims)
    assert np.all(np.isfinite(F)) and F[-1] > 1.05 * F[0]
    assert rho.min() >= 0.0 and rho.max() <= 1.0
