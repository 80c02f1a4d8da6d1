"""The allocation-free entry point ccpr_bind_static_workspace (the library's
static 64 MiB device array as workspace) against ccpr_bind_workspace with a
torch-allocated workspace: two solves in a row on the static array, the
second on a smaller grid, each equal bit for bit to the same solve on a
caller workspace (forward fields, objective, gradient); binding a second
solver unbinds the first; a solve whose fixed workspace exceeds the array
is refused with CCPR_ENOMEM."""
import numpy as np
import pytest

from paper_2305_00234_amd import inputs as I
from tests.gpu_util import require_gpu, say

pytestmark = pytest.mark.gpu


def _run(s, w):
    F = s.forward(w.steps)
    fwd = [s.field(c) for c in range(6)]
    s.adjoint()
    g = s.gradient()
    return F, fwd, g


def _pair(w, torch):
    from paper_2305_00234_amd.solver import configure
    ref = configure(w)
    ref.bind_torch(w.steps)
    expect = _run(ref, w)
    ref.close()
    s = configure(w)
    s.bind_static_workspace(torch.cuda.current_stream().cuda_stream)
    got = _run(s, w)
    return s, expect, got


def _same(expect, got):
    F0, f0, g0 = expect
    F1, f1, g1 = got
    assert F1 == F0
    assert all(np.array_equal(a, b) for a, b in zip(f0, f1))
    assert np.array_equal(g1, g0)


def test_static_workspace_two_solves_in_a_row():
    torch = require_gpu()
    from paper_2305_00234_amd import lib as L
    big = I.drude_dipole_32(steps=200)                      # 32^3, 8-cell CPML
    small = I.drude_dipole_32(steps=120, n=24, npml=4)      # smaller grid, fewer steps
    say("static workspace: first solve", big.shape, big.steps)
    s1, e1, g1 = _pair(big, torch)
    _same(e1, g1)
    say("static workspace: second solve (smaller)", small.shape, small.steps)
    s2, e2, g2 = _pair(small, torch)
    _same(e2, g2)
    # the second bind took the array from the first solver
    with pytest.raises(L.CcprError) as e:
        s1.forward(big.steps)
    assert e.value.status == L.ESTATE
    # and the second solver runs again on it, with the same results
    _same(e2, _run(s2, small))
    s1.close()
    s2.close()
    torch.cuda.synchronize()


def test_static_workspace_rejects_a_solve_too_large():
    require_gpu()
    from paper_2305_00234_amd import lib as L
    from paper_2305_00234_amd.solver import configure
    w = I.gold_gap(n=(160, 160, 160), design=(64, 64, 32), steps=10, name="too_large")
    s = configure(w)
    with pytest.raises(L.CcprError) as e:
        s.bind_static_workspace(0)
    say("too large:", e.value)
    assert e.value.status == L.ENOMEM and "static workspace" in str(e.value)
    s.close()
