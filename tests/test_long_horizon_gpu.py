"""Parity at the configurations' stated step counts, on reduced grids that
keep each configuration's physics (materials, CPML, TF/SF plane wave,
objective, gradient mode, checkpointing): the 320^3 gold gap problem's
6000 steps, the 384^3 anisotropic two-material problem's 8000 steps and the
512x512x256 time-domain problem's 8000 steps with 1000-step checkpoint
segments; and the paper's own problem shape at full size.  GPU (FP32,
through the C-ABI) against the FP64 oracle on the same seeded inputs:
objective, gradient, and the forward field state -- over the whole grid,
inside each region where a local error would be diluted in a whole-grid norm
(design box, gap, CPML slabs, TF/SF shell, far faces, the rest) and as the
largest error of any field word over the state's peak.

Bars: objective relative error <= 1e-5 and gradient relative L2 <= 1e-3 at
the stated horizon.  Field state <= 1e-5 (whole grid, every region holding at
least 1e-4 of the state's norm, max over peak) while the pulse is on the
design (step 1000).  At the stated horizon the pulse has left and the state
has decayed by one to two orders of magnitude, while rounding of FP32
storage leaves a floor that grows with the step count (rounding breaks the
discrete divergence of E and H, so static charge noise accumulates like a
random walk): the oracle itself, with its stored state rounded to FP32 and
its arithmetic in FP64, differs from the FP64 oracle by 5.7e-5 at step 6000
of the gold gap problem (H 6.9e-4, CPML slabs 2.1e-3), so no implementation
with FP32 fields can meet 1e-5 there.  At the stated horizon each error must
therefore be within 2x that FP32-storage floor, measured in the same test
(or within 1e-5, whichever is larger).  The factor is that of FP32
arithmetic on top of FP32 storage: the GPU's vacuum update rounds the curl
difference, its product with the Courant number and the sum as well as the
store, two to three independent roundings where the floor has one, so its
random-walk noise is sqrt(2) to sqrt(3) times the floor's (measured 1.05x
to 1.6x over the regions of the three horizons).
"""
import time

import numpy as np
import pytest

from paper_2305_00234_amd import inputs as I
from tests.gpu_util import (field_errors, fmt_regions, fp32_storage_fields, gpu_fields_after_steps,
                            gpu_gradient, oracle_fields_after_steps, oracle_gradient, region_errors,
                            rel_l2, say)

pytestmark = pytest.mark.gpu

FIELD_TOL = 1e-5
GRAD_TOL = 1e-3
MIN_SHARE = 1e-4
FLOOR_FACTOR = 2.0


def _check_state(tag, g, o, w, floor=None):
    """Whole-grid, per-region and max/peak errors of the GPU state g against
    the FP64 state o; bars 1e-5, or FLOOR_FACTOR x the FP32-storage state
    'floor' where that is larger."""
    st, eE, eH = field_errors(g, o)
    reg = region_errors(g, o, w)
    bar = {"state": FIELD_TOL, "max_abs/peak": FIELD_TOL}
    fl = {}
    if floor is not None:
        fst, _, _ = field_errors(floor, o)
        fl = region_errors(floor, o, w)
        fl["state"] = fst
        bar["state"] = max(FIELD_TOL, FLOOR_FACTOR * fst)
        bar["max_abs/peak"] = max(FIELD_TOL, FLOOR_FACTOR * fl["max_abs/peak"])
    msg = (f"{tag}: state {st:.2e} (E {eE:.2e}, H {eH:.2e}) bar {bar['state']:.2e}; regions: {fmt_regions(reg)}"
           + (f"; FP32-storage floor: state {fl['state']:.2e}, {fmt_regions({k: v for k, v in fl.items() if k != 'state'})}"
              if fl else ""))
    say(msg)
    assert st <= bar["state"], msg
    assert reg["max_abs/peak"] <= bar["max_abs/peak"], msg
    for name, v in reg.items():
        if isinstance(v, tuple) and v[1] >= MIN_SHARE:
            b = FIELD_TOL if not fl else max(FIELD_TOL, FLOOR_FACTOR * fl[name][0])
            assert v[0] <= b, (name, b, msg)


def _check(w, mid=1000, checkpoint_every=None, resident=None):
    t0 = time.time()
    F, g, fwd, _, info = gpu_gradient(w, checkpoint_every=checkpoint_every, resident=resident)
    g_mid = gpu_fields_after_steps(w, mid)
    t1 = time.time()
    Fo, go, fo, _ = oracle_gradient(w)
    o_mid = oracle_fields_after_steps(w, mid)
    f32_mid, f32_end = fp32_storage_fields(w, (mid, w.steps))
    t2 = time.time()
    eF = abs(F - Fo) / abs(Fo)
    eg = rel_l2(g, go)
    gmax = float(np.max(np.abs(np.asarray(g) - go)) / np.max(np.abs(go)))
    msg = (f"{w.name} {w.shape} {w.steps} steps {info}: F rel {eF:.2e}; gradient rel L2 {eg:.2e} "
           f"(max/peak {gmax:.2e}); gpu {t1 - t0:.1f} s, oracle {t2 - t1:.1f} s")
    say(msg)
    assert eF <= FIELD_TOL, msg
    assert eg <= GRAD_TOL, msg
    _check_state(f"{w.name} step {mid}", g_mid, o_mid, w)
    say(f"{w.name} step {mid}: FP32-storage floor state {field_errors(f32_mid, o_mid)[0]:.2e}")
    _check_state(f"{w.name} step {w.steps}", fwd, fo, w, floor=f32_end)
    return info


def test_gold_gap_6000_steps():
    """The 320^3 gold gap workload's physics on 64^3: Table-1 gold (sigma + 3
    pairs) in vacuum, smoothed rho~U[0,1], 4^3 air gap, 12-cell CPML, TF/SF
    x-polarised pulse along +z at 800 nm, DFT objective, time-exact gradient,
    6000 steps."""
    w = I.gold_gap(n=(64, 64, 64), design=(24, 24, 12), gap=4, npml=12, steps=6000, seed=1,
                   name="gold_gap_64_6000")
    _check(w)


def test_anisotropic_two_material_8000_steps():
    """The 384^3 anisotropic workload's physics on 64^3: a Lorentz dielectric
    (rho = 0) and a diagonal-anisotropic metal with a different pole set per
    axis (rho = 1), 4 pole pairs per component, dx = 4 nm, DFT objective,
    8000 steps."""
    w = I.aniso_two_material((64, 64, 64), (24, 24, 12), 8000, npml=12, gap=4,
                             name="aniso_two_material_64_8000")
    _check(w)


def test_time_domain_8000_steps_checkpointed():
    """The 512x512x256 time-domain workload's physics on 64x64x48: Eq. 2 over
    the whole run, 8000 steps in 1000-step segments, three of them resident
    (five recomputed from checkpoints during the adjoint)."""
    w = I.gold_gap(n=(64, 64, 48), design=(24, 24, 8), gap=4, npml=12, steps=8000, seed=2,
                   objective="time", name="gold_gap_td_64x64x48_8000")
    info = _check(w, checkpoint_every=1000, resident=3)
    assert info["segments"] == 8 and info["resident_segments"] == 3


def test_paper_broadband_full_shape():
    """The paper's own problem shape at full size (170 x 95 x 170 cells, the
    100 x 25 x 100 design with its 6 x 25 x 6 air gap, 20-cell CPML, dx =
    2 nm, z-polarised sinc x Hanning plane wave along +y, time-domain
    objective over the whole run), shortened to 600 steps and checkpointed
    in 200-step segments with one resident (two recomputed)."""
    w = I.paper_broadband("gold", steps=600)
    info = _check(w, mid=300, checkpoint_every=200, resident=1)
    assert info["segments"] == 3 and info["resident_segments"] == 1
