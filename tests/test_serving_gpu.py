"""Serving engine (continuous batching) on the GPU: every solve's objective and
gradient are bitwise the same in the mix as alone, solves arriving while
others run are admitted as slots and arena memory free up, several solves are
on the device at once, and a served result meets the oracle bars."""
import time

import numpy as np
import pytest

from paper_2305_00234_amd import inputs as I
from tests.gpu_util import oracle_gradient, rel_l2, require_gpu, say

pytestmark = pytest.mark.gpu

SPECS = [(40, 1, 300), (56, 3, 260), (48, 2, 340), (64, 3, 240), (44, 1, 280), (60, 2, 300)]


def _requests():
    ws = [I.serving_workload(side, p, steps, seed=500 + k) for k, (side, p, steps) in enumerate(SPECS)]
    ws[2].gradient = "dft"  # one request with the DFT-mode gradient in the mix
    ws[4].rho_edges = I.random_edge_densities(ws[4].design_dims, seed=504)  # one per-edge design
    return ws


def _same(g, ga):
    if isinstance(ga, tuple):
        return len(g) == len(ga) and all(np.array_equal(x, y) for x, y in zip(g, ga))
    return np.array_equal(g, ga)


def _alone(w):
    from paper_2305_00234_amd.solver import configure
    s = configure(w)
    s.bind_torch(w.steps)
    F = s.forward(w.steps)
    s.adjoint()
    g = s.gradient()
    s.close()
    return F, g


def test_mix_equals_alone_and_overlaps():
    torch = require_gpu()
    from paper_2305_00234_amd.lib import JOB_DONE, JOB_RUNNING, Engine
    from paper_2305_00234_amd.solver import configure
    ws = _requests()
    alone = [_alone(w) for w in ws]
    torch.cuda.synchronize()
    solvers = [configure(w) for w in ws]
    sizes = [s.workspace_size(w.steps) for s, w in zip(solvers, ws)]
    arena = int(2.5 * max(sizes))  # not every solve fits at once
    say("workspaces MB", [round(b / 2**20, 1) for b in sizes], "arena MB", round(arena / 2**20, 1))
    eng = Engine(arena, max_active=4, chunk_steps=16)
    tickets = [eng.submit(solvers[0], ws[0].steps), eng.submit(solvers[1], ws[1].steps)]
    t0 = time.time()
    while eng.poll(tickets[0]) != JOB_RUNNING and eng.poll(tickets[0]) != JOB_DONE:
        assert time.time() - t0 < 60
        time.sleep(0.001)
    # later arrivals, admitted while the first ones run
    tickets += [eng.submit(s, w.steps) for s, w in zip(solvers[2:], ws[2:])]
    while True:
        states = [eng.poll(t) for t in tickets]
        if all(st == JOB_DONE for st in states):
            break
        assert all(st != 3 for st in states), states
        assert time.time() - t0 < 120
        time.sleep(0.0005)
    spans = []
    for k, (t, (Fa, ga)) in enumerate(zip(tickets, alone)):
        F, g, times = eng.result(t)
        say("request", k, ws[k].name, "F", F, Fa, "submitted/admitted/done", [round(x, 3) for x in times])
        spans.append(times[1:])
        assert F == Fa
        assert _same(g, ga)
        eng.release(t)
    # most solves on the device at once, from the engine's admit/done times
    events = sorted([(a, 1) for a, _ in spans] + [(d, -1) for _, d in spans])
    cur = most = 0
    for _, dlt in events:
        cur += dlt
        most = max(most, cur)
    say("most solves on the device at once", most)
    assert most >= 2
    eng.close()
    for s in solvers:
        s.close()


def test_served_result_meets_oracle_bars():
    require_gpu()
    from paper_2305_00234_amd.lib import Engine
    from paper_2305_00234_amd.solver import configure
    w = I.serving_workload(36, 3, 220, seed=77)
    s = configure(w)
    eng = Engine(2 * s.workspace_size(w.steps), max_active=2, chunk_steps=8)
    t = eng.submit(s, w.steps)
    eng.wait(t)
    F, g, _ = eng.result(t)
    eng.release(t)
    eng.close()
    s.close()
    Fo, go, _, _ = oracle_gradient(w)
    say("served F", F, Fo, "grad rel L2", rel_l2(g, go))
    assert abs(F - Fo) <= 1e-5 * abs(Fo)
    assert rel_l2(g, go) <= 1e-3


def test_submit_rejects_oversized_and_duplicate():
    require_gpu()
    from paper_2305_00234_amd.lib import CcprError, ENOMEM, ESTATE, Engine
    from paper_2305_00234_amd.solver import configure
    w = I.serving_workload(40, 1, 200, seed=5)
    s = configure(w)
    eng = Engine(s.workspace_size(w.steps) // 2, max_active=1)
    with pytest.raises(CcprError) as ei:
        eng.submit(s, w.steps)
    assert ei.value.status == ENOMEM
    eng.close()
    eng = Engine(4 * s.workspace_size(w.steps), max_active=1)
    t = eng.submit(s, w.steps)
    with pytest.raises(CcprError) as ei:
        eng.submit(s, w.steps)
    assert ei.value.status == ESTATE
    eng.wait(t)
    eng.release(t)
    eng.close()
    s.close()


def _small_mix():
    """Twelve solves of two padded x widths (64 and 128 cells), 1-3 pole
    pairs, 4- or 6-cell CPML, 120-300 steps; two with the time-domain
    objective in 40-step checkpointed segments (one resident: the adjoint
    recomputes the others)."""
    specs = [(24, 1, 160, 4), (28, 2, 200, 4), (32, 3, 240, 6), (36, 1, 120, 4), (40, 2, 300, 6),
             (44, 3, 180, 4), (48, 1, 220, 6), (52, 2, 140, 4), (66, 3, 160, 6), (72, 1, 200, 4),
             (80, 2, 180, 6), (100, 3, 120, 4)]
    ws = []
    for k, (side, p, steps, npml) in enumerate(specs):
        w = I.serving_workload(side, p, steps, seed=900 + k, npml=npml)
        if k in (2, 9):
            w.objective = "time"
            w.checkpoint_every = 40
        ws.append(w)
    return ws


def _serve(ws, batching, max_active=12, chunk=8):
    from paper_2305_00234_amd.lib import JOB_DONE, JOB_FAILED, Engine
    from paper_2305_00234_amd.solver import configure
    solvers = [configure(w) for w in ws]
    arena = sum(s.workspace_size(w.steps) for s, w in zip(solvers, ws)) + (64 << 20)
    eng = Engine(arena, max_active=max_active, chunk_steps=chunk, batching=batching)
    tickets = [eng.submit(s, w.steps) for s, w in zip(solvers, ws)]
    t0 = time.time()
    while True:
        states = [eng.poll(t) for t in tickets]
        assert JOB_FAILED not in states, states
        if all(st == JOB_DONE for st in states):
            break
        assert time.time() - t0 < 120
        time.sleep(0.0005)
    out = []
    for t in tickets:
        F, g, _ = eng.result(t)
        out.append((F, g))
        eng.release(t)
    eng.close()
    for s in solvers:
        s.close()
    return out


def test_batched_small_solves_two_widths_equal_alone():
    """Batched launches (one grid, aux and post launch per step for up to 8
    solves of one padded width; twelve solves need two launches of the
    64-cell class per step) give every solve bitwise the objective and
    gradient it has alone, and the same as the engine with batching off."""
    torch = require_gpu()
    ws = _small_mix()
    alone = [_alone(w) for w in ws]
    torch.cuda.synchronize()
    batched = _serve(ws, batching=True)
    plain = _serve(ws, batching=False)
    for k, ((F, g), (Fb, gb), (Fp, gp)) in enumerate(zip(alone, batched, plain)):
        say("request", k, ws[k].name, ws[k].objective, "F", F, Fb, Fp)
        assert Fb == F and Fp == F
        assert _same(gb, g) and _same(gp, g)


def test_diverging_request_fails_alone():
    """A request whose material is not passive (static susceptibility < 0)
    diverges; the watchdog stops its run and the engine reports that job
    FAILED with the reason, while the requests beside it -- in the same
    batched launches, or on streams of their own -- finish with bitwise the
    results they have alone."""
    import math
    torch = require_gpu()
    from paper_2305_00234_amd.lib import EDEVICE, JOB_DONE, JOB_FAILED, CcprError, Engine
    from paper_2305_00234_amd.solver import configure
    good = [I.serving_workload(side, p, steps, seed=950 + k, npml=npml)
            for k, (side, p, steps, npml) in enumerate([(24, 1, 200, 4), (28, 2, 200, 4),
                                                        (40, 1, 300, 6), (66, 3, 160, 4)])]
    bad = I.drude_dipole_32(steps=2000, n=24, npml=0, gamma=0.0)
    bad.design_lo = (8, 8, 8)
    bad.rho = np.ones((8, 8, 8), np.float32)
    bad.gap_lo, bad.gap_dims = (11, 11, 11), (2, 2, 2)
    bad.dipole_cell = (6, 12, 12)
    bad.mat2 = (I.lorentz(1.0, -3.0, 2 * math.pi * 299792458.0 / 500e-9, 1e13),) * 3
    alone = [_alone(w) for w in good]
    torch.cuda.synchronize()
    for batching in (True, False):
        solvers = [configure(w) for w in good]
        sb = configure(bad)
        sb.set_watchdog(64)
        arena = sum(s.workspace_size(w.steps) for s, w in zip(solvers, good)) + sb.workspace_size(bad.steps)
        eng = Engine(arena + (64 << 20), max_active=8, chunk_steps=16, batching=batching)
        tb = eng.submit(sb, bad.steps)
        tickets = [eng.submit(s, w.steps) for s, w in zip(solvers, good)]
        assert eng.wait(tb) == JOB_FAILED
        with pytest.raises(CcprError) as e:
            eng.result(tb)
        assert e.value.status == EDEVICE and "diverged" in str(e.value)
        for k, t in enumerate(tickets):
            assert eng.wait(t) == JOB_DONE
            F, g, _ = eng.result(t)
            assert F == alone[k][0] and np.array_equal(g, alone[k][1]), (batching, k)
            eng.release(t)
        say("batching", batching, "failed request:", e.value)
        eng.release(tb)
        eng.close()
        for s in solvers + [sb]:
            s.close()
