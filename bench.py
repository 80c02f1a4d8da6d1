#!/usr/bin/env python3
"""Benchmark: one step = one whole forward + adjoint + gradient solve of the
paper-shaped gap problem (320^3 cells, 12-cell CPML, 160x160x80 design of
Table-1 gold with 3 CCPR pole pairs, TF/SF plane wave, 6000 leapfrog steps,
DFT |E|^2 over a 4^3 gap, time-exact gradient), inputs resident in HBM.

Prints one JSON line.  value = cell-updates of the forward and adjoint runs
(cells x 2 x 6000 per solve) per second, in millions.  The roofline object is
for the grid pass (ccpr_step_kernel, the kernel that streams every cell; one
or two concurrent launches): the byte model's bytes per pass (grid_model_bytes)
over its average duration, timed with HIP events on the library's streams
around the grid launches inside the timed region (every 10th pass by
default, --timing-every); "step" gives the same for whole leapfrog steps
with the model's bytes of a step (step_model_bytes).  The byte model counts
what the method must move, not what this implementation's kernel split adds
(the E drive hand-over between kernels, the x-layer re-reads).
roofline.copy_GBs is the measured rate of a plain 1 GiB device copy (bytes
read + written per second, the practical HBM ceiling) and frac_of_copy the
grid pass's share of it.  "serving" is the continuous-batching engine on a
Poisson trace of solve requests (--serving-requests, 0 to skip) against the
same solves one after another.  The CPU baseline is the FP64 oracle on a
bounded sample of the same workload (a few forward + adjoint steps on the
full grid).
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "Mcell-updates/s fwd+adjoint (% HBM roofline) vs plain; p50/p99 solve latency"
HBM_PEAK_GBS = 8000.0


def workload_by_name(name, solve_steps=None):
    from paper_2305_00234_amd import inputs as I
    table = {
        "gold_gap_320": lambda m: I.gold_gap_320(steps=m or 6000),
        "drude_dipole_32": lambda m: I.drude_dipole_32(steps=m or 400),
        "gold_gap_td_512x512x256": lambda m: I.gold_gap_timedomain_512(steps=m or 8000),
        "aniso_two_material_384": lambda m: I.aniso_two_material_384(steps=m or 8000),
        "paper_broadband_gold": lambda m: I.paper_broadband("gold", steps=m or 18000),
    }
    return table[name](solve_steps)


def grid_model_bytes(w):
    """Byte model of one grid pass (one leapfrog step of every cell, with
    perfect halo reuse): 48 B per cell (E and H, three FP32 components each,
    read once and written once) and 32 B per (cell, y or z CPML layer) for the
    two psi memories of H (read old, write new) and of E (read, write).  The
    x CPML, the design pole currents and the gradient history are moved by the
    other kernels of the step and are counted in step_model_bytes."""
    nx, ny, nz = w.shape
    n = nx * ny * nz
    p = w.npml
    yz_layer_cells = 2 * p * nx * nz + 2 * p * nx * ny if p else 0
    return 48 * n + 32 * yz_layer_cells


def design_update_bytes(w):
    """Bytes of the design cells' CCPR update per step, averaged over a
    forward and an adjoint step: per design voxel 16 B per pole pair and
    component (complex J, read + write) and 4 B of density (12 B per cell for
    a per-edge design), and the gradient record's 28 B (time-exact) or 48 B
    (DFT mode).  Part of step_model_bytes; counted in the grid pass when the
    grid pass runs the design update itself."""
    nd = design_box_cells(w)
    per_cell = 3 if w.rho_edges is not None else 1
    pairs = sum(w.mat1[a].npairs + w.mat2[a].npairs for a in range(3))
    record = 48 if w.gradient == "dft" else 28
    return (16 * pairs + 4 * per_cell + record) * nd


def design_box_cells(w):
    """Cells the design kernels run over: the design voxels, or for a per-edge
    design the box of N + 1 cells per axis that holds every design edge."""
    d = w.design_dims
    if w.rho_edges is not None:
        return int((d[0] + 1) * (d[1] + 1) * (d[2] + 1))
    return int(np.prod(d))


def step_model_bytes(w):
    """Byte model of a whole leapfrog step, averaged over a forward and an
    adjoint step (what the method must move, with perfect reuse inside the
    step): 48 B per cell; 32 B per (cell, CPML layer) on each of the three
    axes (psi of H and of E, read + write); per design voxel 16 B per pole pair
    and component (complex J read + write, FP32) and 4 B of density (12 B per
    cell for a per-edge design); the gradient record: time-exact 24 B per
    design voxel written in the forward step and 24 + 8 B read (history and
    gradient accumulator) in the adjoint step, 28 B on average; DFT-mode
    gradient 48 B per design voxel (the running transforms, read + write).
    The history model stores E and the pole term per component; this
    implementation stores one FP32 factor per component (12 B), below the
    model."""
    nx, ny, nz = w.shape
    p = w.npml
    layer_cells = 2 * p * (ny * nz + nx * nz + nx * ny) if p else 0
    return 48 * nx * ny * nz + 32 * layer_cells + design_update_bytes(w)


def traffic_from_profile(kernel_src_hash, workload):
    """HBM bytes per launch from committed rocprofv3 counter summaries, if they
    were taken on the current kernel source and this workload; else None."""
    path = os.path.join(ROOT, "profiles", f"step_kernel_hbm_traffic_{workload}.json")
    if not os.path.exists(path):
        return None
    try:
        d = json.load(open(path))
    except Exception:
        return None
    if d.get("kernel_source_sha256") != kernel_src_hash:
        return None
    return d.get("hbm_bytes_per_launch")


def kernel_hash():
    src = os.path.join(ROOT, "paper_2305_00234_amd", "csrc", "ccpr_kernels.hip")
    return hashlib.sha256(open(src, "rb").read()).hexdigest()


def cpu_model():
    """Host CPU model name (from /proc/cpuinfo), or None."""
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def cpu_baseline(w, sample_steps):
    """FP64 oracle, as it stands, on the full grid of the same workload for
    sample_steps forward + sample_steps adjoint steps."""
    from oracle import build as obuild
    from oracle.oracle import OBJ_DFT, OBJ_TIME, num_threads
    if not os.path.exists(obuild.LIB):
        obuild.build()
    from tests.oracle_setup import oracle_from_workload
    o = oracle_from_workload(w)
    kind = OBJ_DFT if w.objective == "dft" else OBJ_TIME
    t0 = time.perf_counter()
    o.gradient(sample_steps, kind, w.gap_lo, w.gap_dims, w.omega, w.window[0], sample_steps + 1)
    dt = time.perf_counter() - t0
    o.close()
    upd = w.cells * 2 * sample_steps
    return {"value": upd / dt / 1e6, "unit": "Mcell-updates/s", "cores": num_threads(),
            "kind": "oracle", "cpu_model": cpu_model(),
            "sample": f"{w.name}: full {w.shape[0]}x{w.shape[1]}x{w.shape[2]} grid, "
                      f"{sample_steps} forward + {sample_steps} adjoint FP64 steps incl. "
                      f"objective and gradient ({dt:.1f} s wall)"}


def serving(args, n_requests=None, emit=True, sides=(64, 192), rate=None):
    """Serving trace (Poisson arrivals, uneven grids and pole counts): the
    engine's continuous batching (batched launches per padded x width)
    against the same engine with every solve on its own streams and against
    the same solves run one after another with the plain path; same results
    bitwise, solves/s and p50/p99 latency (arrival to result) for each."""
    import torch
    from paper_2305_00234_amd import inputs as I
    from paper_2305_00234_amd.lib import JOB_DONE, JOB_FAILED, Engine
    from paper_2305_00234_amd.solver import configure

    rate = rate or args.rate
    trace = I.serving_trace(n_requests=n_requests or args.serving, rate=rate, seed=3, side_range=sides)
    arrivals = np.array([r.arrival for r in trace]) - trace[0].arrival

    def progress(msg):
        print(f"[serving] {msg}", file=sys.stderr, flush=True)

    # sequential plain solves (one at a time, back to back)
    seq_F, service = [], []
    for k, r in enumerate(trace):
        w = r.workload
        s = configure(w)
        s.bind_torch(w.steps)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        F = s.forward(w.steps)
        s.adjoint()
        s.gradient()
        torch.cuda.synchronize()
        service.append(time.perf_counter() - t0)
        seq_F.append(F)
        s.close()
        del s
        torch.cuda.empty_cache()
    progress(f"sequential: {len(trace)} solves, {sum(service):.2f} s of service")
    seq_done, t = [], 0.0
    for a, d in zip(arrivals, service):
        t = max(t, a) + d
        seq_done.append(t)
    seq_lat = np.array(seq_done) - arrivals

    def engine_run(batching):
        # continuous batching: submit at the arrival times
        solvers = [configure(r.workload) for r in trace]
        eng = Engine(args.arena_gb << 30, max_active=args.max_active, chunk_steps=args.chunk,
                     batching=batching)
        tickets = []
        t0 = time.perf_counter()
        k = 0
        done_t = {}
        while len(done_t) < len(trace):
            now = time.perf_counter() - t0
            while k < len(trace) and arrivals[k] <= now:
                tickets.append(eng.submit(solvers[k], trace[k].workload.steps))
                k += 1
            for q, tk in enumerate(tickets):
                if q not in done_t:
                    st = eng.poll(tk)
                    if st == JOB_FAILED:
                        raise RuntimeError(f"served solve {q} failed")
                    if st == JOB_DONE:
                        done_t[q] = time.perf_counter() - t0
            time.sleep(0.0005)
        wall = max(done_t.values())
        lat = np.array([done_t[q] for q in range(len(trace))]) - arrivals
        same = True
        for q, tk in enumerate(tickets):
            F, _, _ = eng.result(tk)
            same &= F == seq_F[q]
            eng.release(tk)
        eng.close()
        for s in solvers:
            s.close()
        torch.cuda.empty_cache()
        progress(f"engine (batching {batching}): wall {wall:.2f} s, results identical: {same}")
        return wall, lat, same

    wall, bat_lat, same = engine_run(True)
    wall_s, str_lat, same_s = engine_run(False)
    seq_wall = seq_done[-1]
    out = {
        "metric": "served solves/s (continuous batching) vs sequential plain solves; p50/p99 latency",
        "value": round(len(trace) / wall, 3),
        "unit": "solves/s",
        "sequential_solves_per_s": round(len(trace) / seq_wall, 3),
        "speedup": round(seq_wall / wall, 3),
        "latency_ms": {"p50": round(float(np.percentile(bat_lat, 50)) * 1e3, 1),
                       "p99": round(float(np.percentile(bat_lat, 99)) * 1e3, 1)},
        "sequential_latency_ms": {"p50": round(float(np.percentile(seq_lat, 50)) * 1e3, 1),
                                  "p99": round(float(np.percentile(seq_lat, 99)) * 1e3, 1)},
        "per_solve_streams_solves_per_s": round(len(trace) / wall_s, 3),
        "per_solve_streams_latency_ms": {"p50": round(float(np.percentile(str_lat, 50)) * 1e3, 1),
                                         "p99": round(float(np.percentile(str_lat, 99)) * 1e3, 1)},
        "results_identical": bool(same and same_s),
        "n_gpus": 1, "dtype": "f32", "data": "synthetic",
        "config": {"workload": "serving_trace", "requests": len(trace), "rate_per_s": rate,
                   "sides": f"U{{{sides[0]}..{sides[1]}}}", "pole_pairs": "U{1..3}", "steps": "U{1500..4000}",
                   "max_active": args.max_active, "chunk_steps": args.chunk,
                   "arena_GiB": args.arena_gb,
                   "cell_updates": int(sum(2 * r.workload.cells * r.workload.steps for r in trace))},
    }
    if emit:
        print(json.dumps(out), flush=True)
    return out


def other_workload(name):
    """One whole solve (forward + adjoint + gradient, setup included) of another
    configuration, timed by the wall clock, with the step and grid-pass
    durations from HIP events: Mcell-updates/s (the forward and adjoint runs'
    cell updates; recomputed segments count as overhead) and the byte-model
    fractions."""
    import torch
    from paper_2305_00234_amd.solver import solver_for
    w = workload_by_name(name)
    s = solver_for(w)
    grad = torch.empty(s.gradient_size, dtype=torch.float64, device="cuda")
    s.set_timing(True, every=10)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    s.forward(w.steps)
    s.adjoint()
    s.gradient(out=grad)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    step_ms, steps = s.timing()
    grid_ms, passes = s.grid_timing()
    info = s.info()
    s.close()
    del s, grad
    torch.cuda.empty_cache()
    step_s = step_ms / 1e3 / max(steps, 1)
    pass_s = grid_ms / 1e3 / max(passes, 1)
    return {"workload": w.name, "grid": list(w.shape), "leapfrog_steps_per_solve": w.steps,
            "objective": w.objective, "solve_s": round(wall, 3),
            "value": round(w.cells * 2 * w.steps / wall / 1e6, 1), "unit": "Mcell-updates/s",
            "segments": info["segments"], "resident_segments": info["resident_segments"],
            "avg_step_us": round(step_s * 1e6, 2),
            "step_frac": round(step_model_bytes(w) / step_s / 1e9 / HBM_PEAK_GBS, 4),
            "grid_pass_us": round(pass_s * 1e6, 2),
            "design_update_in_grid_pass": bool(info.get("design_fused")),
            "grid_frac": round((grid_model_bytes(w) + (design_update_bytes(w) if info.get("design_fused") else 0))
                               / pass_s / 1e9 / HBM_PEAK_GBS, 4)}


def copy_rate_gbs(nbytes=1 << 30, reps=10):
    """Measured HBM ceiling: bytes read + written per second by a plain
    device-to-device copy of 1 GiB on torch's current stream (HIP events on
    that stream).  None if the memory is not there."""
    import torch
    try:
        src = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
        dst = torch.empty_like(src)
    except torch.cuda.OutOfMemoryError:
        return None
    dst.copy_(src)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        dst.copy_(src)
    e1.record()
    e1.synchronize()
    ms = e0.elapsed_time(e1) / reps
    del src, dst
    torch.cuda.empty_cache()
    return 2 * nbytes / (ms * 1e-3) / 1e9


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="gold_gap_320")
    ap.add_argument("--solve-steps", type=int, default=None,
                    help="leapfrog steps per solve (default: the workload's)")
    ap.add_argument("--tile-planes", type=int, default=None)
    ap.add_argument("--tile-rows", type=int, default=None)
    ap.add_argument("--per-edge", action="store_true",
                    help="one density per E edge (seeded uniform) instead of per voxel")
    ap.add_argument("--gradient", choices=["time", "dft"], default="time",
                    help="time: exact discrete gradient (default); dft: single-frequency estimator")
    ap.add_argument("--cpu-sample-steps", type=int, default=10,
                    help="forward + adjoint steps of the oracle sample (about 10 s on 16 cores at 320^3)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--design-fusion", action="store_true",
                    help="run the design cells' update inside the grid pass where the "
                         "library can (default: the separate design pass)")
    ap.add_argument("--timing-every", type=int, default=10,
                    help="time every k-th grid pass with HIP events (fewer events in the stream)")
    ap.add_argument("--serving", type=int, default=0,
                    help="run only the serving trace, with this many requests")
    ap.add_argument("--serving-requests", type=int, default=24,
                    help="requests of the serving record in the default run (0: skip it)")
    ap.add_argument("--other-workloads",
                    default="gold_gap_td_512x512x256,aniso_two_material_384,paper_broadband_gold",
                    help="comma-separated configurations solved once each after the timed region ('' to skip)")
    ap.add_argument("--serving-small-requests", type=int, default=48,
                    help="requests of the small-grid serving record (sides U{24..64}, 200 requests/s; 0: skip)")
    ap.add_argument("--rate", type=float, default=20.0)
    ap.add_argument("--max-active", type=int, default=8)
    ap.add_argument("--chunk", type=int, default=32)
    ap.add_argument("--arena-gb", type=int, default=96)
    args = ap.parse_args()

    if args.gpus != 1:
        print(f"bench.py measures one GPU (asked for {args.gpus}): the library runs a solve on "
              "one GPU and has no multi-GPU path.", file=sys.stderr)
        sys.exit(2)

    import torch
    if not torch.cuda.is_available():
        print("bench.py needs a ROCm GPU", file=sys.stderr)
        sys.exit(1)
    if args.serving:
        serving(args)
        return
    from paper_2305_00234_amd.solver import solver_for

    w = workload_by_name(args.workload, args.solve_steps)
    w.gradient = args.gradient
    if args.per_edge:
        from paper_2305_00234_amd import inputs as I
        w.rho_edges = I.random_edge_densities(w.design_dims, seed=7)
        w.name += "_edges"
    M = w.steps
    s = solver_for(w)
    if args.tile_planes:
        s.set_tile_planes(args.tile_planes)
    if args.tile_rows:
        s.set_tile_rows(args.tile_rows)
    if args.design_fusion:
        s.set_design_fusion(True)
    grad = torch.empty(s.gradient_size, dtype=torch.float64, device="cuda")

    def one_solve():
        F = s.forward(M)
        s.adjoint()
        s.gradient(out=grad)
        return F

    def progress(msg):
        print(f"[bench] {msg}", file=sys.stderr, flush=True)

    progress(f"{w.name}: {w.shape} cells, {M} steps per solve, {args.warmup} warmup + {args.steps} timed")
    for q in range(args.warmup):
        one_solve()
        torch.cuda.synchronize()
        progress(f"warmup solve {q + 1} done")

    s.set_timing(True, every=args.timing_every)
    lat = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    F = None
    for _ in range(args.steps):
        a = time.perf_counter()
        F = one_solve()
        torch.cuda.synchronize()
        lat.append(time.perf_counter() - a)
        progress(f"timed solve {len(lat)} done: {lat[-1]:.2f} s")
    torch.cuda.synchronize()
    total = time.perf_counter() - t0
    step_ms, launches = s.timing()
    grid_ms, grid_launches = s.grid_timing()
    s.set_timing(False)
    info = s.info()

    ms_per_step = total / args.steps * 1e3
    updates = w.cells * 2 * M
    value = updates / (total / args.steps) / 1e6
    avg_step_s = step_ms / 1e3 / max(launches, 1)
    avg_launch_s = grid_ms / 1e3 / max(grid_launches, 1)
    # with the design update inside the grid pass its bytes belong to the pass
    fused = bool(info.get("design_fused"))
    alg = grid_model_bytes(w) + (design_update_bytes(w) if fused else 0)
    achieved = alg / avg_launch_s / 1e9
    sb = step_model_bytes(w)
    traffic = traffic_from_profile(kernel_hash(), w.name)
    copy_gbs = copy_rate_gbs()

    out = {
        "metric": METRIC,
        "value": round(value, 1),
        "unit": "Mcell-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 2),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": w.name, "cells": w.cells, "grid": list(w.shape),
                   "leapfrog_steps_per_solve": M, "design": list(w.design_dims),
                   "pole_pairs_per_axis": w.max_pairs(), "cpml": w.npml,
                   "source": w.source, "objective": w.objective,
                   "gradient": "time-exact" if w.gradient == "time" else "dft",
                   "design_variables": "per-edge" if w.rho_edges is not None else "per-voxel",
                   "history_segments": info["segments"], "tile_planes": info["tile_planes"]},
        "latency_ms": {"p50": round(float(np.percentile(lat, 50)) * 1e3, 2),
                       "p99": round(float(np.percentile(lat, 99)) * 1e3, 2)},
        "objective": F,
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                     "traffic": traffic,
                     "kernel": "ccpr_step_kernel + ccpr_step_des_kernel" if fused else "ccpr_step_kernel",
                     "design_update_in_grid_pass": fused,
                     "grid_model_bytes": int(alg),
                     "avg_launch_us": round(avg_launch_s * 1e6, 2), "launches": grid_launches,
                     "copy_GBs": round(copy_gbs, 1) if copy_gbs else None,
                     "frac_of_copy": round(achieved / copy_gbs, 4) if copy_gbs else None},
        "step": {"avg_step_us": round(avg_step_s * 1e6, 2), "step_model_bytes": int(sb),
                 "achieved_GBs": round(sb / avg_step_s / 1e9, 1),
                 "frac": round(sb / avg_step_s / 1e9 / HBM_PEAK_GBS, 4), "steps": launches},
    }
    if args.serving_requests > 0 or args.serving_small_requests > 0 or args.other_workloads:
        s.close()
        del s, grad
        torch.cuda.empty_cache()
    if args.other_workloads:
        out["other_workloads"] = []
        for name in args.other_workloads.split(","):
            progress(f"one solve of {name}")
            out["other_workloads"].append(other_workload(name))
    if args.serving_requests > 0:
        progress(f"serving trace ({args.serving_requests} requests)")
        sv = serving(args, n_requests=args.serving_requests, emit=False)
        out["serving"] = {k: sv[k] for k in ("value", "unit", "sequential_solves_per_s", "speedup",
                                             "per_solve_streams_solves_per_s", "latency_ms",
                                             "sequential_latency_ms", "per_solve_streams_latency_ms",
                                             "results_identical")}
        out["serving"]["config"] = sv["config"]
    if args.serving_small_requests > 0:
        progress(f"small-grid serving trace ({args.serving_small_requests} requests)")
        sv = serving(args, n_requests=args.serving_small_requests, emit=False, sides=(24, 64), rate=200.0)
        out["serving_small"] = {k: sv[k] for k in ("value", "sequential_solves_per_s", "speedup",
                                                   "per_solve_streams_solves_per_s", "latency_ms",
                                                   "sequential_latency_ms", "results_identical")}
        out["serving_small"]["config"] = sv["config"]
    if not args.no_cpu_baseline:
        progress("cpu baseline (FP64 oracle sample)")
        out["cpu_baseline"] = cpu_baseline(w, args.cpu_sample_steps)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
