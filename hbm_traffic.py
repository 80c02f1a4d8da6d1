"""HBM traffic of the step kernels from rocprofv3 counters: the grid pass
(ccpr_step_kernel, both tile variants), the design-voxel kernel
(ccpr_aux_kernel) and the x-CPML post/pre kernel (ccpr_post_fused_kernel).

The counters are calibrated against a plain device copy of known size, run in
the same process: the factor (bytes moved) / (counter reading) of the copy
scales the grid kernel's readings.

Steps (from the repository root; each 'run' under its own counter pass):

  rocprofv3 --pmc FETCH_SIZE --output-format csv -d OUT/fetch -o fetch -- \\
      python3 hbm_traffic.py run
  rocprofv3 --pmc WRITE_SIZE --output-format csv -d OUT/write -o write -- \\
      python3 hbm_traffic.py run
  python3 hbm_traffic.py summarize OUT/fetch OUT/write \\
      profiles/step_kernel_hbm_traffic_gold_gap_320.json

'run' copies a 1 GiB device buffer four times (hipMemcpy device to device),
then runs a 10-step forward solve of the 320^3 gold gap workload.
'summarize' writes the HBM bytes of one grid pass (fetch and write,
calibrated; a pass is one dispatch of each grid-kernel variant), the
calibration factors and the kernel source hash to the JSON file.
"""
from __future__ import annotations

import csv
import glob
import hashlib
import json
import os
import sys

ROOT = os.path.dirname(os.path.abspath(__file__))
COPY_BYTES = 1 << 30
GRID_KERNEL = "ccpr_step_kernel"
# other step kernels reported per dispatch (one dispatch per step each)
OTHER_KERNELS = ("ccpr_aux_kernel", "ccpr_post_fused_kernel")


def run(steps: int = 10) -> None:
    sys.path.insert(0, ROOT)
    import torch
    from paper_2305_00234_amd import inputs as I
    from paper_2305_00234_amd.solver import solver_for

    a = torch.empty(COPY_BYTES // 4, dtype=torch.float32, device="cuda").fill_(1.0)
    b = torch.empty_like(a)
    for _ in range(4):
        b.copy_(a)
    torch.cuda.synchronize()
    del a, b
    w = I.gold_gap_320(steps=steps)
    s = solver_for(w)
    s.forward(steps)
    torch.cuda.synchronize()
    s.close()
    print(f"hbm_traffic run: 4 copies of {COPY_BYTES >> 20} MiB, {steps} forward steps of {w.name}",
          flush=True)


def _per_dispatch(directory: str):
    """{kernel name: [(dispatch id, counter value)]} from a rocprofv3 counter CSV."""
    files = glob.glob(os.path.join(directory, "**", "*counter_collection.csv"), recursive=True)
    if not files:
        raise FileNotFoundError(f"no *counter_collection.csv under {directory}")
    per = {}
    for row in csv.DictReader(open(files[0])):
        key = (row["Kernel_Name"], int(row.get("Dispatch_Id") or row.get("Correlation_Id")))
        per[key] = per.get(key, 0.0) + float(row["Counter_Value"])
    out = {}
    for (name, disp), v in sorted(per.items(), key=lambda kv: kv[0][1]):
        out.setdefault(name, []).append((disp, v))
    return out


def _pick(table, needles, first=None):
    """Counter values of the dispatches of the first kernel whose name contains
    one of needles (the first 'first' dispatches in launch order if given)."""
    for needle in needles:
        names = [n for n in table if needle in n]
        if names:
            rows = sorted((r for n in names for r in table[n]), key=lambda r: r[0])
            if first:
                rows = rows[:first]
            return names[0], [v for _, v in rows]
    raise KeyError(f"no kernel matching {needles}: {sorted(table)[:8]}")


def summarize(fetch_dir: str, write_dir: str, out_json: str) -> dict:
    fetch = _per_dispatch(fetch_dir)
    write = _per_dispatch(write_dir)
    # the calibration copies are the first four copy dispatches of the run
    copy_names = ("copyBuffer", "direct_copy", "copy_kernel", "elementwise")
    copy_name, cf = _pick(fetch, copy_names, first=4)
    _, cw = _pick(write, copy_names, first=4)
    # counters are in KiB per dispatch; calibrate: bytes moved / bytes reported
    f_fac = COPY_BYTES / (sum(cf) / len(cf) * 1024.0)
    w_fac = COPY_BYTES / (sum(cw) / len(cw) * 1024.0)
    # one grid pass = one dispatch of each grid-kernel variant (interior
    # tiles, CPML tiles): sum the variants' per-dispatch averages
    names = sorted(n for n in fetch if GRID_KERNEL in n)
    if not names:
        raise KeyError(f"no {GRID_KERNEL} dispatches")
    per_f = {n: sum(v for _, v in fetch[n]) / len(fetch[n]) for n in names}
    per_w = {n: sum(v for _, v in write[n]) / len(write[n]) for n in names}
    name = " + ".join(names)
    gf = [per_f[n] for n in names]
    gw = [per_w[n] for n in names]
    fetch_b = sum(gf) * 1024.0 * f_fac
    write_b = sum(gw) * 1024.0 * w_fac
    others = {}
    for k in OTHER_KERNELS:
        kn = sorted(n for n in fetch if k in n)
        if not kn:
            continue
        fv = [v for n in kn for _, v in fetch[n]]
        wv = [v for n in kn for _, v in write.get(n, [])]
        others[k] = {
            "dispatches": len(fv),
            "hbm_fetch_bytes_per_dispatch": sum(fv) / len(fv) * 1024.0 * f_fac,
            "hbm_write_bytes_per_dispatch": (sum(wv) / len(wv) * 1024.0 * w_fac) if wv else None,
        }
    src = os.path.join(ROOT, "paper_2305_00234_amd", "csrc", "ccpr_kernels.hip")
    d = {
        "kernel": name,
        "workload": "gold_gap_320 (320^3 cells, 12-cell CPML, 160x160x80 gold design, TF/SF)",
        "dispatches_per_variant": {n: len(fetch[n]) for n in names},
        "fetch_KiB_per_pass_raw": sum(gf),
        "write_KiB_per_pass_raw": sum(gw),
        "copy_kernel": copy_name,
        "copy_bytes_read_and_written": COPY_BYTES,
        "fetch_calibration_factor": f_fac,
        "write_calibration_factor": w_fac,
        "hbm_fetch_bytes_per_launch": fetch_b,
        "hbm_write_bytes_per_launch": write_b,
        "hbm_bytes_per_launch": fetch_b + write_b,  # per grid pass (all variants)
        "other_kernels": others,
        "kernel_source_sha256": hashlib.sha256(open(src, "rb").read()).hexdigest(),
    }
    with open(out_json, "w") as f:
        json.dump(d, f, indent=1)
    return d


if __name__ == "__main__":
    if len(sys.argv) >= 2 and sys.argv[1] == "run":
        run(int(sys.argv[2]) if len(sys.argv) > 2 else 10)
    elif len(sys.argv) == 5 and sys.argv[1] == "summarize":
        print(json.dumps(summarize(sys.argv[2], sys.argv[3], sys.argv[4]), indent=1))
    else:
        print(__doc__)
        sys.exit(2)
