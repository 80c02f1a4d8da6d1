"""bench.py on the host: the multi-GPU refusal and the byte model of the
roofline (the per-unit figures the benchmark divides by kernel time)."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in (r.stdout + r.stderr)


def test_byte_model_of_the_320_cube_workload():
    """48 B per cell and 32 B per (cell, y/z CPML layer) for the grid pass;
    the whole step adds the x layers, 16 B per pole pair and component and
    4 B of density per design voxel, and a 28 B average of the gradient
    record (24 B written forward, 24 + 8 B read adjoint)."""
    sys.path.insert(0, ROOT)
    import bench
    w = bench.workload_by_name("gold_gap_320", 10)
    n, p = 320, 12
    cells = n ** 3
    yz = 2 * p * n * n * 2
    assert bench.grid_model_bytes(w) == 48 * cells + 32 * yz == 1730150400
    nd = 160 * 160 * 80
    pairs = sum(w.mat1[a].npairs + w.mat2[a].npairs for a in range(3))
    assert pairs == 9
    step = 48 * cells + 32 * (3 * 2 * p * n * n) + (16 * pairs + 4 + 28) * nd
    assert bench.step_model_bytes(w) == step == 2169241600
