"""FP64 numpy oracle of the design filtering and projection (test
infrastructure only: only tests/, the smoke check and the benchmark's
CPU-baseline leg may use this module).

Written from the paper's Sec. "Filtering and projection", on the per-voxel
density grid of the design box (one density per voxel, x fastest, arrays
shaped [nz][ny][nx]; distances in voxel units):

- Eq. FilterFunction: rho_t[n] = sum_m w(n,m) rho[m] / sum_m w(n,m) over the
  design voxels m inside the sphere of radius R around n, with the cone
  weight w = R - |r_m - r_n| (so only |r_m - r_n| < R contributes);
- Eq. Projection: the smoothed Heaviside
  rho_b = (tanh(beta eta) + tanh(beta (rho_t - eta))) /
          (tanh(beta eta) + tanh(beta (1 - eta)));
- Eq. GradientsFiltered: dF/drho[n] = sum_m dF/drho_b[m] drho_b/drho_t[m]
  drho_t[m]/drho[n], with drho_t[m]/drho[n] = w(m,n) / W[m], W[m] the
  weight sum of m;
- Eq. MeasureOfNon-discretness: M_nd = sum 4 rho_b (1 - rho_b) / N x 100 %.

The filter visits the sphere's offsets one at a time and shifts the whole
array (zero outside the design box), which is the definition written out.
"""
from __future__ import annotations

import math

import numpy as np


def sphere_offsets(radius: float):
    """Integer offsets (dz, dy, dx) with |d| < radius and their cone weights
    radius - |d| (all positive)."""
    r = int(math.ceil(radius))
    out = []
    for dz in range(-r, r + 1):
        for dy in range(-r, r + 1):
            for dx in range(-r, r + 1):
                d = math.sqrt(dx * dx + dy * dy + dz * dz)
                if d < radius:
                    out.append((dz, dy, dx, radius - d))
    return out


def _shifted(a: np.ndarray, dz: int, dy: int, dx: int) -> np.ndarray:
    """b[k,j,i] = a[k+dz, j+dy, i+dx], zero where that index is outside."""
    nz, ny, nx = a.shape
    b = np.zeros_like(a)
    zs, ze = max(0, -dz), min(nz, nz - dz)
    ys, ye = max(0, -dy), min(ny, ny - dy)
    xs, xe = max(0, -dx), min(nx, nx - dx)
    if zs < ze and ys < ye and xs < xe:
        b[zs:ze, ys:ye, xs:xe] = a[zs + dz:ze + dz, ys + dy:ye + dy, xs + dx:xe + dx]
    return b


def weight_sums(shape, radius: float) -> np.ndarray:
    """W[n] = sum of the cone weights of the design voxels around n."""
    one = np.ones(shape, dtype=np.float64)
    W = np.zeros(shape, dtype=np.float64)
    for dz, dy, dx, w in sphere_offsets(radius):
        W += w * _shifted(one, dz, dy, dx)
    return W


def cone_filter(rho: np.ndarray, radius: float) -> np.ndarray:
    """Eq. FilterFunction."""
    rho = np.asarray(rho, dtype=np.float64)
    num = np.zeros_like(rho)
    for dz, dy, dx, w in sphere_offsets(radius):
        num += w * _shifted(rho, dz, dy, dx)
    return num / weight_sums(rho.shape, radius)


def project(rho_t: np.ndarray, beta: float, eta: float) -> np.ndarray:
    """Eq. Projection (smoothed Heaviside)."""
    den = math.tanh(beta * eta) + math.tanh(beta * (1.0 - eta))
    return (math.tanh(beta * eta) + np.tanh(beta * (np.asarray(rho_t, np.float64) - eta))) / den


def project_derivative(rho_t: np.ndarray, beta: float, eta: float) -> np.ndarray:
    """d rho_b / d rho_t of Eq. Projection."""
    den = math.tanh(beta * eta) + math.tanh(beta * (1.0 - eta))
    t = np.tanh(beta * (np.asarray(rho_t, np.float64) - eta))
    return beta * (1.0 - t * t) / den


def filter_project_grad(dF_drho_b: np.ndarray, rho: np.ndarray, radius: float, beta: float,
                        eta: float) -> np.ndarray:
    """Eq. GradientsFiltered: the chain rule from dF/drho_b back to dF/drho."""
    rho_t = cone_filter(rho, radius)
    u = np.asarray(dF_drho_b, np.float64) * project_derivative(rho_t, beta, eta)
    v = u / weight_sums(rho.shape, radius)
    g = np.zeros_like(v)
    # dF/drho[n] = sum_m w(m,n) v[m]; w is symmetric, so the same sphere
    for dz, dy, dx, w in sphere_offsets(radius):
        g += w * _shifted(v, dz, dy, dx)
    return g


def nondiscreteness(rho_b: np.ndarray) -> float:
    """Eq. MeasureOfNon-discretness, in percent."""
    r = np.asarray(rho_b, np.float64).ravel()
    return float(np.sum(4.0 * r * (1.0 - r)) / r.size * 100.0)
