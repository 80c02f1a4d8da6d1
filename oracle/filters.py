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

Both the per-voxel density grid and the per-edge variables (one density per
E edge at the staggered edge centres, the sphere then spanning all three
components) are covered.

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


# ----------------------------------------------------- per-edge design
# With one density per E edge (Sec. "FDTD implementation and design
# export") the variables sit at the staggered edge centres: for a design of
# N = (Nx, Ny, Nz) cells, the x edges at (i + 1/2, j, k) with i < Nx, j <= Ny,
# k <= Nz, the y edges at (i, j + 1/2, k), the z edges at (i, j, k + 1/2).
# Eq. FilterFunction then sums over every variable, of any component, whose
# position lies within R of the output's position.

def edge_shape(dims, c):
    """(z, y, x) shape of the component-c edges of an N-cell design."""
    e = [dims[l] + (0 if l == c else 1) for l in range(3)]
    return (e[2], e[1], e[0])


def _half(c):
    """(z, y, x) half-cell offset of component c's positions."""
    h = [0.0, 0.0, 0.0]
    h[2 - c] = 0.5
    return h


def edge_pair_offsets(radius: float, a: int, b: int):
    """Integer index offsets o = (dz, dy, dx) such that input edge m = n + o
    of component b lies within radius of output edge n of component a, with
    the cone weight radius - |o + h_b - h_a|."""
    ha, hb = _half(a), _half(b)
    s = [hb[q] - ha[q] for q in range(3)]
    r = int(math.ceil(radius)) + 1
    out = []
    for dz in range(-r, r + 1):
        for dy in range(-r, r + 1):
            for dx in range(-r, r + 1):
                d = math.sqrt((dz + s[0]) ** 2 + (dy + s[1]) ** 2 + (dx + s[2]) ** 2)
                if d < radius:
                    out.append((dz, dy, dx, radius - d))
    return out


def _shifted_to(src: np.ndarray, out_shape, dz: int, dy: int, dx: int) -> np.ndarray:
    """b[k,j,i] = src[k+dz, j+dy, i+dx] on out_shape, zero outside src."""
    b = np.zeros(out_shape, dtype=np.float64)
    lo = [max(0, -o) for o in (dz, dy, dx)]
    hi = [min(out_shape[q], src.shape[q] - o) for q, o in enumerate((dz, dy, dx))]
    if all(lo[q] < hi[q] for q in range(3)):
        b[lo[0]:hi[0], lo[1]:hi[1], lo[2]:hi[2]] = src[lo[0] + dz:hi[0] + dz, lo[1] + dy:hi[1] + dy,
                                                       lo[2] + dx:hi[2] + dx]
    return b


def _edge_weighted_sums(vals, dims, radius):
    """out_a[n] = sum_b sum_m w(|r_b(m) - r_a(n)|) vals_b[m] over the edges
    within radius (vals: three arrays in edge_shape(dims, b))."""
    out = []
    for a in range(3):
        acc = np.zeros(edge_shape(dims, a), dtype=np.float64)
        for b in range(3):
            src = np.asarray(vals[b], dtype=np.float64)
            for dz, dy, dx, w in edge_pair_offsets(radius, a, b):
                acc += w * _shifted_to(src, acc.shape, dz, dy, dx)
        out.append(acc)
    return out


def edge_weight_sums(dims, radius: float):
    """W_a[n] = sum of the cone weights of all design edges around edge n."""
    return _edge_weighted_sums([np.ones(edge_shape(dims, c)) for c in range(3)], dims, radius)


def cone_filter_edges(rho_edges, dims, radius: float):
    """Eq. FilterFunction over the per-edge variables (x, y, z arrays)."""
    num = _edge_weighted_sums(rho_edges, dims, radius)
    W = edge_weight_sums(dims, radius)
    return [num[a] / W[a] for a in range(3)]


def filter_project_grad_edges(dF_drho_b, rho_edges, dims, radius: float, beta: float, eta: float):
    """Eq. GradientsFiltered over the per-edge variables: dF/drho_n =
    sum_m w(m, n) v_m with v = dF/drho_b * drho_b/drho_t / W (w symmetric)."""
    rt = cone_filter_edges(rho_edges, dims, radius)
    W = edge_weight_sums(dims, radius)
    v = [np.asarray(dF_drho_b[a], np.float64) * project_derivative(rt[a], beta, eta) / W[a] for a in range(3)]
    return _edge_weighted_sums(v, dims, radius)
