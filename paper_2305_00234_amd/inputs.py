"""Seeded synthetic inputs: material coefficient sets, waveforms, densities and
workload geometry.

This module is shared by the product's drivers (benchmark, smoke check) and by
the tests that run the FP64 oracle.  It holds no arithmetic of the method
itself -- no field update, no objective, no gradient -- only the numbers that
go *into* a solve.

Material data: the paper's Table 1 CCPR fits (350-1000 nm) stand in for the
measured datasets it fitted; they are reused verbatim as inputs.  The column
headed "Ag" is the set the text calls aluminium; it is exposed under both
names.
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional, Sequence, Tuple

import numpy as np

C0 = 299792458.0
EPS0 = 8.8541878128e-12


# ----------------------------------------------------------------- materials
@dataclasses.dataclass(frozen=True)
class CCPRMaterial:
    """eps(w) = eps_inf + sigma/(j w eps0) + sum_p [c_p/(jw-a_p) + c_p*/(jw-a_p*)]."""

    eps_inf: float
    sigma: float = 0.0
    a: Tuple[complex, ...] = ()
    c: Tuple[complex, ...] = ()

    @property
    def npairs(self) -> int:
        return len(self.a)

    def first_pairs(self, p: int) -> "CCPRMaterial":
        return CCPRMaterial(self.eps_inf, self.sigma, self.a[:p], self.c[:p])

    def scaled_imag_a(self, f: float) -> "CCPRMaterial":
        return CCPRMaterial(self.eps_inf, self.sigma,
                            tuple(complex(z.real, z.imag * f) for z in self.a), self.c)


VACUUM = CCPRMaterial(1.0)

# Table 1 of the paper (CCPR parameters for the spectral fits).
GOLD_TABLE1 = CCPRMaterial(
    eps_inf=2.31, sigma=1.21e7,
    a=(-1.28e14 + 0j, -6.36e14 - 3.89e15j, -2.96e15 - 6.12e15j),
    c=(-6.85e17 + 0j, 2.06e15 + 8.70e14j, 1.60e13 + 1.47e16j))
ALUMINIUM_TABLE1 = CCPRMaterial(
    eps_inf=3.07, sigma=1.49e7,
    a=(-1.89e14 + 0j, -5.46e14 - 6.37e15j, -5.68e14 - 3.43e14j),
    c=(-1.00e18 + 0j, 1.30e15 + 1.54e15j, 1.61e17 + 1.00e12j))
SILICON_TABLE1 = CCPRMaterial(
    eps_inf=1.0, sigma=0.0,
    a=(-8.00e14 + 6.39e15j, -2.32e14 + 5.12e15j),
    c=(7.31e14 - 2.89e16j, 4.68e15 - 4.55e15j))
TIO2_ORDINARY_TABLE1 = CCPRMaterial(eps_inf=2.87, a=(-6.65e15j,), c=(1.01e16j,))
TIO2_EXTRAORDINARY_TABLE1 = CCPRMaterial(eps_inf=3.26, a=(-6.49e15j,), c=(1.29e16j,))


def drude(eps_inf: float, omega_p: float, gamma_d: float) -> CCPRMaterial:
    """Drude metal eps_inf - wp^2/(w^2 - j w gD) in CCPR form: a conductivity
    eps0 wp^2/gD plus one real pole pair a=-gD, c=-wp^2/(2 gD)."""
    return CCPRMaterial(eps_inf, EPS0 * omega_p ** 2 / gamma_d,
                        (complex(-gamma_d, 0.0),), (complex(-omega_p ** 2 / (2 * gamma_d), 0.0),))


def lorentz(eps_inf: float, d_eps: float, omega0: float, delta: float) -> CCPRMaterial:
    """Lorentz oscillator eps_inf + d_eps w0^2/(w0^2 - w^2 + j w delta) in CCPR
    form: a = -delta/2 + j wr, c = -j d_eps w0^2/(2 wr), wr = sqrt(w0^2-delta^2/4)."""
    wr = math.sqrt(omega0 ** 2 - delta ** 2 / 4)
    return CCPRMaterial(eps_inf, 0.0, (complex(-delta / 2, wr),),
                        (complex(0.0, -d_eps * omega0 ** 2 / (2 * wr)),))


# ----------------------------------------------------------------- waveforms
def gaussian_sine(t: np.ndarray, lambda0: float, fwhm: float, t0: float, amp: float = 1.0):
    """exp(-4 ln2 (t-t0)^2/fwhm^2) sin(w0 (t-t0)), w0 = 2 pi c0/lambda0."""
    w0 = 2 * math.pi * C0 / lambda0
    return amp * np.exp(-4 * math.log(2) * (t - t0) ** 2 / fwhm ** 2) * np.sin(w0 * (t - t0))


def sinc_hanning(t: np.ndarray, f0: float, rel_bandwidth: float = 0.5, lobes: int = 3,
                 amp: float = 1.0) -> np.ndarray:
    """Broadband excitation of the paper's optimisation runs (Sec. "Topology
    Optimization Setup"): a sinc truncated to 'lobes' lobes on each side of
    its peak, modulating a carrier of frequency f0, times a Hanning window
    over the truncation.  The sinc's width gives a rectangular band of
    rel_bandwidth * f0 around f0 (the paper quotes ~50 % at half maximum and
    does not give the lobe count: 3 is this package's reading).  Zero outside
    the window [0, 2 lobes / B]."""
    B = rel_bandwidth * f0
    Tw = 2.0 * lobes / B
    tc = t - Tw / 2.0
    win = np.where((t >= 0) & (t <= Tw), 0.5 * (1.0 - np.cos(2 * math.pi * t / Tw)), 0.0)
    return amp * np.sinc(B * tc) * np.cos(2 * math.pi * f0 * tc) * win


def dt_of(dx: float, courant: float) -> float:
    return courant * dx / C0


# ----------------------------------------------------------------- densities
def uniform_density(shape_zyx: Sequence[int], seed: int) -> np.ndarray:
    """rho ~ U[0,1) from numpy's default_rng(seed), drawn in float64 and cast to
    float32: the exact bytes both the GPU path and the oracle consume."""
    rng = np.random.default_rng(seed)
    return rng.random(tuple(shape_zyx), dtype=np.float64).astype(np.float32)


def smooth3(rho: np.ndarray, sigma_cells: float = 1.0, taps: int = 3) -> np.ndarray:
    """Separable Gaussian smoothing (truncated to `taps`, edge-reflect)."""
    h = taps // 2
    k = np.exp(-0.5 * (np.arange(-h, h + 1) / sigma_cells) ** 2)
    k /= k.sum()
    out = rho.astype(np.float64)
    for ax in range(3):
        pad = [(0, 0)] * 3
        pad[ax] = (h, h)
        p = np.pad(out, pad, mode="reflect")
        acc = np.zeros_like(out)
        for t in range(taps):
            sl = [slice(None)] * 3
            sl[ax] = slice(t, t + out.shape[ax])
            acc += k[t] * p[tuple(sl)]
        out = acc
    return np.clip(out, 0.0, 1.0).astype(np.float32)


# ----------------------------------------------------------------- workloads
@dataclasses.dataclass
class Workload:
    """Everything a forward + adjoint + gradient solve needs (SI units)."""

    name: str
    shape: Tuple[int, int, int]             # (nx, ny, nz)
    dx: float
    courant: float
    npml: int
    steps: int
    mat1: Tuple[CCPRMaterial, CCPRMaterial, CCPRMaterial]  # rho=0, per axis x,y,z
    mat2: Tuple[CCPRMaterial, CCPRMaterial, CCPRMaterial]  # rho=1, per axis x,y,z
    design_lo: Tuple[int, int, int]
    rho: np.ndarray                          # float32, shape (dz, dy, dx)
    gamma: float
    source: str                              # "dipole" | "planewave"
    wave: np.ndarray                         # float64 samples
    dipole_cell: Tuple[int, int, int] = (0, 0, 0)
    dipole_axis: int = 0
    pw_prop_axis: int = 2
    pw_sign: int = 1
    pw_pol_axis: int = 0
    tfsf_lo: Tuple[int, int, int] = (0, 0, 0)
    tfsf_hi: Tuple[int, int, int] = (0, 0, 0)
    objective: str = "dft"                   # "dft" | "time"
    gap_lo: Tuple[int, int, int] = (0, 0, 0)
    gap_dims: Tuple[int, int, int] = (1, 1, 1)
    omega: float = 0.0
    window: Tuple[int, int] = (0, -1)        # time objective [n_begin, n_end); -1 = M+1
    checkpoint_every: int = 0                # 0 = let the library choose
    gradient: str = "time"                   # "time" (exact) | "dft" (single-frequency estimator)
    pml_m: float = 3.0
    pml_kappa_max: float = 1.0
    pml_alpha_max: float = 0.05
    pml_sigma_scale: float = 1.0
    # per-edge design (one density per E edge, Sec. "FDTD implementation and
    # design export"): (rho_x, rho_y, rho_z), rho_c shaped edge_shape(N, c)
    # for a design of N cells; None = one density per voxel (rho)
    rho_edges: Optional[Tuple[np.ndarray, np.ndarray, np.ndarray]] = None

    @property
    def dt(self) -> float:
        return dt_of(self.dx, self.courant)

    @property
    def cells(self) -> int:
        return self.shape[0] * self.shape[1] * self.shape[2]

    @property
    def design_dims(self) -> Tuple[int, int, int]:
        if self.rho_edges is not None:
            z = self.rho_edges[2].shape  # (Nz, Ny + 1, Nx + 1)
            return (z[2] - 1, z[1] - 1, z[0])
        return (self.rho.shape[2], self.rho.shape[1], self.rho.shape[0])

    @property
    def window_end(self) -> int:
        return self.steps + 1 if self.window[1] < 0 else self.window[1]

    def max_pairs(self) -> int:
        return max(self.mat1[a].npairs + self.mat2[a].npairs for a in range(3))


def edge_shape(dims: Tuple[int, int, int], c: int) -> Tuple[int, int, int]:
    """(z, y, x) shape of the component-c edges of a per-edge design of
    dims = (Nx, Ny, Nz) cells: N_l + 1 along the two axes other than c."""
    e = [dims[l] + (0 if l == c else 1) for l in range(3)]
    return (e[2], e[1], e[0])


def random_edge_densities(dims: Tuple[int, int, int], seed: int):
    """Per-edge densities ~ U[0,1) (FP64 draws cast to FP32), x, y, z edges."""
    rng = np.random.default_rng(seed)
    return tuple(rng.random(edge_shape(dims, c)).astype(np.float32) for c in range(3))


def voxel_edge_densities(rho: np.ndarray, fill: float = 0.0):
    """Per-edge densities equal to a per-voxel design on the edges the voxels
    own (edge (i,j,k) of each component belongs to voxel (i,j,k)); the extra
    edges on the far faces of the box get 'fill'."""
    nz, ny, nx = rho.shape
    out = []
    for c in range(3):
        e = np.full(edge_shape((nx, ny, nz), c), fill, dtype=np.float32)
        e[:nz, :ny, :nx] = rho
        out.append(e)
    return tuple(out)


def _iso(m: CCPRMaterial):
    return (m, m, m)


def _gap_zero(rho: np.ndarray, design_lo, gap_lo, gap_dims):
    r = rho.copy()
    z0, y0, x0 = (gap_lo[2] - design_lo[2], gap_lo[1] - design_lo[1], gap_lo[0] - design_lo[0])
    r[z0:z0 + gap_dims[2], y0:y0 + gap_dims[1], x0:x0 + gap_dims[0]] = 0.0
    return r


def drude_dipole_32(steps: int = 400, gamma: float = 5e4, seed: int = 0, n: int = 32,
                    npml: int = 8) -> Workload:
    """Plain method, CPU-sized: 32^3 cells, dx=10 nm, S=0.5, 8-cell CPML; vacuum
    plus an 8^3 design box [12,20)^3 of rho~U[0,1] interpolating vacuum and a
    Drude metal (eps_inf=1, plasma 1.37e16 rad/s, damping 1e14 rad/s); an
    x-polarised Gaussian-pulse dipole (500 nm, fwhm 50 fs, envelope peak at
    t=0) on the Ex edge of cell (10,16,16); DFT |E|^2 at 500 nm over the 2^3
    air gap [15,17)^3 (rho fixed to 0)."""
    dx, S = 10e-9, 0.5
    c = n // 2
    lo = (c - 4, c - 4, c - 4)
    gap_lo, gap_dims = (c - 1, c - 1, c - 1), (2, 2, 2)
    rho = _gap_zero(uniform_density((8, 8, 8), seed), lo, gap_lo, gap_dims)
    metal = drude(1.0, 1.37e16, 1e14)
    t = (np.arange(steps) + 0.5) * dt_of(dx, S)
    wave = gaussian_sine(t, 500e-9, 50e-15, 0.0, amp=1e9)
    return Workload("drude_dipole_32", (n, n, n), dx, S, npml, steps, _iso(VACUUM), _iso(metal),
                    lo, rho, gamma, "dipole", wave, dipole_cell=(c - 6, c, c), dipole_axis=0,
                    objective="dft", gap_lo=gap_lo, gap_dims=gap_dims,
                    omega=2 * math.pi * C0 / 500e-9)


def gold_gap(n: Tuple[int, int, int] = (320, 320, 320), design: Tuple[int, int, int] = (160, 160, 80),
             gap: int = 4, dx: float = 5e-9, npml: int = 12, steps: int = 6000,
             seed: int = 1, gamma: float = 5e4, objective: str = "dft",
             name: Optional[str] = None, tfsf_margin: int = 4) -> Workload:
    """Gap field-enhancement problem shaped like the paper's (Methods,
    "Technical details"): vacuum grid with a CPML, a centred design box of
    smoothed rho~U[0,1] interpolating vacuum and Table-1 gold (sigma + 3 CCPR
    pairs), an x-polarised TF/SF plane wave travelling along +z (Gaussian
    pulse, 800 nm, fwhm 2.4 fs, t0 = 3 fwhm), the objective over a gap^3 air
    gap at the centre (rho fixed to 0)."""
    nx, ny, nz = n
    lo = ((nx - design[0]) // 2, (ny - design[1]) // 2, (nz - design[2]) // 2)
    gap_lo = (nx // 2 - gap // 2, ny // 2 - gap // 2, nz // 2 - gap // 2)
    gap_dims = (gap, gap, gap)
    rho = smooth3(uniform_density((design[2], design[1], design[0]), seed))
    rho = _gap_zero(rho, lo, gap_lo, gap_dims)
    S = 0.5
    t = np.arange(steps + 1) * dt_of(dx, S)
    wave = gaussian_sine(t, 800e-9, 2.4e-15, 7.2e-15, amp=1.0)
    m = npml + tfsf_margin
    return Workload(name or f"gold_gap_{nx}x{ny}x{nz}", n, dx, S, npml, steps, _iso(VACUUM),
                    _iso(GOLD_TABLE1), lo, rho, gamma, "planewave", wave,
                    pw_prop_axis=2, pw_sign=1, pw_pol_axis=0,
                    tfsf_lo=(m, m, m), tfsf_hi=(nx - m, ny - m, nz - m),
                    objective=objective, gap_lo=gap_lo, gap_dims=gap_dims,
                    omega=2 * math.pi * C0 / 800e-9)


def paper_broadband(material: str = "gold", steps: int = 18000, seed: int = 6) -> Workload:
    """The paper's optimisation problem for the metals (Sec. "Technical details
    of the optimization"): a 100 x 25 x 100 cell design region (200 x 50 x 200
    nm at dx = 2 nm) with a 6 x 25 x 6 air gap at its centre, a z-polarised
    plane wave travelling along +y (sinc x Hanning pulse on a 576.5 THz
    carrier), 18000 steps at Courant 0.5 (dt = 3.34e-3 fs, 60.1 fs), the
    time-domain objective (Eq. 2) over the whole run, gamma = 5e4, a 20-cell
    CPML.  The paper does not give the vacuum margins: here 10 cells between
    the design and the TF/SF box and 5 between the box and the CPML.  rho is
    seeded U[0,1], smoothed, zero in the gap."""
    mat = {"gold": GOLD_TABLE1, "aluminium": ALUMINIUM_TABLE1}[material]
    design, npml, inner, outer = (100, 25, 100), 20, 10, 5
    m = npml + outer
    n = tuple(d + 2 * (m + inner) for d in design)
    lo = tuple(m + inner for _ in range(3))
    gap_dims = (6, 25, 6)
    gap_lo = (lo[0] + (design[0] - 6) // 2, lo[1], lo[2] + (design[2] - 6) // 2)
    rho = smooth3(uniform_density((design[2], design[1], design[0]), seed))
    rho = _gap_zero(rho, lo, gap_lo, gap_dims)
    dx, S = 2e-9, 0.5
    t = np.arange(steps + 1) * dt_of(dx, S)
    wave = sinc_hanning(t, 576.5e12, 0.5, 3)
    w = Workload(f"paper_broadband_{material}", n, dx, S, npml, steps, _iso(VACUUM), _iso(mat), lo, rho, 5e4,
                 "planewave", wave, pw_prop_axis=1, pw_sign=1, pw_pol_axis=2,
                 tfsf_lo=(m, m, m), tfsf_hi=(n[0] - m, n[1] - m, n[2] - m),
                 objective="time", gap_lo=gap_lo, gap_dims=gap_dims,
                 omega=2 * math.pi * 576.5e12)
    return w


def gold_gap_320(steps: int = 6000) -> Workload:
    """Paper-shaped gap problem: 320^3, dx=5 nm, 12-cell CPML, 160x160x80
    design, 3 gold pole pairs, 6000 steps, DFT |E|^2 over a 4^3 gap."""
    return gold_gap(steps=steps, name="gold_gap_320")


def gold_gap_timedomain_512(steps: int = 8000, checkpoint_every: int = 1000) -> Workload:
    """Differentiation workload: 512x512x256 cells, 256x256x64 design, 3 gold
    pairs, time-domain objective (Eq. 2) over the whole run, checkpoints every
    1000 steps."""
    w = gold_gap(n=(512, 512, 256), design=(256, 256, 64), steps=steps, seed=2,
                 objective="time", name="gold_gap_td_512x512x256")
    w.checkpoint_every = checkpoint_every
    return w


def aniso_two_material(n: Tuple[int, int, int], design: Tuple[int, int, int], steps: int,
                       npml: int = 12, seed: int = 4, name: Optional[str] = None,
                       gap: int = 4) -> Workload:
    """Anisotropic multi-material gap problem (dx=4 nm): rho=0 is a dispersive
    dielectric (eps_inf 2.1, Lorentz at 150 nm, d_eps 1, damping 1e14), rho=1
    a diagonal-anisotropic metal (x: Table-1 gold, y: Table-1 aluminium set,
    z: gold with Im a_p x 1.1); 4 pole pairs per component, different per axis."""
    w = gold_gap(n=n, design=design, dx=4e-9, steps=steps, seed=seed, npml=npml, gap=gap,
                 name=name or f"aniso_two_material_{n[0]}x{n[1]}x{n[2]}")
    diel = lorentz(2.1, 1.0, 2 * math.pi * C0 / 150e-9, 1e14)
    w.mat1 = _iso(diel)
    w.mat2 = (GOLD_TABLE1, ALUMINIUM_TABLE1, GOLD_TABLE1.scaled_imag_a(1.1))
    return w


def aniso_two_material_384(steps: int = 8000) -> Workload:
    """The 384^3 anisotropic two-material workload: 192x192x96 design, 8000 steps."""
    return aniso_two_material((384, 384, 384), (192, 192, 96), steps, name="aniso_two_material_384")


@dataclasses.dataclass
class ServingRequest:
    arrival: float
    workload: Workload


def serving_trace(n_requests: int = 500, rate: float = 20.0, seed: int = 3,
                  side_range: Tuple[int, int] = (64, 192),
                  steps_range: Tuple[int, int] = (1500, 4000)) -> List[ServingRequest]:
    """Poisson stream of forward+adjoint requests: cubic grids of side
    ~U{64..192}, design boxes of side/4, 1-3 gold pole pairs, rho~U[0,1],
    1500-4000 steps, dx=10 nm, 8-cell CPML, dipole source and DFT gap probe."""
    rng = np.random.default_rng(seed)
    t = 0.0
    out = []
    for r in range(n_requests):
        t += rng.exponential(1.0 / rate)
        side = int(rng.integers(side_range[0], side_range[1] + 1))
        P = int(rng.integers(1, 4))
        steps = int(rng.integers(steps_range[0], steps_range[1] + 1))
        out.append(ServingRequest(t, serving_workload(side, P, steps, seed=1000 + r)))
    return out


def serving_workload(side: int, pairs: int, steps: int, seed: int, dx: float = 10e-9,
                     npml: int = 8, gamma: float = 5e4) -> Workload:
    d = max(2, side // 4)
    c = side // 2
    lo = (c - d // 2, c - d // 2, c - d // 2)
    gap_lo, gap_dims = (c - 1, c - 1, c - 1), (2, 2, 2)
    rho = _gap_zero(uniform_density((d, d, d), seed), lo, gap_lo, gap_dims)
    S = 0.5
    t = (np.arange(steps) + 0.5) * dt_of(dx, S)
    wave = gaussian_sine(t, 500e-9, 2.0e-15, 6.0e-15, amp=1e9)
    metal = GOLD_TABLE1.first_pairs(pairs)
    dip = (max(npml + 2, lo[0] - 3), c, c)
    return Workload(f"serve_{side}_p{pairs}_m{steps}", (side, side, side), dx, S, npml, steps,
                    _iso(VACUUM), _iso(metal), lo, rho, gamma, "dipole", wave,
                    dipole_cell=dip, dipole_axis=0, objective="dft", gap_lo=gap_lo,
                    gap_dims=gap_dims, omega=2 * math.pi * C0 / 500e-9)
