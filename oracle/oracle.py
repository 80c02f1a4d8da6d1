"""ctypes binding of the FP64 CPU oracle (test infrastructure only).

Only tests/, the smoke check and the benchmark's CPU-baseline leg may use this
module.  Arguments are numpy arrays in SI units; see ccpr_oracle.h for the grid
convention and the meaning of every call.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
_LIB = None

OBJ_TIME = 0
OBJ_DFT = 1

_d = C.c_double
_i = C.c_int
_p = C.c_void_p
_dp = C.POINTER(C.c_double)
_ip = C.POINTER(C.c_int)


def _lib():
    global _LIB
    if _LIB is None:
        path = os.path.join(HERE, "liboracle.so")
        if not os.path.exists(path):
            from . import build as _b  # noqa: WPS433 (test infrastructure)
            _b.build()
        lib = C.CDLL(path)
        lib.or_create.restype = _p
        lib.or_create.argtypes = [_i, _i, _i, _d, _d, _i, _d, _d, _d, _d]
        lib.or_destroy.argtypes = [_p]
        lib.or_dt.restype = _d
        lib.or_dt.argtypes = [_p]
        lib.or_set_material.argtypes = [_p, _i, _i, _d, _d, _i, _dp, _dp]
        lib.or_set_design.argtypes = [_p, _ip, _ip, _d, _dp]
        lib.or_set_design_edges.argtypes = [_p, _ip, _ip, _d, _dp]
        lib.or_design_outputs.argtypes = [_p]
        lib.or_design_outputs.restype = C.c_longlong
        lib.or_set_dipole.argtypes = [_p, _ip, _i, _dp, _i]
        lib.or_set_planewave.argtypes = [_p, _i, _i, _i, _ip, _ip, _dp, _i]
        lib.or_set_box_source.argtypes = [_p, _ip, _ip, _dp, _i]
        lib.or_clear_sources.argtypes = [_p]
        lib.or_reset.argtypes = [_p]
        lib.or_run.argtypes = [_p, _i]
        lib.or_step_count.restype = _i
        lib.or_step_count.argtypes = [_p]
        lib.or_get_field.argtypes = [_p, _i, _dp]
        lib.or_set_field.argtypes = [_p, _i, _dp]
        lib.or_get_forward_end_field.restype = _i
        lib.or_get_forward_end_field.argtypes = [_p, _i, _dp]
        lib.or_gradient.argtypes = [_p, _i, _i, _ip, _ip, _d, _i, _i, _dp, _dp, _dp]
        lib.or_objective.argtypes = [_p, _i, _i, _ip, _ip, _d, _i, _i, _dp]
        lib.or_gradient_dft.argtypes = [_p, _i, _ip, _ip, _d, _dp, _dp]
        lib.or_dft_window.restype = _i
        lib.or_dft_window.argtypes = [_i, _d, _d]
        lib.or_edge_response.argtypes = [_p, _i, _d, _d, _dp, _i, _dp]
        lib.or_eps_ccpr.argtypes = [_p, _i, _d, _d, _d, _dp, _dp]
        lib.or_num_threads.restype = _i
        lib.or_set_fp32_storage.argtypes = [_p, _i]
        lib.or_get_pml_coef.restype = _i
        lib.or_get_pml_coef.argtypes = [_p, _i, _i, _i, _dp, _dp, _dp]
        _LIB = lib
    return _LIB


def _iv(x):
    a = (C.c_int * 3)(*[int(v) for v in x])
    return a


def _dv(a):
    a = np.ascontiguousarray(a, dtype=np.float64)
    return a, a.ctypes.data_as(_dp)


def edge_shape(dims, c):
    """(z, y, x) shape of the component-c design edges of a design of
    dims = (Nx, Ny, Nz) cells: N_l + 1 along the two axes other than c."""
    e = [dims[l] + (0 if l == c else 1) for l in range(3)]
    return (e[2], e[1], e[0])


def num_threads() -> int:
    return _lib().or_num_threads()


class OracleSim:
    """One FP64 Yee/CCPR/CPML simulation on an nx*ny*nz grid (x fastest)."""

    def __init__(self, nx, ny, nz, dx, courant=0.5, npml=0, pml_m=3.0,
                 pml_kappa_max=1.0, pml_alpha_max=0.05, pml_sigma_scale=1.0):
        self.shape = (int(nz), int(ny), int(nx))
        self._h = _lib().or_create(nx, ny, nz, dx, courant, npml, pml_m,
                                   pml_kappa_max, pml_alpha_max, pml_sigma_scale)
        if not self._h:
            raise ValueError("oracle: invalid grid")
        self.dt = _lib().or_dt(self._h)
        self.dx = dx
        self.design_dims = None
        self.per_edge = False

    def close(self):
        if self._h:
            _lib().or_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _chk(self, rc, what):
        if rc != 0:
            raise ValueError(f"oracle: {what} rejected")

    def set_material(self, slot, axis, eps_inf, sigma=0.0, a=(), c=()):
        a = np.asarray(a, dtype=np.complex128).ravel()
        c = np.asarray(c, dtype=np.complex128).ravel()
        assert a.shape == c.shape
        ai, ap = _dv(np.stack([a.real, a.imag], -1).ravel() if a.size else np.zeros(1))
        ci, cp = _dv(np.stack([c.real, c.imag], -1).ravel() if c.size else np.zeros(1))
        self._chk(_lib().or_set_material(self._h, slot, axis, eps_inf, sigma, a.size, ap, cp),
                  "material")

    def set_material_all_axes(self, slot, eps_inf, sigma=0.0, a=(), c=()):
        for ax in range(3):
            self.set_material(slot, ax, eps_inf, sigma, a, c)

    def set_design(self, lo, rho, gamma=0.0):
        """rho has shape (dz, dy, dx) (x fastest)."""
        rho = np.asarray(rho, dtype=np.float64)
        dims = (rho.shape[2], rho.shape[1], rho.shape[0])
        r, rp = _dv(rho.ravel())
        self._rho_keep = r
        self.design_dims = dims
        self.per_edge = False
        self._chk(_lib().or_set_design(self._h, _iv(lo), _iv(dims), gamma, rp), "design")

    def set_design_edges(self, lo, dims, rho_edges, gamma=0.0):
        """One density per E edge of a design of dims = (Nx, Ny, Nz) cells:
        rho_edges = (rho_x, rho_y, rho_z), rho_c shaped edge_shape(dims, c)."""
        parts = []
        for c in range(3):
            r = np.asarray(rho_edges[c], dtype=np.float64)
            assert r.shape == edge_shape(dims, c), (r.shape, edge_shape(dims, c))
            parts.append(r.ravel())
        r, rp = _dv(np.concatenate(parts))
        self._rho_keep = r
        self.design_dims = tuple(dims)
        self.per_edge = True
        self._chk(_lib().or_set_design_edges(self._h, _iv(lo), _iv(dims), gamma, rp), "edge design")

    def _grad_shape(self, g):
        """Flat gradient -> (dz, dy, dx) per voxel, or the three per-edge arrays."""
        d = self.design_dims
        if not self.per_edge:
            return g.reshape(d[2], d[1], d[0])
        out, o = [], 0
        for c in range(3):
            shp = edge_shape(d, c)
            n = int(np.prod(shp))
            out.append(g[o:o + n].reshape(shp))
            o += n
        return tuple(out)

    def set_dipole(self, cell, axis, wave):
        w, wp = _dv(wave)
        self._chk(_lib().or_set_dipole(self._h, _iv(cell), axis, wp, w.size), "dipole")

    def set_planewave(self, prop_axis, sign, pol_axis, lo, hi, wave):
        w, wp = _dv(wave)
        self._chk(_lib().or_set_planewave(self._h, prop_axis, sign, pol_axis, _iv(lo), _iv(hi),
                                          wp, w.size), "plane wave")

    def set_box_source(self, lo, dims, table):
        """table shape (nsteps, ncell, 3), cells x-fastest within the box."""
        t = np.asarray(table, dtype=np.float64)
        tt, tp = _dv(t.ravel())
        self._chk(_lib().or_set_box_source(self._h, _iv(lo), _iv(dims), tp, t.shape[0]),
                  "box source")

    def clear_sources(self):
        _lib().or_clear_sources(self._h)

    def reset(self):
        _lib().or_reset(self._h)

    def run(self, nsteps):
        _lib().or_run(self._h, int(nsteps))

    @property
    def step(self):
        return _lib().or_step_count(self._h)

    def field(self, comp):
        out = np.empty(self.shape, dtype=np.float64)
        _lib().or_get_field(self._h, comp, out.ctypes.data_as(_dp))
        return out

    def fields(self):
        return [self.field(c) for c in range(6)]

    def set_fp32_storage(self, on=True):
        """Diagnostic: round every stored state word to FP32 after each update
        (FP64 arithmetic), to measure the floor FP32 storage alone sets."""
        _lib().or_set_fp32_storage(self._h, 1 if on else 0)

    def pml_coefficients(self, axis, half):
        """(b, a, kappa) arrays of the CPML recursion along axis at the
        integer nodes (half = False) or at q + 1/2 (half = True)."""
        n = self.shape[2 - axis]
        out = np.empty((3, n))
        for q in range(n):
            b, a, k = C.c_double(), C.c_double(), C.c_double()
            self._chk(_lib().or_get_pml_coef(self._h, axis, 1 if half else 0, q, C.byref(b), C.byref(a),
                                             C.byref(k)), "pml coefficients")
            out[:, q] = (b.value, a.value, k.value)
        return out[0], out[1], out[2]

    def forward_end_fields(self):
        """The six fields at the end of the forward run inside the last
        gradient / gradient_dft / objective call."""
        out = []
        for c in range(6):
            a = np.empty(self.shape, dtype=np.float64)
            self._chk(_lib().or_get_forward_end_field(self._h, c, a.ctypes.data_as(_dp)), "forward end field")
            out.append(a)
        return out

    def set_field(self, comp, arr):
        a, ap = _dv(np.broadcast_to(arr, self.shape))
        _lib().or_set_field(self._h, comp, ap)

    def gradient(self, nsteps, kind, gap_lo, gap_dims, omega=0.0, n_begin=0, n_end=None,
                 want_hist=False):
        if n_end is None:
            n_end = nsteps + 1
        nd = int(_lib().or_design_outputs(self._h))
        F = C.c_double(0.0)
        g = np.zeros(nd, dtype=np.float64)
        ncell = int(np.prod(gap_dims))
        hist = np.zeros((nsteps + 1, ncell, 3)) if want_hist else None
        hp = hist.ctypes.data_as(_dp) if want_hist else None
        self._chk(_lib().or_gradient(self._h, nsteps, kind, _iv(gap_lo), _iv(gap_dims), omega,
                                     n_begin, n_end, C.byref(F), g.ctypes.data_as(_dp), hp),
                  "gradient")
        g = self._grad_shape(g)
        return (F.value, g, hist) if want_hist else (F.value, g)

    def gradient_dft(self, nsteps, gap_lo, gap_dims, omega):
        """DFT-mode gradient estimator of the DFT objective (or_gradient_dft)."""
        nd = int(_lib().or_design_outputs(self._h))
        F = C.c_double(0.0)
        g = np.zeros(nd, dtype=np.float64)
        self._chk(_lib().or_gradient_dft(self._h, nsteps, _iv(gap_lo), _iv(gap_dims), omega,
                                         C.byref(F), g.ctypes.data_as(_dp)), "DFT-mode gradient")
        return F.value, self._grad_shape(g)

    def objective(self, nsteps, kind, gap_lo, gap_dims, omega=0.0, n_begin=0, n_end=None):
        if n_end is None:
            n_end = nsteps + 1
        F = C.c_double(0.0)
        self._chk(_lib().or_objective(self._h, nsteps, kind, _iv(gap_lo), _iv(gap_dims), omega,
                                      n_begin, n_end, C.byref(F)), "objective")
        return F.value

    @staticmethod
    def dft_window(nsteps, omega, dt):
        return int(_lib().or_dft_window(nsteps, omega, dt))

    def edge_response(self, axis, rho, gamma, src):
        s, sp = _dv(src)
        out = np.zeros(s.size + 1)
        self._chk(_lib().or_edge_response(self._h, axis, rho, gamma, sp, s.size,
                                          out.ctypes.data_as(_dp)), "edge response")
        return out

    def eps_ccpr(self, axis, rho, gamma, w):
        re, im = C.c_double(), C.c_double()
        _lib().or_eps_ccpr(self._h, axis, rho, gamma, w, C.byref(re), C.byref(im))
        return complex(re.value, im.value)
