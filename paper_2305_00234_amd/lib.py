"""ctypes binding of libccprfdtd.so (the C-ABI of include/ccprfdtd.h).

Argument marshalling only: every step of the path runs in the library's gfx950
kernels.  PyTorch supplies device memory (the workspace, device densities and
gradients) and the HIP stream; there is no fallback of any kind -- if the
library has not been built, ``load()`` raises.
"""
from __future__ import annotations

import contextlib
import ctypes as C
import os
from typing import Optional, Sequence

import numpy as np

from .inputs import edge_shape

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libccprfdtd.so")

OK, EINVAL, ECFL, ENOMEM, EDEVICE, ESTATE, EDIVERGED, ENOTSUP = 0, -1, -2, -3, -4, -5, -6, -7
STATUS_NAMES = {0: "CCPR_OK", -1: "CCPR_EINVAL", -2: "CCPR_ECFL", -3: "CCPR_ENOMEM",
                -4: "CCPR_EDEVICE", -5: "CCPR_ESTATE", -6: "CCPR_EDIVERGED", -7: "CCPR_ENOTSUP"}
MEM_HOST, MEM_DEVICE = 0, 1
OBJ_TIME_E2, OBJ_DFT_E2 = 0, 1
EX, EY, EZ, HX, HY, HZ = range(6)

# every entry point declared in include/ccprfdtd.h
EXPORTS = [
    "ccpr_create", "ccpr_destroy", "ccpr_last_error", "ccpr_set_material", "ccpr_set_design",
    "ccpr_set_design_edges", "ccpr_workspace_size_max", "ccpr_set_resident_segments",
    "ccpr_get_resident_segments",
    "ccpr_set_source_dipole", "ccpr_set_source_planewave", "ccpr_set_objective",
    "ccpr_set_checkpointing", "ccpr_set_gradient_mode", "ccpr_workspace_size", "ccpr_bind_workspace",
    "ccpr_bind_static_workspace", "ccpr_forward",
    "ccpr_adjoint", "ccpr_gradient", "ccpr_gap_spectrum", "ccpr_reset", "ccpr_step", "ccpr_get_field",
    "ccpr_step_count", "ccpr_set_timing", "ccpr_get_timing", "ccpr_get_grid_timing", "ccpr_get_info",
    "ccpr_set_tile_planes", "ccpr_set_tile_rows", "ccpr_set_design_fusion", "ccpr_get_design_fusion",
    "ccpr_set_watchdog", "ccpr_forward_serial",
    "ccpr_engine_create", "ccpr_engine_submit", "ccpr_engine_poll", "ccpr_engine_wait",
    "ccpr_engine_result", "ccpr_engine_release", "ccpr_engine_last_error", "ccpr_engine_destroy",
    "ccpr_engine_set_batching",
    "ccpr_filter_project", "ccpr_filter_project_grad", "ccpr_nondiscreteness",
    "ccpr_filter_project_edges", "ccpr_filter_project_grad_edges",
]
JOB_QUEUED, JOB_RUNNING, JOB_DONE, JOB_FAILED = 0, 1, 2, 3
GRAD_TIME_EXACT, GRAD_DFT = 0, 1


class CcprGrid(C.Structure):
    _fields_ = [("nx", C.c_int), ("ny", C.c_int), ("nz", C.c_int), ("dx", C.c_double),
                ("courant", C.c_double), ("npml", C.c_int), ("pml_order", C.c_double),
                ("pml_kappa_max", C.c_double), ("pml_alpha_max", C.c_double),
                ("pml_sigma_scale", C.c_double)]


class CcprError(RuntimeError):
    def __init__(self, status: int, what: str, msg: str):
        super().__init__(f"{what}: {STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


_LIB = None
_p = C.c_void_p
_i = C.c_int
_d = C.c_double
_ip = C.POINTER(C.c_int)
_dp = C.POINTER(C.c_double)
_fp = C.POINTER(C.c_float)


def load():
    """Load the built library (raises FileNotFoundError if it was not built)."""
    global _LIB
    if _LIB is not None:
        return _LIB
    if not os.path.exists(LIB_PATH):
        raise FileNotFoundError(
            f"{LIB_PATH} is missing: build it with `python -m paper_2305_00234_amd.build`")
    lib = C.CDLL(LIB_PATH)
    sig = {
        "ccpr_create": (_i, [C.POINTER(CcprGrid), C.POINTER(_p)]),
        "ccpr_destroy": (None, [_p]),
        "ccpr_last_error": (C.c_char_p, [_p]),
        "ccpr_set_material": (_i, [_p, _i, _i, _d, _d, _i, _dp, _dp]),
        "ccpr_set_design": (_i, [_p, _ip, _ip, _d, _p, _i]),
        "ccpr_set_design_edges": (_i, [_p, _ip, _ip, _d, _p, _i]),
        "ccpr_set_source_dipole": (_i, [_p, _ip, _i, _dp, _i]),
        "ccpr_set_source_planewave": (_i, [_p, _i, _i, _i, _ip, _ip, _dp, _i]),
        "ccpr_set_objective": (_i, [_p, _i, _ip, _ip, _d, _i, _i]),
        "ccpr_set_checkpointing": (_i, [_p, _i]),
        "ccpr_set_gradient_mode": (_i, [_p, _i]),
        "ccpr_workspace_size": (_i, [_p, _i, C.POINTER(C.c_uint64)]),
        "ccpr_workspace_size_max": (_i, [_p, _i, C.POINTER(C.c_uint64)]),
        "ccpr_set_resident_segments": (_i, [_p, _i]),
        "ccpr_get_resident_segments": (_i, [_p, _ip]),
        "ccpr_bind_workspace": (_i, [_p, _p, C.c_uint64, _p]),
        "ccpr_bind_static_workspace": (_i, [_p, _p]),
        "ccpr_forward": (_i, [_p, _i, _dp]),
        "ccpr_adjoint": (_i, [_p]),
        "ccpr_gradient": (_i, [_p, _p, _i]),
        "ccpr_gap_spectrum": (_i, [_p, _dp, _i, _dp]),
        "ccpr_reset": (_i, [_p]),
        "ccpr_step": (_i, [_p, _i]),
        "ccpr_get_field": (_i, [_p, _i, _p, _i]),
        "ccpr_step_count": (_i, [_p]),
        "ccpr_set_timing": (_i, [_p, _i]),
        "ccpr_get_timing": (_i, [_p, _dp, C.POINTER(C.c_longlong)]),
        "ccpr_get_grid_timing": (_i, [_p, _dp, C.POINTER(C.c_longlong)]),
        "ccpr_get_info": (_i, [_p, _ip, _ip, _ip]),
        "ccpr_set_tile_planes": (_i, [_p, _i]),
        "ccpr_set_tile_rows": (_i, [_p, _i]),
        "ccpr_set_design_fusion": (_i, [_p, _i]),
        "ccpr_get_design_fusion": (_i, [_p, _ip]),
        "ccpr_set_watchdog": (_i, [_p, _i, _d]),
        "ccpr_forward_serial": (C.c_longlong, [_p]),
        "ccpr_engine_create": (_i, [_p, C.c_uint64, _i, _i, C.POINTER(_p)]),
        "ccpr_engine_submit": (_i, [_p, _p, _i, C.POINTER(C.c_uint64)]),
        "ccpr_engine_poll": (_i, [_p, C.c_uint64, _ip]),
        "ccpr_engine_wait": (_i, [_p, C.c_uint64, _ip]),
        "ccpr_engine_result": (_i, [_p, C.c_uint64, _dp, _dp, _dp]),
        "ccpr_engine_release": (_i, [_p, C.c_uint64]),
        "ccpr_engine_last_error": (C.c_char_p, [_p]),
        "ccpr_engine_destroy": (None, [_p]),
        "ccpr_engine_set_batching": (_i, [_p, _i]),
        "ccpr_filter_project": (_i, [_p, _p, _p, _p, _ip, _d, _d, _d, _p]),
        "ccpr_filter_project_grad": (_i, [_p, _p, _p, _p, _ip, _d, _d, _d, _p]),
        "ccpr_filter_project_edges": (_i, [_p, _p, _p, _p, _ip, _d, _d, _d, _p]),
        "ccpr_filter_project_grad_edges": (_i, [_p, _p, _p, _p, _ip, _d, _d, _d, _p]),
        "ccpr_nondiscreteness": (_i, [_p, C.c_longlong, _p, _p]),
    }
    for name, (res, args) in sig.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    _LIB = lib
    return lib


def _i3(v: Sequence[int]):
    return (C.c_int * 3)(*[int(x) for x in v])


def _f64(a):
    a = np.ascontiguousarray(a, dtype=np.float64)
    return a, a.ctypes.data_as(_dp)


def _check_free(st, what):
    if st != OK:
        raise CcprError(st, what, "")


def _cuda_tensor(t, dtype, name):
    import torch
    if not (isinstance(t, torch.Tensor) and t.is_cuda and t.dtype == dtype and t.is_contiguous()
            and t.dim() == 3):
        raise ValueError(f"{name} must be a contiguous 3-D CUDA {dtype} tensor (dz, dy, dx)")
    return t


def filter_project(rho, radius: float, beta: float, eta: float):
    """ccpr_filter_project on a float32 CUDA density tensor (dz, dy, dx), on
    torch's current stream: returns (rho_filtered, rho_projected, weight_sum)."""
    import torch
    _cuda_tensor(rho, torch.float32, "rho")
    rt, rb, ws = torch.empty_like(rho), torch.empty_like(rho), torch.empty_like(rho)
    dims = _i3((rho.shape[2], rho.shape[1], rho.shape[0]))
    st = load().ccpr_filter_project(C.c_void_p(rho.data_ptr()), C.c_void_p(rt.data_ptr()),
                                    C.c_void_p(rb.data_ptr()), C.c_void_p(ws.data_ptr()), dims, radius,
                                    beta, eta, C.c_void_p(torch.cuda.current_stream(rho.device).cuda_stream))
    _check_free(st, "ccpr_filter_project")
    return rt, rb, ws


def filter_project_grad(dF_dprojected, rho_filtered, weight_sum, radius: float, beta: float, eta: float):
    """ccpr_filter_project_grad: dF/drho (float64) from dF/drho_projected
    (float64) and the forward call's rho_filtered and weight_sum."""
    import torch
    _cuda_tensor(dF_dprojected, torch.float64, "dF_dprojected")
    _cuda_tensor(rho_filtered, torch.float32, "rho_filtered")
    _cuda_tensor(weight_sum, torch.float32, "weight_sum")
    g = torch.empty_like(dF_dprojected)
    dims = _i3((g.shape[2], g.shape[1], g.shape[0]))
    st = load().ccpr_filter_project_grad(C.c_void_p(dF_dprojected.data_ptr()),
                                         C.c_void_p(rho_filtered.data_ptr()), C.c_void_p(weight_sum.data_ptr()),
                                         C.c_void_p(g.data_ptr()), dims, radius, beta, eta,
                                         C.c_void_p(torch.cuda.current_stream(g.device).cuda_stream))
    _check_free(st, "ccpr_filter_project_grad")
    return g


def edge_count(dims) -> int:
    """Design edges of an N-cell per-edge design (N~_x + N~_y + N~_z)."""
    return sum(int(np.prod(edge_shape(dims, c))) for c in range(3))


def _flat_cuda(t, dtype, n, name):
    import torch
    if not (isinstance(t, torch.Tensor) and t.is_cuda and t.dtype == dtype and t.is_contiguous()
            and t.numel() == n):
        raise ValueError(f"{name} must be a contiguous CUDA {dtype} tensor of {n} values (per-edge layout)")
    return t


def filter_project_edges(rho, dims, radius: float, beta: float, eta: float):
    """ccpr_filter_project_edges on a flat float32 CUDA tensor of per-edge
    densities (x, y, z edges of a dims-cell design): returns
    (rho_filtered, rho_projected, weight_sum), same layout."""
    import torch
    _flat_cuda(rho, torch.float32, edge_count(dims), "rho")
    rt, rb, ws = torch.empty_like(rho), torch.empty_like(rho), torch.empty_like(rho)
    st = load().ccpr_filter_project_edges(C.c_void_p(rho.data_ptr()), C.c_void_p(rt.data_ptr()),
                                          C.c_void_p(rb.data_ptr()), C.c_void_p(ws.data_ptr()), _i3(dims),
                                          radius, beta, eta,
                                          C.c_void_p(torch.cuda.current_stream(rho.device).cuda_stream))
    _check_free(st, "ccpr_filter_project_edges")
    return rt, rb, ws


def filter_project_grad_edges(dF_dprojected, rho_filtered, weight_sum, dims, radius: float, beta: float,
                              eta: float):
    """ccpr_filter_project_grad_edges: the per-edge chain rule (float64)."""
    import torch
    n = edge_count(dims)
    _flat_cuda(dF_dprojected, torch.float64, n, "dF_dprojected")
    _flat_cuda(rho_filtered, torch.float32, n, "rho_filtered")
    _flat_cuda(weight_sum, torch.float32, n, "weight_sum")
    g = torch.empty_like(dF_dprojected)
    st = load().ccpr_filter_project_grad_edges(C.c_void_p(dF_dprojected.data_ptr()),
                                               C.c_void_p(rho_filtered.data_ptr()),
                                               C.c_void_p(weight_sum.data_ptr()), C.c_void_p(g.data_ptr()),
                                               _i3(dims), radius, beta, eta,
                                               C.c_void_p(torch.cuda.current_stream(g.device).cuda_stream))
    _check_free(st, "ccpr_filter_project_grad_edges")
    return g


def nondiscreteness(rho_projected) -> float:
    """ccpr_nondiscreteness (per cent); synchronises to return the value."""
    import torch
    if not (rho_projected.is_cuda and rho_projected.dtype == torch.float32 and rho_projected.is_contiguous()):
        raise ValueError("rho_projected must be a contiguous float32 CUDA tensor")
    out = torch.empty(1, dtype=torch.float64, device=rho_projected.device)
    st = load().ccpr_nondiscreteness(C.c_void_p(rho_projected.data_ptr()), rho_projected.numel(),
                                     C.c_void_p(out.data_ptr()),
                                     C.c_void_p(torch.cuda.current_stream(out.device).cuda_stream))
    _check_free(st, "ccpr_nondiscreteness")
    return float(out.item())


class Solver:
    """One solver handle.  Methods mirror the C-ABI one to one."""

    def __init__(self, nx, ny, nz, dx, courant=0.5, npml=0, pml_order=3.0, pml_kappa_max=1.0,
                 pml_alpha_max=0.05, pml_sigma_scale=1.0):
        self._lib = load()
        g = CcprGrid(nx, ny, nz, dx, courant, npml, pml_order, pml_kappa_max, pml_alpha_max,
                     pml_sigma_scale)
        h = _p()
        st = self._lib.ccpr_create(C.byref(g), C.byref(h))
        if st != OK:
            raise CcprError(st, "ccpr_create", self._lib.ccpr_last_error(None).decode())
        self._h = h
        self.shape = (nz, ny, nx)
        self._keep = []
        self.design_dims = None
        self.per_edge = False
        self._bound_stream = None   # torch stream the workspace was bound with

    # -- plumbing
    def _chk(self, st, what):
        if st != OK:
            raise CcprError(st, what, self._lib.ccpr_last_error(self._h).decode())

    @contextlib.contextmanager
    def _ordered(self):
        """The library enqueues on the stream bound with the workspace.  When
        torch's current stream is another one, order the bound stream after
        the work already on the current stream (device inputs) and the current
        stream after the call's work (device outputs)."""
        bs = self._bound_stream
        if bs is None:
            yield
            return
        import torch
        cur = torch.cuda.current_stream(bs.device)
        other = cur.cuda_stream != bs.cuda_stream
        if other:
            bs.wait_stream(cur)
        try:
            yield
        finally:
            if other:
                cur.wait_stream(bs)

    def close(self):
        if getattr(self, "_h", None):
            self._lib.ccpr_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def handle(self):
        return self._h

    # -- configuration
    def set_material(self, slot, axis, eps_inf, sigma=0.0, a=(), c=()):
        a = np.asarray(a, dtype=np.complex128).ravel()
        c = np.asarray(c, dtype=np.complex128).ravel()
        aa, ap = _f64(np.stack([a.real, a.imag], -1).ravel() if a.size else np.zeros(2))
        cc, cp = _f64(np.stack([c.real, c.imag], -1).ravel() if c.size else np.zeros(2))
        self._chk(self._lib.ccpr_set_material(self._h, slot, axis, eps_inf, sigma, a.size, ap, cp),
                  "ccpr_set_material")

    def set_design(self, lo, rho, gamma=0.0):
        """rho: numpy float32 (dz, dy, dx) on the host, or a torch float32 CUDA tensor."""
        if hasattr(rho, "data_ptr") and getattr(rho, "is_cuda", False):
            import torch
            assert rho.dtype == torch.float32 and rho.is_contiguous() and rho.dim() == 3
            dims = (rho.shape[2], rho.shape[1], rho.shape[0])
            with self._ordered():
                self._chk(self._lib.ccpr_set_design(self._h, _i3(lo), _i3(dims), gamma,
                                                    C.c_void_p(rho.data_ptr()), MEM_DEVICE),
                          "ccpr_set_design")
        else:
            r = np.ascontiguousarray(rho, dtype=np.float32)
            dims = (r.shape[2], r.shape[1], r.shape[0])
            self._chk(self._lib.ccpr_set_design(self._h, _i3(lo), _i3(dims), gamma,
                                                r.ctypes.data_as(C.c_void_p), MEM_HOST),
                      "ccpr_set_design")
        self.design_dims = dims
        self.per_edge = False

    def set_design_edges(self, lo, dims, rho_edges, gamma=0.0):
        """One density per E edge of a design of dims = (Nx, Ny, Nz) cells:
        rho_edges = (rho_x, rho_y, rho_z) host float32 arrays shaped
        edge_shape(dims, c), or one flat torch float32 CUDA tensor holding
        the x, y, z edges in turn."""
        dims = tuple(int(d) for d in dims)
        n = sum(int(np.prod(edge_shape(dims, c))) for c in range(3))
        if hasattr(rho_edges, "data_ptr") and getattr(rho_edges, "is_cuda", False):
            import torch
            assert rho_edges.dtype == torch.float32 and rho_edges.is_contiguous() and rho_edges.numel() == n
            with self._ordered():
                self._chk(self._lib.ccpr_set_design_edges(self._h, _i3(lo), _i3(dims), gamma,
                                                          C.c_void_p(rho_edges.data_ptr()), MEM_DEVICE),
                          "ccpr_set_design_edges")
        else:
            parts = []
            for c in range(3):
                r = np.asarray(rho_edges[c], dtype=np.float32)
                if r.shape != edge_shape(dims, c):
                    raise ValueError(f"edge densities of component {c}: shape {r.shape}, "
                                     f"expected {edge_shape(dims, c)}")
                parts.append(r.ravel())
            flat = np.ascontiguousarray(np.concatenate(parts))
            self._chk(self._lib.ccpr_set_design_edges(self._h, _i3(lo), _i3(dims), gamma,
                                                      flat.ctypes.data_as(C.c_void_p), MEM_HOST),
                      "ccpr_set_design_edges")
        self.design_dims = dims
        self.per_edge = True

    @property
    def gradient_size(self) -> int:
        """Number of gradient values: voxels, or design edges."""
        d = self.design_dims
        if self.per_edge:
            return sum(int(np.prod(edge_shape(d, c))) for c in range(3))
        return int(np.prod(d))

    def split_edges(self, flat):
        """Flat per-edge values -> (x, y, z) arrays shaped edge_shape(dims, c)."""
        out, o = [], 0
        for c in range(3):
            shp = edge_shape(self.design_dims, c)
            k = int(np.prod(shp))
            out.append(flat[o:o + k].reshape(shp))
            o += k
        return tuple(out)

    def set_source_dipole(self, cell, axis, wave):
        w, wp = _f64(wave)
        self._chk(self._lib.ccpr_set_source_dipole(self._h, _i3(cell), axis, wp, w.size),
                  "ccpr_set_source_dipole")

    def set_source_planewave(self, prop_axis, sign, pol_axis, lo, hi, wave):
        w, wp = _f64(wave)
        self._chk(self._lib.ccpr_set_source_planewave(self._h, prop_axis, sign, pol_axis, _i3(lo),
                                                      _i3(hi), wp, w.size),
                  "ccpr_set_source_planewave")

    def set_objective(self, kind, lo, dims, omega=0.0, n_begin=0, n_end=-1):
        self._chk(self._lib.ccpr_set_objective(self._h, kind, _i3(lo), _i3(dims), omega, n_begin,
                                               n_end), "ccpr_set_objective")

    def set_checkpointing(self, every):
        self._chk(self._lib.ccpr_set_checkpointing(self._h, every), "ccpr_set_checkpointing")

    def set_resident_segments(self, max_resident):
        """At most this many segments keep the forward history (0: as many as fit)."""
        self._chk(self._lib.ccpr_set_resident_segments(self._h, max_resident), "ccpr_set_resident_segments")

    def set_gradient_mode(self, mode):
        """"time" (exact discrete gradient, default) or "dft" (single-frequency
        estimator for the DFT objective)."""
        code = {"time": GRAD_TIME_EXACT, "dft": GRAD_DFT}[mode]
        self._chk(self._lib.ccpr_set_gradient_mode(self._h, code), "ccpr_set_gradient_mode")

    def workspace_size(self, nsteps):
        b = C.c_uint64(0)
        self._chk(self._lib.ccpr_workspace_size(self._h, nsteps, C.byref(b)), "ccpr_workspace_size")
        return int(b.value)

    def workspace_size_max(self, nsteps):
        b = C.c_uint64(0)
        self._chk(self._lib.ccpr_workspace_size_max(self._h, nsteps, C.byref(b)), "ccpr_workspace_size_max")
        return int(b.value)

    def bind_workspace(self, ptr: int, nbytes: int, stream: int = 0):
        self._chk(self._lib.ccpr_bind_workspace(self._h, C.c_void_p(ptr), nbytes, C.c_void_p(stream)),
                  "ccpr_bind_workspace")
        self._bound_stream = None

    def bind_static_workspace(self, stream: int = 0):
        """ccpr_bind_static_workspace: the library's static 64 MiB device array
        of the current device as workspace (no allocation), with a raw HIP
        stream handle (0: the null stream)."""
        self._chk(self._lib.ccpr_bind_static_workspace(self._h, C.c_void_p(stream)),
                  "ccpr_bind_static_workspace")
        self._bound_stream = None
        self._ws = None

    def bind_torch(self, nsteps: int, device=None, extra: int = 0, reserve: int = 4 << 30,
                   greedy: bool = True):
        """Allocate the workspace as a torch uint8 CUDA tensor and bind it with
        torch's current stream on that device.  It takes what the solve can use
        (ccpr_workspace_size_max: every checkpointed segment's history resident;
        greedy=False: only ccpr_workspace_size) up to the device's free memory
        less 'reserve' bytes; with less, the library keeps as many segments
        resident as fit and recomputes the others (or, with
        ccpr_set_checkpointing(0), the default, picks the segmentation that
        recomputes least)."""
        import torch
        dev = torch.device(device or "cuda")
        want = self.workspace_size_max(nsteps) if greedy else 0
        nbytes = max(self.workspace_size(nsteps), want) + extra
        free, _ = torch.cuda.mem_get_info(dev)
        if nbytes > free - reserve:
            nbytes = max(free - reserve, 1 << 20)
        ws = torch.empty(nbytes, dtype=torch.uint8, device=dev)
        stream = torch.cuda.current_stream(dev)
        self.bind_workspace(ws.data_ptr(), nbytes, stream.cuda_stream)
        self._bound_stream = stream
        self._ws = ws
        return ws

    # -- running
    def forward(self, nsteps) -> float:
        F = C.c_double(0.0)
        with self._ordered():
            self._chk(self._lib.ccpr_forward(self._h, nsteps, C.byref(F)), "ccpr_forward")
        return F.value

    def adjoint(self):
        with self._ordered():
            self._chk(self._lib.ccpr_adjoint(self._h), "ccpr_adjoint")

    @property
    def forward_serial(self) -> int:
        """Serial of the forward run the next adjoint would use (-1: none)."""
        return int(self._lib.ccpr_forward_serial(self._h))

    def set_watchdog(self, every: int = 128, limit: float = 1e15):
        """Divergence watchdog: check the gap box every 'every' steps (0: off)."""
        self._chk(self._lib.ccpr_set_watchdog(self._h, int(every), float(limit)), "ccpr_set_watchdog")

    def gap_spectrum(self, omegas):
        """Mean |E_hat(omega)|^2 over the gap edges of the last forward run, for
        each angular frequency in omegas (numpy float64)."""
        w, wp = _f64(np.atleast_1d(omegas))
        out = np.zeros(w.size, dtype=np.float64)
        self._chk(self._lib.ccpr_gap_spectrum(self._h, wp, w.size, out.ctypes.data_as(_dp)),
                  "ccpr_gap_spectrum")
        return out

    def gradient(self, out=None):
        """Host numpy (dz,dy,dx) float64 by default (per-edge designs: the
        (x, y, z) edge arrays); pass a torch float64 CUDA tensor of
        gradient_size values to receive it on the device (stream-ordered)."""
        d = self.design_dims
        if out is not None and getattr(out, "is_cuda", False):
            if out.numel() != self.gradient_size:
                raise ValueError(f"gradient output holds {out.numel()} values, need {self.gradient_size}")
            with self._ordered():
                self._chk(self._lib.ccpr_gradient(self._h, C.c_void_p(out.data_ptr()), MEM_DEVICE),
                          "ccpr_gradient")
            return out
        g = np.empty(self.gradient_size, dtype=np.float64)
        self._chk(self._lib.ccpr_gradient(self._h, g.ctypes.data_as(C.c_void_p), MEM_HOST),
                  "ccpr_gradient")
        return self.split_edges(g) if self.per_edge else g.reshape(d[2], d[1], d[0])

    def reset(self):
        with self._ordered():
            self._chk(self._lib.ccpr_reset(self._h), "ccpr_reset")

    def step(self, n=1):
        with self._ordered():
            self._chk(self._lib.ccpr_step(self._h, int(n)), "ccpr_step")

    def field(self, comp, out=None):
        if out is not None and getattr(out, "is_cuda", False):
            with self._ordered():
                self._chk(self._lib.ccpr_get_field(self._h, comp, C.c_void_p(out.data_ptr()), MEM_DEVICE),
                          "ccpr_get_field")
            return out
        f = np.empty(self.shape, dtype=np.float32)
        self._chk(self._lib.ccpr_get_field(self._h, comp, f.ctypes.data_as(C.c_void_p), MEM_HOST),
                  "ccpr_get_field")
        return f

    @property
    def step_count(self):
        return self._lib.ccpr_step_count(self._h)

    # -- diagnostics
    def set_timing(self, on=True, every: int = 1):
        """Event timing of the loops and of every 'every'-th grid pass."""
        self._chk(self._lib.ccpr_set_timing(self._h, max(1, int(every)) if on else 0), "ccpr_set_timing")

    def timing(self):
        ms = C.c_double(0.0)
        n = C.c_longlong(0)
        self._chk(self._lib.ccpr_get_timing(self._h, C.byref(ms), C.byref(n)), "ccpr_get_timing")
        return ms.value, n.value

    def grid_timing(self):
        """(total ms, launches) of the grid kernel inside the timed loops."""
        ms = C.c_double(0.0)
        n = C.c_longlong(0)
        self._chk(self._lib.ccpr_get_grid_timing(self._h, C.byref(ms), C.byref(n)), "ccpr_get_grid_timing")
        return ms.value, n.value

    def info(self):
        a, b, c = C.c_int(0), C.c_int(0), C.c_int(0)
        self._chk(self._lib.ccpr_get_info(self._h, C.byref(a), C.byref(b), C.byref(c)),
                  "ccpr_get_info")
        r = C.c_int(0)
        self._chk(self._lib.ccpr_get_resident_segments(self._h, C.byref(r)), "ccpr_get_resident_segments")
        f = C.c_int(0)
        self._chk(self._lib.ccpr_get_design_fusion(self._h, C.byref(f)), "ccpr_get_design_fusion")
        return {"segments": a.value, "segment_steps": b.value, "tile_planes": c.value,
                "resident_segments": r.value, "design_fused": f.value}

    def set_tile_planes(self, planes):
        self._chk(self._lib.ccpr_set_tile_planes(self._h, planes), "ccpr_set_tile_planes")

    def set_tile_rows(self, rows):
        self._chk(self._lib.ccpr_set_tile_rows(self._h, rows), "ccpr_set_tile_rows")

    def set_design_fusion(self, on: bool):
        """Let the grid pass finish the design cells itself where it can
        (default), or always leave them to the separate design pass."""
        self._chk(self._lib.ccpr_set_design_fusion(self._h, 1 if on else 0), "ccpr_set_design_fusion")


class Engine:
    """Serving engine (ccpr_engine_*): continuous batching of whole solves.

    The arena is a torch uint8 CUDA tensor owned by this object; the engine
    sub-allocates the solves' workspaces from it.  Solvers passed to submit()
    are kept alive here until their job is released."""

    def __init__(self, arena_bytes: int, max_active: int = 4, chunk_steps: int = 32, device=None,
                 batching: bool = True):
        import torch
        self._lib = load()
        self._arena = torch.empty(int(arena_bytes), dtype=torch.uint8, device=torch.device(device or "cuda"))
        h = _p()
        st = self._lib.ccpr_engine_create(C.c_void_p(self._arena.data_ptr()), int(arena_bytes), max_active,
                                          chunk_steps, C.byref(h))
        if st != OK:
            raise CcprError(st, "ccpr_engine_create", "bad engine arguments")
        self._h = h
        self._solvers = {}
        if not batching:
            self._chk(self._lib.ccpr_engine_set_batching(self._h, 0), "ccpr_engine_set_batching")

    def _chk(self, st, what):
        if st != OK:
            raise CcprError(st, what, self._lib.ccpr_engine_last_error(self._h).decode())

    def submit(self, solver: Solver, nsteps: int) -> int:
        t = C.c_uint64(0)
        self._chk(self._lib.ccpr_engine_submit(self._h, solver.handle, int(nsteps), C.byref(t)),
                  "ccpr_engine_submit")
        self._solvers[t.value] = solver
        return t.value

    def poll(self, ticket: int) -> int:
        st = C.c_int(0)
        self._chk(self._lib.ccpr_engine_poll(self._h, ticket, C.byref(st)), "ccpr_engine_poll")
        return st.value

    def wait(self, ticket: int) -> int:
        st = C.c_int(0)
        self._chk(self._lib.ccpr_engine_wait(self._h, ticket, C.byref(st)), "ccpr_engine_wait")
        return st.value

    def result(self, ticket: int):
        """(objective, gradient (dz, dy, dx) float64, (submitted, admitted, done)
        in seconds since the engine was created)."""
        s = self._solvers[ticket]
        d = s.design_dims
        g = np.empty(s.gradient_size, dtype=np.float64)
        F = C.c_double(0.0)
        times = (C.c_double * 3)()
        self._chk(self._lib.ccpr_engine_result(self._h, ticket, C.byref(F), g.ctypes.data_as(_dp), times),
                  "ccpr_engine_result")
        g = s.split_edges(g) if s.per_edge else g.reshape(d[2], d[1], d[0])
        return F.value, g, tuple(times)

    def release(self, ticket: int):
        self._chk(self._lib.ccpr_engine_release(self._h, ticket), "ccpr_engine_release")
        self._solvers.pop(ticket, None)

    def close(self):
        if getattr(self, "_h", None):
            self._lib.ccpr_engine_destroy(self._h)
            self._h = None
            self._arena = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
