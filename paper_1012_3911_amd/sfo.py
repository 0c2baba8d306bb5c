"""Python binding of libsfo (the gfx950 split-operator library).

Argument marshalling only: every step of the method runs in the HIP kernels
behind the C ABI declared in include/sfo.h.  PyTorch supplies device memory
and the stream.  The binding fails loudly when the library is missing or no
GPU is present; there is no CPU fallback.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libsfo.so")

SFO_OK, SFO_E_INVALID, SFO_E_UNSUPPORTED, SFO_E_NOMEM, SFO_E_HIP, SFO_E_STATE, SFO_E_NUMERIC = 0, -1, -2, -3, -4, -5, -6
SCHRODINGER, DIRAC = 0, 1
C64, C128 = 0, 1
UNFUSED = 1 << 1

_STATUS_NAMES = {0: "SFO_OK", -1: "SFO_E_INVALID", -2: "SFO_E_UNSUPPORTED", -3: "SFO_E_NOMEM",
                 -4: "SFO_E_HIP", -5: "SFO_E_STATE", -6: "SFO_E_NUMERIC"}


class SfoError(RuntimeError):
    def __init__(self, status: int, where: str, message: str):
        self.status = status
        super().__init__("%s failed: %s: %s" % (where, _STATUS_NAMES.get(status, status), message))


class GridDesc(ctypes.Structure):
    _fields_ = [
        ("ndim", ctypes.c_int32),
        ("n", ctypes.c_int64 * 3),
        ("xmin", ctypes.c_double * 3),
        ("xmax", ctypes.c_double * 3),
        ("equation", ctypes.c_int32),
        ("dtype", ctypes.c_int32),
        ("dt", ctypes.c_double),
        ("mass", ctypes.c_double),
        ("charge", ctypes.c_double),
        ("c", ctypes.c_double),
        ("hbar", ctypes.c_double),
        ("flags", ctypes.c_uint32),
    ]


_lib = None

EXPORTS = ["sfo_create_grid", "sfo_destroy_grid", "sfo_set_potential", "sfo_set_field",
           "sfo_set_vector_potential", "sfo_step", "sfo_propagate", "sfo_adjoint", "sfo_norm",
           "sfo_overlap", "sfo_fft", "sfo_create_batch", "sfo_destroy_batch", "sfo_propagate_batch",
           "sfo_adjoint_batch", "sfo_batch_set_graph", "sfo_batch_check", "sfo_batch_autotune", "sfo_autotune",
           "sfo_get_plan",
           "sfo_set_plan", "sfo_profile_enable", "sfo_profile_read", "sfo_time_pass", "sfo_autocorrelation",
           "sfo_spectrum", "sfo_set_vector_field", "sfo_eigenfunction", "sfo_adjoint_noalloc", "sfo_set_norm_watch", "sfo_adjoint_velocity", "sfo_last_error",
           "sfo_version"]

KERNEL_ROW, KERNEL_COLUMN, KERNEL_ZCOLUMN, KERNEL_LINE1D = 0, 1, 2, 3
TIME_IN_STEP = 16  # or'ed into a kernel kind: time the pass within whole steps


def load_library(path: str = LIB_PATH):
    """Load libsfo.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError("libsfo.so is not built (%s); run __graft_entry__.build()" % path)
    lib = ctypes.CDLL(path)
    P, I64, I32 = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32
    sig = {
        "sfo_create_grid": [ctypes.POINTER(GridDesc), P, ctypes.POINTER(P)],
        "sfo_destroy_grid": [P],
        "sfo_set_potential": [P, P],
        "sfo_set_field": [P, P, I64],
        "sfo_set_vector_potential": [P, P, I64],
        "sfo_step": [P, P, I64],
        "sfo_propagate": [P, P, I64, I64],
        "sfo_adjoint": [P, P, P, I64, I64, P, P],
        "sfo_adjoint_noalloc": [P, P, P, I64, I64, P, P],
        "sfo_adjoint_velocity": [P, P, P, I64, I64, P, P, P],
        "sfo_norm": [P, P, P],
        "sfo_set_norm_watch": [P, ctypes.c_double, ctypes.c_double],
        "sfo_overlap": [P, P, P, P],
        "sfo_fft": [P, P, I32],
        "sfo_autotune": [P, I32],
        "sfo_get_plan": [P, P],
        "sfo_set_plan": [P, P],
        "sfo_profile_enable": [P, I32],
        "sfo_profile_read": [P, I32, P, P],
        "sfo_time_pass": [P, I32, I32, P],
        "sfo_autocorrelation": [P, P, I64, P],
        "sfo_spectrum": [P, P, I64, P, I32, P],
        "sfo_set_vector_field": [P, P, P, I64],
        "sfo_eigenfunction": [P, P, I64, ctypes.c_double, P],
        "sfo_create_batch": [P, I32, P, ctypes.POINTER(P)],
        "sfo_destroy_batch": [P],
        "sfo_propagate_batch": [P, P, I64, I64],
        "sfo_adjoint_batch": [P, P, P, I64, I64, P, P],
        "sfo_batch_set_graph": [P, I32],
        "sfo_batch_check": [P],
        "sfo_batch_autotune": [P, I32],
    }
    for name, args in sig.items():
        f = getattr(lib, name)
        f.argtypes = args
        f.restype = ctypes.c_int
    lib.sfo_last_error.restype = ctypes.c_char_p
    lib.sfo_last_error.argtypes = []
    lib.sfo_version.restype = ctypes.c_char_p
    lib.sfo_version.argtypes = []
    _lib = lib
    return lib


def _check(rc: int, where: str):
    if rc != SFO_OK:
        raise SfoError(rc, where, _lib.sfo_last_error().decode())


def _torch():
    import torch

    return torch


class Grid:
    """A grid handle bound to one CUDA/HIP stream (torch's current stream by default)."""

    def __init__(self, n: Sequence[int], xmin: Sequence[float], xmax: Sequence[float], dt: float, *,
                 dtype: str = "c128", equation: str = "schrodinger", mass: float = 1.0,
                 charge: float = -1.0, c: float = 137.036, hbar: float = 1.0, flags: int = 0,
                 stream=None):
        torch = _torch()
        lib = load_library()
        if not torch.cuda.is_available():
            raise RuntimeError("sfo needs a GPU (torch.cuda.is_available() is False)")
        d = GridDesc()
        d.ndim = len(n)
        for a in range(3):
            d.n[a] = int(n[a]) if a < len(n) else 1
            d.xmin[a] = float(xmin[a]) if a < len(n) else 0.0
            d.xmax[a] = float(xmax[a]) if a < len(n) else 1.0
        d.equation = {"schrodinger": SCHRODINGER, "dirac": DIRAC}[equation]
        d.dtype = {"c64": C64, "c128": C128}[dtype]
        d.dt, d.mass, d.charge, d.c, d.hbar, d.flags = dt, mass, charge, c, hbar, flags
        self.desc = d
        self.n = tuple(int(x) for x in n)
        self.ndim = len(n)
        self.ncomp = (2 if len(n) == 1 else 4) if equation == "dirac" else 1
        self.dtype = dtype
        self.torch_dtype = torch.complex64 if dtype == "c64" else torch.complex128
        self.stream = stream if stream is not None else torch.cuda.current_stream()
        h = ctypes.c_void_p()
        _check(lib.sfo_create_grid(ctypes.byref(d), ctypes.c_void_p(self.stream.cuda_stream), ctypes.byref(h)),
               "sfo_create_grid")
        self._h = h
        self.shape = ((self.ncomp,) if self.ncomp > 1 else ()) + self.n[::-1]
        self._keep = []
        self.tables_version = 0  # counts successful potential / field installs

    def close(self):
        if getattr(self, "_h", None) and self._h.value:
            _check(_lib.sfo_destroy_grid(self._h), "sfo_destroy_grid")
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ------------------------------------------------------------- helpers --
    def _state(self, psi, name="psi"):
        torch = _torch()
        if not isinstance(psi, torch.Tensor) or not psi.is_cuda:
            raise TypeError("%s must be a CUDA tensor" % name)
        if psi.dtype != self.torch_dtype or not psi.is_contiguous() or tuple(psi.shape) != self.shape:
            raise ValueError("%s must be a contiguous %s tensor of shape %s (got %s %s)"
                             % (name, self.torch_dtype, self.shape, psi.dtype, tuple(psi.shape)))
        return ctypes.c_void_p(psi.data_ptr())

    # ----------------------------------------------------------------- API --
    def set_potential(self, V0):
        torch = _torch()
        v = torch.as_tensor(V0, dtype=torch.float64, device="cuda").contiguous()
        if v.numel() != int(np.prod(self.n)):
            raise ValueError("V0 must have %d values" % int(np.prod(self.n)))
        with torch.cuda.stream(self.stream):
            _check(_lib.sfo_set_potential(self._h, ctypes.c_void_p(v.data_ptr())), "sfo_set_potential")
        self.tables_version += 1
        self._keep = [v]  # the copy is enqueued on the stream; keep the source alive until it runs

    def set_field(self, ebar: Optional[np.ndarray]):
        if ebar is None:
            _check(_lib.sfo_set_field(self._h, None, 0), "sfo_set_field")
            self.tables_version += 1
            return
        e = np.ascontiguousarray(ebar, dtype=np.float64)
        if e.ndim != 2 or e.shape[1] != self.ndim:
            raise ValueError("ebar must have shape (nsteps, %d)" % self.ndim)
        _check(_lib.sfo_set_field(self._h, e.ctypes.data_as(ctypes.c_void_p), e.shape[0]), "sfo_set_field")
        self.tables_version += 1

    def set_vector_field(self, abar: Optional[np.ndarray], a2bar: Optional[np.ndarray] = None):
        """Velocity gauge: per-step integrals of A(t) (nsteps, ndim) and of |A|^2 (nsteps,)."""
        self.tables_version += 1  # a failed call may have released the field (sfo.h)
        if abar is None:
            _check(_lib.sfo_set_vector_field(self._h, None, None, 0), "sfo_set_vector_field")
            return
        a = np.ascontiguousarray(abar, dtype=np.float64)
        a2 = np.ascontiguousarray(a2bar, dtype=np.float64)
        if a.ndim != 2 or a.shape[1] != self.ndim or a2.shape != (a.shape[0],):
            raise ValueError("abar must have shape (nsteps, %d) and a2bar (nsteps,)" % self.ndim)
        _check(_lib.sfo_set_vector_field(self._h, a.ctypes.data_as(ctypes.c_void_p),
                                         a2.ctypes.data_as(ctypes.c_void_p), a.shape[0]), "sfo_set_vector_field")

    def set_vector_potential(self, abar_y: Optional[np.ndarray]):
        if abar_y is None:
            _check(_lib.sfo_set_vector_potential(self._h, None, 0), "sfo_set_vector_potential")
            return
        a = np.ascontiguousarray(abar_y, dtype=np.float64)
        if a.ndim != 2 or a.shape[1] != self.n[0]:
            raise ValueError("abar_y must have shape (nsteps, %d)" % self.n[0])
        _check(_lib.sfo_set_vector_potential(self._h, a.ctypes.data_as(ctypes.c_void_p), a.shape[0]),
               "sfo_set_vector_potential")

    def step(self, psi, step_index: int):
        _check(_lib.sfo_step(self._h, self._state(psi), int(step_index)), "sfo_step")

    def propagate(self, psi, step0: int, nsteps: int):
        _check(_lib.sfo_propagate(self._h, self._state(psi), int(step0), int(nsteps)), "sfo_propagate")

    def autocorrelation(self, psi, nsteps: int):
        """Advance psi by nsteps steps (no field) and return chi_j = <psi_0|psi_j>,
        j < nsteps, as a complex128 CUDA tensor."""
        torch = _torch()
        chi = torch.empty(2 * int(nsteps), dtype=torch.float64, device="cuda")
        _check(_lib.sfo_autocorrelation(self._h, self._state(psi), int(nsteps),
                                        ctypes.c_void_p(chi.data_ptr())), "sfo_autocorrelation")
        return torch.view_as_complex(chi.view(-1, 2))

    def eigenfunction(self, psi, nsteps: int, energy: float):
        """Advance psi by nsteps steps (no field) and return the windowed sum
        sum_j dt w_j exp(i E j dt / hbar) psi_j (unnormalised) as a new state tensor."""
        torch = _torch()
        out = torch.empty_like(psi)
        _check(_lib.sfo_eigenfunction(self._h, self._state(psi), int(nsteps), float(energy), self._state(out, "out")),
               "sfo_eigenfunction")
        return out

    def spectrum(self, chi, energies):
        """Windowed transform of an autocorrelation at the given energies (complex128 CUDA tensor)."""
        torch = _torch()
        c = torch.view_as_real(chi.to(torch.complex128)).contiguous().view(-1)
        E = torch.as_tensor(energies, dtype=torch.float64, device="cuda").contiguous()
        out = torch.empty(2 * E.numel(), dtype=torch.float64, device="cuda")
        _check(_lib.sfo_spectrum(self._h, ctypes.c_void_p(c.data_ptr()), c.numel() // 2,
                                 ctypes.c_void_p(E.data_ptr()), int(E.numel()),
                                 ctypes.c_void_p(out.data_ptr())), "sfo_spectrum")
        return torch.view_as_complex(out.view(-1, 2))

    def adjoint(self, psi, g, step0: int, nsteps: int, want_dV0: bool = True):
        torch = _torch()
        de = torch.zeros((nsteps, self.ndim), dtype=torch.float64, device="cuda")
        dv = torch.zeros(self.n[::-1], dtype=torch.float64, device="cuda") if want_dV0 else None
        _check(_lib.sfo_adjoint(self._h, self._state(psi), self._state(g, "g"), int(step0), int(nsteps),
                                ctypes.c_void_p(de.data_ptr()),
                                ctypes.c_void_p(dv.data_ptr()) if dv is not None else None), "sfo_adjoint")
        return de, dv

    def adjoint_velocity(self, psi, g, step0: int, nsteps: int, want_dV0: bool = True):
        """Reverse sweep of a velocity-gauge run: returns (dL/dAbar (nsteps, ndim), dL/dA2bar (nsteps,),
        dL/dV0 or None) as FP64 CUDA tensors."""
        torch = _torch()
        da = torch.zeros((nsteps, self.ndim), dtype=torch.float64, device="cuda")
        da2 = torch.zeros(nsteps, dtype=torch.float64, device="cuda")
        dv = torch.zeros(self.n[::-1], dtype=torch.float64, device="cuda") if want_dV0 else None
        _check(_lib.sfo_adjoint_velocity(self._h, self._state(psi), self._state(g, "g"), int(step0), int(nsteps),
                                         ctypes.c_void_p(da.data_ptr()), ctypes.c_void_p(da2.data_ptr()),
                                         ctypes.c_void_p(dv.data_ptr()) if dv is not None else None),
               "sfo_adjoint_velocity")
        return da, da2, dv

    def adjoint_noalloc(self, psi, g, step0: int, nsteps: int, de, dv=None):
        """sfo_adjoint_noalloc into caller-allocated outputs de (nsteps x ndim FP64) and dv (N points FP64 or None)."""
        _check(_lib.sfo_adjoint_noalloc(self._h, self._state(psi), self._state(g, "g"), int(step0), int(nsteps),
                                        ctypes.c_void_p(de.data_ptr()),
                                        ctypes.c_void_p(dv.data_ptr()) if dv is not None else None),
               "sfo_adjoint_noalloc")
        return de, dv

    def set_norm_watch(self, reference: float, tolerance: float):
        """sfo_norm then raises (SFO_E_NUMERIC) once |norm/reference - 1| > tolerance; reference 0 = off."""
        _check(_lib.sfo_set_norm_watch(self._h, float(reference), float(tolerance)), "sfo_set_norm_watch")

    def norm(self, psi) -> float:
        out = ctypes.c_double()
        _check(_lib.sfo_norm(self._h, self._state(psi), ctypes.byref(out)), "sfo_norm")
        return out.value

    def overlap(self, a, b) -> complex:
        out = (ctypes.c_double * 2)()
        _check(_lib.sfo_overlap(self._h, self._state(a, "a"), self._state(b, "b"), out), "sfo_overlap")
        return complex(out[0], out[1])

    def autotune(self, reps: int = 20):
        _check(_lib.sfo_autotune(self._h, int(reps)), "sfo_autotune")
        return self.plan

    @property
    def plan(self):
        out = (ctypes.c_int32 * 3)()
        _check(_lib.sfo_get_plan(self._h, out), "sfo_get_plan")
        return tuple(out)

    @plan.setter
    def plan(self, p):
        arr = (ctypes.c_int32 * 3)(*[int(x) for x in p])
        _check(_lib.sfo_set_plan(self._h, arr), "sfo_set_plan")

    def profile(self, on: bool = True):
        _check(_lib.sfo_profile_enable(self._h, 1 if on else 0), "sfo_profile_enable")

    def profile_read(self, kind: int):
        """(launch count, summed milliseconds) of one kernel kind since profiling was enabled."""
        cnt = ctypes.c_int64()
        ms = ctypes.c_double()
        _check(_lib.sfo_profile_read(self._h, int(kind), ctypes.byref(cnt), ctypes.byref(ms)),
               "sfo_profile_read")
        return cnt.value, ms.value

    def time_pass(self, kind: int, reps: int = 100, in_step: bool = False) -> float:
        """Average milliseconds per launch of one pass shape: from back-to-back
        launches of that pass, or (in_step) within steps of the propagation's
        pass sequence, each launch timestamped by its own dispatch."""
        ms = ctypes.c_double()
        k = int(kind) | (TIME_IN_STEP if in_step else 0)
        _check(_lib.sfo_time_pass(self._h, k, int(reps), ctypes.byref(ms)), "sfo_time_pass")
        return ms.value

    def fft(self, psi, sign: int = -1):
        _check(_lib.sfo_fft(self._h, self._state(psi), int(sign)), "sfo_fft")


class Batch:
    """Many independent Schroedinger grids (1-D and 2-D) advanced together.

    The grids (all of one dtype) keep their own box, time step, potential and
    field table.  Each pass is launched once per group of same-shape grids;
    the batch runs on one stream (torch's current stream by default) and
    replays a captured HIP graph per (direction, step0, nsteps).
    """

    def __init__(self, grids: Sequence[Grid], stream=None, graph: bool = True):
        torch = _torch()
        lib = load_library()
        if not grids:
            raise ValueError("a batch needs at least one grid")
        self.grids = list(grids)
        self.stream = stream if stream is not None else torch.cuda.current_stream()
        arr = (ctypes.c_void_p * len(grids))(*[g._h.value for g in grids])
        h = ctypes.c_void_p()
        _check(lib.sfo_create_batch(arr, len(grids), ctypes.c_void_p(self.stream.cuda_stream), ctypes.byref(h)),
               "sfo_create_batch")
        self._h = h
        if not graph:
            _check(lib.sfo_batch_set_graph(self._h, 0), "sfo_batch_set_graph")

    def close(self):
        if getattr(self, "_h", None) and self._h.value:
            _check(_lib.sfo_destroy_batch(self._h), "sfo_destroy_batch")
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _ptrs(self, states, name):
        if len(states) != len(self.grids):
            raise ValueError("%s: need %d states, got %d" % (name, len(self.grids), len(states)))
        return (ctypes.c_void_p * len(states))(*[g._state(x, name).value for g, x in zip(self.grids, states)])

    def set_graph(self, on: bool):
        _check(_lib.sfo_batch_set_graph(self._h, 1 if on else 0), "sfo_batch_set_graph")

    def autotune(self, reps: int = 10):
        _check(_lib.sfo_batch_autotune(self._h, int(reps)), "sfo_batch_autotune")

    def propagate(self, psis, step0: int, nsteps: int):
        _check(_lib.sfo_propagate_batch(self._h, self._ptrs(psis, "psi"), int(step0), int(nsteps)),
               "sfo_propagate_batch")

    def adjoint(self, psis, gs, step0: int, nsteps: int, want_dV0: bool = True):
        """Reverse sweep of every problem; returns (list of dL/dEbar, list of dL/dV0 or None)."""
        torch = _torch()
        des = [torch.zeros((nsteps, g.ndim), dtype=torch.float64, device="cuda") for g in self.grids]
        dvs = [torch.zeros(g.n[::-1], dtype=torch.float64, device="cuda") for g in self.grids] if want_dV0 else None
        de_arr = (ctypes.c_void_p * len(des))(*[d.data_ptr() for d in des])
        dv_arr = (ctypes.c_void_p * len(dvs))(*[d.data_ptr() for d in dvs]) if dvs is not None else None
        _check(_lib.sfo_adjoint_batch(self._h, self._ptrs(psis, "psi"), self._ptrs(gs, "g"), int(step0),
                                      int(nsteps), de_arr, dv_arr), "sfo_adjoint_batch")
        return des, dvs

    def check(self):
        """Wait for the batch's stream; raise if a launch gave up on a dependency."""
        _check(_lib.sfo_batch_check(self._h), "sfo_batch_check")


def version() -> str:
    return load_library().sfo_version().decode()
