"""Plain FP64 CPU oracle of the Fourier split-operator step (test infrastructure).

Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import this package.  The GPU library never does, and this
package imports nothing from it: the two share no code.  The arithmetic lives
in ``sfo_oracle.c`` (FP64, its own radix-2 FFT); this module only marshals
numpy arrays into it with ctypes.

Arrays use the C order of numpy, so a 3-D state of shape (nz, ny, nx) has x
fastest, matching the flat layout the C file documents.  Grid extents are
given per axis in x, y, z order (``n[0]`` is the x size).

Which passage of the paper each routine follows is stated in the C source;
in short: the Strang step of Sec. 2.1 (eqs. U_split, step_t_to_t+dt_F), the
Schroedinger split of Sec. 2.2 and the Dirac split of Sec. 2.3 (eqs.
exp_alpha, U_A_2_DE).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "sfo_oracle.c")
_LIB = os.path.join(_HERE, "liborc.so")

_lib = None


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (FP64, IEEE semantics, OpenMP)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp%d" % os.getpid()
        cmd = ["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-fopenmp",
               "-fcx-fortran-rules", "-fno-fast-math", "-o", tmp, _SRC, "-lm"]
        subprocess.check_call(cmd)
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB):
        build(force=False)
    lib = ctypes.CDLL(_LIB)
    P = ctypes.c_void_p
    I64 = ctypes.c_int64
    I = ctypes.c_int
    D = ctypes.c_double
    lib.orc_fft.argtypes = [P, I, P, I, I]
    lib.orc_norm.argtypes = [I, P, P, P, I, P, P]
    lib.orc_overlap.argtypes = [I, P, P, P, I, P, P, P]
    lib.orc_schrodinger.argtypes = [I, P, P, P, D, D, D, P, P, P, I64, I64, I, P]
    lib.orc_schrodinger_adjoint.argtypes = [I, P, P, P, D, D, D, P, P, P, P, I64, I64, P, P]
    lib.orc_dirac2d.argtypes = [P, P, P, D, D, D, D, D, P, P, P, I64, I64, I]
    lib.orc_schrodinger_velocity.argtypes = [I, P, P, P, D, D, D, D, P, P, P, P, I64, I64]
    lib.orc_dirac1d.argtypes = [I64, D, D, D, D, D, D, D, P, P, P, I64, I64]
    lib.orc_schrodinger_velocity_adjoint.argtypes = [I, P, P, P, D, D, D, D, P, P, P, P, P, I64, I64, P, P, P]
    lib.orc_num_threads.restype = I
    lib.orc_set_num_threads.argtypes = [I]
    for f in (lib.orc_fft, lib.orc_norm, lib.orc_overlap, lib.orc_schrodinger,
              lib.orc_schrodinger_adjoint, lib.orc_dirac2d, lib.orc_schrodinger_velocity, lib.orc_dirac1d,
              lib.orc_schrodinger_velocity_adjoint):
        f.restype = I
    _lib = lib
    return lib


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def _axes(n, xmin, xmax):
    ndim = len(n)
    nn = np.zeros(3, np.int64)
    lo = np.zeros(3, np.float64)
    hi = np.ones(3, np.float64)
    nn[:ndim] = n
    lo[:ndim] = xmin
    hi[:ndim] = xmax
    return ndim, nn, lo, hi


def _c128(a) -> np.ndarray:
    a = np.ascontiguousarray(a, dtype=np.complex128)
    return a


def _check(rc, what):
    if rc != 0:
        raise RuntimeError("oracle %s failed (rc=%d)" % (what, rc))


def num_threads() -> int:
    return int(_load().orc_num_threads())


def set_num_threads(t: int) -> None:
    _load().orc_set_num_threads(int(t))


def fft(a: np.ndarray, sign: int = -1, ncomp: int = 1) -> np.ndarray:
    """Unnormalised DFT along every spatial axis, exp(sign 2 pi i j m / N).

    ``a`` has shape ([ncomp,] *spatial) with spatial in (z, y, x) order."""
    out = _c128(a).copy()
    spatial = out.shape[1:] if ncomp > 1 else out.shape
    n = np.array(spatial[::-1], np.int64)
    _check(_load().orc_fft(_ptr(out), len(n), _ptr(n), int(sign), int(ncomp)), "fft")
    return out


def norm(psi, n, xmin, xmax, ncomp: int = 1) -> float:
    """dV * sum |psi|^2 over all points and components."""
    ndim, nn, lo, hi = _axes(n, xmin, xmax)
    p = _c128(psi)
    out = np.zeros(1)
    _check(_load().orc_norm(ndim, _ptr(nn), _ptr(lo), _ptr(hi), ncomp, _ptr(p), _ptr(out)), "norm")
    return float(out[0])


def overlap(a, b, n, xmin, xmax, ncomp: int = 1) -> complex:
    """dV * sum conj(a) b."""
    ndim, nn, lo, hi = _axes(n, xmin, xmax)
    pa, pb = _c128(a), _c128(b)
    out = np.zeros(2)
    _check(_load().orc_overlap(ndim, _ptr(nn), _ptr(lo), _ptr(hi), ncomp, _ptr(pa), _ptr(pb),
                               _ptr(out)), "overlap")
    return complex(out[0], out[1])


def schrodinger(psi0, n, xmin, xmax, dt, V0, ebar=None, *, step0=0, nsteps=1, mass=1.0,
                hbar=1.0, direction=1, return_norms=False):
    """Strang steps of the Schroedinger equation (dipole approximation).

    ``ebar`` is the per-step integrated field, shape (total_steps, ndim); the
    potential energy over step n is tau*V0(x) + x.ebar[n].  direction=-1
    undoes the steps (inverse step, last step first)."""
    ndim, nn, lo, hi = _axes(n, xmin, xmax)
    psi = _c128(psi0).copy()
    v = np.ascontiguousarray(V0, dtype=np.float64)
    assert v.size == psi.size
    e = None
    if ebar is not None:
        e = np.ascontiguousarray(ebar, dtype=np.float64)
        assert e.shape[1] == ndim and e.shape[0] >= step0 + nsteps
    norms = np.zeros(nsteps + 1) if return_norms else None
    rc = _load().orc_schrodinger(ndim, _ptr(nn), _ptr(lo), _ptr(hi), float(dt), float(mass),
                                 float(hbar), _ptr(v), _ptr(e) if e is not None else None,
                                 _ptr(psi), int(step0), int(nsteps), int(direction),
                                 _ptr(norms) if norms is not None else None)
    _check(rc, "schrodinger")
    return (psi, norms) if return_norms else psi


def autocorrelation(psi0, n, xmin, xmax, dt, V0, nsteps, *, mass=1.0, hbar=1.0):
    """chi(t_j) = integral of conj(Psi(x, 0)) Psi(x, t_j), j = 0..nsteps-1, t_j = j dt
    (the autocorrelation function of the paper's eigenstate section): the
    oracle's own Strang steps in the time-independent potential V0, one at a
    time, and its FP64 overlap after each.  Returns (chi, psi after nsteps)."""
    psi = _c128(psi0).copy()
    chi = np.zeros(nsteps, complex)
    for j in range(nsteps):
        chi[j] = overlap(psi0, psi, n, xmin, xmax)
        psi = schrodinger(psi, n, xmin, xmax, dt, V0, None, step0=0, nsteps=1, mass=mass, hbar=hbar)
    return chi, psi


def spectrum(chi, dt, energies, hbar=1.0):
    """Windowed Fourier transform of the autocorrelation (eigenstate section):
    chi~(E) = integral_0^T chi(t) (1 - cos(2 pi t / T)) exp(i t E / hbar) dt with
    T = len(chi) dt, as the rectangle rule over t_j = j dt (the window vanishes
    at both ends, so it equals the trapezoid rule).  FP64, one energy at a time."""
    chi = np.asarray(chi, complex)
    S = len(chi)
    t = dt * np.arange(S)
    w = 1.0 - np.cos(2.0 * np.pi * np.arange(S) / S)
    out = np.zeros(len(energies), complex)
    for i, E in enumerate(energies):
        out[i] = dt * np.sum(chi * w * np.exp(1j * t * E / hbar))
    return out


def eigenfunction(psi0, n, xmin, xmax, dt, V0, nsteps, E, *, mass=1.0, hbar=1.0):
    """Psi_E(x) ~ integral_0^T Psi(x, t) (1 - cos(2 pi t / T)) exp(i E t / hbar) dt
    (eigenstate section), the rectangle rule over the oracle's own steps,
    normalised to dV sum |Psi_E|^2 = 1."""
    psi = _c128(psi0).copy()
    acc = np.zeros_like(psi)
    for j in range(nsteps):
        w = 1.0 - np.cos(2.0 * np.pi * j / nsteps)
        acc += dt * w * np.exp(1j * E * j * dt / hbar) * psi
        psi = schrodinger(psi, n, xmin, xmax, dt, V0, None, step0=0, nsteps=1, mass=mass, hbar=hbar)
    return acc / np.sqrt(norm(acc, n, xmin, xmax))


def peak_energy(energies, spec):
    """Energy of the largest |spec| on a uniform grid, refined by the vertex of
    the parabola through it and its two neighbours."""
    a = np.abs(np.asarray(spec))
    i = int(np.argmax(a))
    i = min(max(i, 1), len(a) - 2)
    y0, y1, y2 = a[i - 1], a[i], a[i + 1]
    d = 0.5 * (y0 - y2) / (y0 - 2.0 * y1 + y2)
    return float(energies[i] + d * (energies[1] - energies[0]))


def schrodinger_velocity(psi0, n, xmin, xmax, dt, V0, abar, a2bar, *, step0=0, nsteps=1, mass=1.0,
                         hbar=1.0, charge=-1.0):
    """Strang steps in the velocity gauge of the dipole approximation: the
    kinetic factor exp(-i/(2 m hbar) [tau p^2 - 2 q p.Abar_n + q^2 A2bar_n])
    (the momentum-space operator of eq. SE_K integrated over the step), the
    potential half steps with tau V0 only.  ``abar``: (total_steps, ndim) step
    integrals of A(t); ``a2bar``: (total_steps,) step integrals of |A(t)|^2."""
    ndim, nn, lo, hi = _axes(n, xmin, xmax)
    psi = _c128(psi0).copy()
    v = np.ascontiguousarray(V0, dtype=np.float64)
    a = np.ascontiguousarray(abar, dtype=np.float64)
    a2 = np.ascontiguousarray(a2bar, dtype=np.float64)
    assert v.size == psi.size and a.shape[1] == ndim and a.shape[0] >= step0 + nsteps and a2.size >= step0 + nsteps
    rc = _load().orc_schrodinger_velocity(ndim, _ptr(nn), _ptr(lo), _ptr(hi), float(dt), float(mass), float(hbar),
                                          float(charge), _ptr(v), _ptr(a), _ptr(a2), _ptr(psi), int(step0),
                                          int(nsteps))
    _check(rc, "schrodinger_velocity")
    return psi


def schrodinger_velocity_adjoint(psi0, gT, n, xmin, xmax, dt, V0, abar, a2bar, *, step0=0, nsteps=1, mass=1.0,
                                 hbar=1.0, charge=-1.0, want_dV0=True):
    """Gradient through ``nsteps`` velocity-gauge steps from a stored FP64
    trajectory, the derivative of each step's kinetic factor written out.
    gT is 2*dL/dconj(psi_T).  Returns (g0, dL_dabar[nsteps, ndim],
    dL_da2bar[nsteps], dL_dV0)."""
    ndim, nn, lo, hi = _axes(n, xmin, xmax)
    p0 = _c128(psi0)
    g = _c128(gT).copy()
    v = np.ascontiguousarray(V0, dtype=np.float64)
    a = np.ascontiguousarray(abar, dtype=np.float64)
    a2 = np.ascontiguousarray(a2bar, dtype=np.float64)
    assert a.shape[1] == ndim and a.shape[0] >= step0 + nsteps and a2.size >= step0 + nsteps
    da = np.zeros((nsteps, ndim))
    da2 = np.zeros(nsteps)
    dv = np.zeros(p0.shape) if want_dV0 else None
    rc = _load().orc_schrodinger_velocity_adjoint(ndim, _ptr(nn), _ptr(lo), _ptr(hi), float(dt), float(mass),
                                                  float(hbar), float(charge), _ptr(v), _ptr(a), _ptr(a2), _ptr(p0),
                                                  _ptr(g), int(step0), int(nsteps), _ptr(da), _ptr(da2),
                                                  _ptr(dv) if dv is not None else None)
    _check(rc, "schrodinger_velocity_adjoint")
    return g, da, da2, dv


def schrodinger_adjoint(psi0, gT, n, xmin, xmax, dt, V0, ebar=None, *, step0=0, nsteps=1,
                        mass=1.0, hbar=1.0, want_dV0=True):
    """Gradient through ``nsteps`` forward steps from a stored FP64 trajectory.

    gT is 2*dL/dconj(psi_T).  Returns (g0, dL_debar[nsteps, ndim], dL_dV0)."""
    ndim, nn, lo, hi = _axes(n, xmin, xmax)
    p0 = _c128(psi0)
    g = _c128(gT).copy()
    v = np.ascontiguousarray(V0, dtype=np.float64)
    e = None
    if ebar is not None:
        e = np.ascontiguousarray(ebar, dtype=np.float64)
        assert e.shape[1] == ndim and e.shape[0] >= step0 + nsteps
    de = np.zeros((nsteps, ndim))
    dv = np.zeros(p0.shape) if want_dV0 else None
    rc = _load().orc_schrodinger_adjoint(ndim, _ptr(nn), _ptr(lo), _ptr(hi), float(dt), float(mass),
                                         float(hbar), _ptr(v), _ptr(e) if e is not None else None,
                                         _ptr(p0), _ptr(g), int(step0), int(nsteps), _ptr(de),
                                         _ptr(dv) if dv is not None else None)
    _check(rc, "schrodinger_adjoint")
    return g, de, dv


def dirac1d(psi0, n, xmin, xmax, dt, V0, abar=None, *, step0=0, nsteps=1, mass=1.0, charge=-1.0,
            c=137.036, hbar=1.0):
    """Strang steps of the 1-D two-component Dirac equation, 2-spinor of shape
    (2, n).  ``abar`` has shape (total_steps, n): the step integral of A_1(x, t)."""
    n = int(n[0]) if hasattr(n, "__len__") else int(n)
    lo = float(xmin[0]) if hasattr(xmin, "__len__") else float(xmin)
    hi = float(xmax[0]) if hasattr(xmax, "__len__") else float(xmax)
    psi = _c128(psi0).copy()
    assert psi.shape == (2, n)
    v = np.ascontiguousarray(V0, dtype=np.float64)
    a = None
    if abar is not None:
        a = np.ascontiguousarray(abar, dtype=np.float64)
        assert a.shape[1] == n and a.shape[0] >= step0 + nsteps
    rc = _load().orc_dirac1d(n, lo, hi, float(dt), float(mass), float(charge), float(c), float(hbar), _ptr(v),
                             _ptr(a) if a is not None else None, _ptr(psi), int(step0), int(nsteps))
    _check(rc, "dirac1d")
    return psi


def dirac2d(psi0, n, xmin, xmax, dt, V0, abar_y=None, *, step0=0, nsteps=1, mass=1.0,
            charge=-1.0, c=137.036, hbar=1.0, direction=1):
    """Strang steps of the 2-D Dirac equation, 4-spinor of shape (4, ny, nx).

    ``abar_y`` has shape (total_steps, nx): the step integral of A_y(x, t)."""
    nn = np.array([n[0], n[1]], np.int64)
    lo = np.array(xmin[:2], np.float64)
    hi = np.array(xmax[:2], np.float64)
    psi = _c128(psi0).copy()
    assert psi.shape == (4, n[1], n[0])
    v = np.ascontiguousarray(V0, dtype=np.float64)
    a = None
    if abar_y is not None:
        a = np.ascontiguousarray(abar_y, dtype=np.float64)
        assert a.shape[1] == n[0] and a.shape[0] >= step0 + nsteps
    rc = _load().orc_dirac2d(_ptr(nn), _ptr(lo), _ptr(hi), float(dt), float(mass), float(charge),
                             float(c), float(hbar), _ptr(v), _ptr(a) if a is not None else None,
                             _ptr(psi), int(step0), int(nsteps), int(direction))
    _check(rc, "dirac2d")
    return psi
