"""Seeded synthetic inputs for the split-operator workloads.

This module only builds inputs (grids, potentials, field tables, initial and
target states).  It holds none of the method's arithmetic: no step, no
transform of a state through time, no propagator.  Both the GPU library's
tests and the CPU oracle's tests draw their inputs from here.

Units are atomic units (hbar = 1, m = 1, electron charge q = -1, Sec. 5 of the
paper).  Grids are periodic boxes [xmin, xmax) with x_j = xmin + j*dx; arrays
are numpy C-order with shape (nz, ny, nx), x fastest; ``n`` lists sizes in
(x, y, z) order.

Workload shapes follow the paper's experiments (Gaussian packets in harmonic
and soft-core potentials, eq. soft_core; the laser pulse of eq. laserpulse;
the Dirac packet of Sec. 5.1) at the sizes the benchmark suite names.
"""
from __future__ import annotations

import dataclasses
import math
from typing import Optional, Sequence

import numpy as np

C_LIGHT = 137.036


@dataclasses.dataclass
class Workload:
    name: str
    equation: str  # "schrodinger" | "dirac"
    n: tuple  # sizes in (x, y, z) order
    xmin: tuple
    xmax: tuple
    dt: float
    nsteps: int
    V0: np.ndarray  # potential energy, float64, spatial shape
    psi0: np.ndarray  # complex128, spatial shape (Dirac: (4, ny, nx))
    ebar: Optional[np.ndarray] = None  # (nsteps, ndim) step integrals of E(t)
    abar_y: Optional[np.ndarray] = None  # (nsteps, nx) step integrals of A_y(x, t)
    mass: float = 1.0
    charge: float = -1.0
    c: float = C_LIGHT
    hbar: float = 1.0
    meta: dict = dataclasses.field(default_factory=dict)

    @property
    def ndim(self) -> int:
        return len(self.n)

    @property
    def npoints(self) -> int:
        return int(np.prod(self.n))

    @property
    def ncomp(self) -> int:
        return 4 if self.equation == "dirac" else 1

    @property
    def dx(self) -> tuple:
        return tuple((b - a) / m for a, b, m in zip(self.xmin, self.xmax, self.n))

    @property
    def dv(self) -> float:
        return float(np.prod(self.dx))


def axes(n: Sequence[int], xmin: Sequence[float], xmax: Sequence[float]):
    """Coordinate vectors per axis, in (x, y, z) order."""
    return [xmin[a] + (xmax[a] - xmin[a]) / n[a] * np.arange(n[a]) for a in range(len(n))]


def mesh(n, xmin, xmax):
    """Coordinate arrays in numpy order: returns [X, Y, Z][:ndim], each of spatial shape."""
    ax = axes(n, xmin, xmax)
    grids = np.meshgrid(*ax[::-1], indexing="ij")  # (z, y, x) order
    return grids[::-1]


def _normalise(psi: np.ndarray, dv: float) -> np.ndarray:
    return psi / math.sqrt(float(np.sum(np.abs(psi) ** 2)) * dv)


def gaussian(n, xmin, xmax, x0, sigma, k0) -> np.ndarray:
    """exp(-|x-x0|^2/(4 sigma^2) + i k0.x), unit norm; sigma is the std of |psi|^2
    per axis (the paper's /4 form of the Gaussian, Sec. 5.1)."""
    X = mesh(n, xmin, xmax)
    arg = np.zeros(X[0].shape, np.complex128)
    for a in range(len(n)):
        arg += -((X[a] - x0[a]) ** 2) / (4.0 * sigma**2) + 1j * k0[a] * X[a]
    dv = float(np.prod([(xmax[a] - xmin[a]) / n[a] for a in range(len(n))]))
    return _normalise(np.exp(arg), dv)


# ----------------------------------------------------------------- configs --

def harmonic_1d(n=1024, nsteps=1000, seed=1, dt=0.01, L=50.0) -> Workload:
    """1-D Gaussian packet in V = x^2/2 on [-L, L): x0 ~ U[-5,5], k0 ~ U[-2,2], sigma = 1."""
    rng = np.random.default_rng(seed)
    x0 = rng.uniform(-5.0, 5.0)
    k0 = rng.uniform(-2.0, 2.0)
    (x,) = axes((n,), (-L,), (L,))
    return Workload(
        name="1d_harmonic_%d" % n, equation="schrodinger", n=(n,), xmin=(-L,), xmax=(L,), dt=dt,
        nsteps=nsteps, V0=0.5 * x**2, psi0=gaussian((n,), (-L,), (L,), (x0,), 1.0, (k0,)),
        ebar=np.zeros((nsteps, 1)), meta=dict(x0=x0, k0=k0, sigma=1.0))


def laser_envelope_field(t, E0=0.05, omega=0.057, Tp=10.0):
    """E(t) = E0 sin^2(pi t / Tp) cos(omega t) for 0 <= t <= Tp, else 0."""
    t = np.asarray(t, dtype=np.float64)
    on = (t >= 0) & (t <= Tp)
    return np.where(on, E0 * np.sin(np.pi * t / Tp) ** 2 * np.cos(omega * t), 0.0)


def softcore_2d_laser(n=2048, nsteps=500, dt=0.02, L=100.0, E0=0.05, omega=0.057) -> Workload:
    """2-D soft-core Coulomb atom V0 = -1/sqrt(r^2+1) driven by x.E(t), E(t) polarised
    along x with a sin^2 envelope lasting the whole run; psi0 ~ exp(-r^2/2)."""
    N = (n, n)
    lo, hi = (-L, -L), (L, L)
    X, Y = mesh(N, lo, hi)
    V0 = -1.0 / np.sqrt(X**2 + Y**2 + 1.0)
    psi0 = gaussian(N, lo, hi, (0.0, 0.0), 1.0 / math.sqrt(2.0), (0.0, 0.0))
    Tp = nsteps * dt
    tmid = (np.arange(nsteps) + 0.5) * dt
    ebar = np.zeros((nsteps, 2))
    ebar[:, 0] = dt * laser_envelope_field(tmid, E0, omega, Tp)  # midpoint rule
    return Workload(name="2d_softcore_laser_%d" % n, equation="schrodinger", n=N, xmin=lo, xmax=hi,
                    dt=dt, nsteps=nsteps, V0=V0, psi0=psi0, ebar=ebar,
                    meta=dict(E0=E0, omega=omega, Tp=Tp))


def wells_3d(n=256, nsteps=200, seed=3, dt=0.01, L=40.0, nwells=8) -> Workload:
    """3-D random sum of Gaussian wells: centres ~ U[-10,10]^3, depths ~ U[0.5,2],
    widths ~ U[0.5,2]; Gaussian packet sigma = 1 at the origin, k0 = 0."""
    rng = np.random.default_rng(seed)
    centres = rng.uniform(-10.0, 10.0, size=(nwells, 3))
    depths = rng.uniform(0.5, 2.0, size=nwells)
    widths = rng.uniform(0.5, 2.0, size=nwells)
    N = (n, n, n)
    lo, hi = (-L,) * 3, (L,) * 3
    X, Y, Z = mesh(N, lo, hi)
    V0 = np.zeros(X.shape)
    for j in range(nwells):
        r2 = (X - centres[j, 0]) ** 2 + (Y - centres[j, 1]) ** 2 + (Z - centres[j, 2]) ** 2
        V0 -= depths[j] * np.exp(-r2 / (2.0 * widths[j] ** 2))
    psi0 = gaussian(N, lo, hi, (0.0, 0.0, 0.0), 1.0, (0.0, 0.0, 0.0))
    return Workload(name="3d_wells_%d" % n, equation="schrodinger", n=N, xmin=lo, xmax=hi, dt=dt,
                    nsteps=nsteps, V0=V0, psi0=psi0, ebar=np.zeros((nsteps, 3)),
                    meta=dict(centres=centres, depths=depths, widths=widths))


# ------------------------------------------------------------------ Dirac --

def pulse_envelope_integral(eta, j=4, l=1):
    """F(eta) = Int_{-j pi}^{eta} sin(s) f_{j,l}(s) ds for the trapezoid envelope
    f_{j,l} of eq. laserpulse (linear ramps of l half cycles, j half cycles in all)."""
    eta = np.asarray(eta, dtype=np.float64)
    pi = math.pi
    a, b, c = -j * pi, (-j + l) * pi, -l * pi

    def ramp_up(s):  # antiderivative of sin(s) (s + j pi)/(l pi)
        return (-np.cos(s) * (s + j * pi) + np.sin(s)) / (l * pi)

    def plateau(s):
        return -np.cos(s)

    def ramp_down(s):  # antiderivative of -s sin(s)/(l pi)
        return (s * np.cos(s) - np.sin(s)) / (l * pi)

    F_b = ramp_up(b) - ramp_up(a)
    F_c = F_b + plateau(c) - plateau(b)
    F_0 = F_c + ramp_down(0.0) - ramp_down(c)
    out = np.zeros_like(eta)
    m1 = (eta >= a) & (eta < b)
    m2 = (eta >= b) & (eta < c)
    m3 = (eta >= c) & (eta < 0.0)
    m4 = eta >= 0.0
    out[m1] = ramp_up(eta[m1]) - ramp_up(a)
    out[m2] = F_b + plateau(eta[m2]) - plateau(b)
    out[m3] = F_c + ramp_down(eta[m3]) - ramp_down(c)
    out[m4] = F_0
    return out


def laser_vector_potential(x, t, E0=3072.0, lam=10.0, j=4, l=1, c=C_LIGHT):
    """A_y(x, t) of a pulse travelling along +x with E along y: A_y = (E0/omega) F(kx - omega t),
    so that E_y = -dA_y/dt = E0 sin(eta) f(eta) (eq. laserpulse)."""
    k = 2.0 * math.pi / lam
    omega = c * k
    return (E0 / omega) * pulse_envelope_integral(k * np.asarray(x) - omega * t, j, l)


def dirac_spinor_up(px, py, mass=1.0, c=C_LIGHT):
    """Positive-energy spin-up plane-wave spinor d+ e1 + d- (p1 + i p2)/|p| e4
    (a column of the diagonalising matrix u(p) of eq. u_p); unit length."""
    p2 = px**2 + py**2
    x2 = p2 / (mass * c) ** 2
    dp = np.sqrt(0.5 + 0.5 / np.sqrt(1.0 + x2))
    dm = np.sqrt(np.maximum(0.5 - 0.5 / np.sqrt(1.0 + x2), 0.0))
    pabs = np.sqrt(p2)
    safe = np.where(pabs > 0, pabs, 1.0)
    s = np.zeros((4,) + np.shape(px), np.complex128)
    s[0] = dp
    s[3] = np.where(pabs > 0, dm * (px + 1j * py) / safe, 0.0)
    return s


def dirac_packet(n, xmin, xmax, pbar=(40.0, 0.0), sigma_f=80.0, sigma_s=20.0, mass=1.0,
                 c=C_LIGHT, hbar=1.0):
    """Gaussian momentum distribution of Sec. 5.1 times the positive-energy spin-up
    spinor, brought to real space by the inverse DFT on the grid (k in FFT order,
    phase exp(i k xmin) for the box origin); unit norm."""
    nx, ny = n
    Lx, Ly = xmax[0] - xmin[0], xmax[1] - xmin[1]
    kx = 2 * math.pi * np.fft.fftfreq(nx, d=Lx / nx)
    ky = 2 * math.pi * np.fft.fftfreq(ny, d=Ly / ny)
    KY, KX = np.meshgrid(ky, kx, indexing="ij")
    PX, PY = hbar * KX, hbar * KY
    phi = math.atan2(pbar[1], pbar[0])
    R = np.array([[math.cos(phi), -math.sin(phi)], [math.sin(phi), math.cos(phi)]])
    Sinv = R @ np.diag([1 / sigma_f**2, 1 / sigma_s**2]) @ R.T
    dpx, dpy = PX - pbar[0], PY - pbar[1]
    quad = Sinv[0, 0] * dpx**2 + 2 * Sinv[0, 1] * dpx * dpy + Sinv[1, 1] * dpy**2
    amp = np.exp(-quad / 4.0)
    spin = dirac_spinor_up(PX, PY, mass, c)
    shift = np.exp(1j * (KX * xmin[0] + KY * xmin[1]))
    psik = spin * (amp * shift)[None]
    psi = np.fft.ifft2(psik, axes=(1, 2))
    dv = (Lx / nx) * (Ly / ny)
    return _normalise(psi, dv)


def dirac_softcore_laser(n=1024, nsteps=200, dt=1e-5, L=2.0, Z=20.0, zeta=0.791, E0=3072.0,
                         lam=10.0, sigma_f=80.0, sigma_s=20.0) -> Workload:
    """2-D Dirac 4-spinor: soft-core nucleus V0 = -Z/sqrt(r^2 + (zeta/Z)^2) (eq. soft_core),
    a linearly polarised pulse along +x with A along y (eq. laserpulse, 4 half cycles,
    1-half-cycle ramps), and a positive-energy spin-up packet with pbar = (40, 0)."""
    N = (n, n)
    lo, hi = (-L, -L), (L, L)
    X, Y = mesh(N, lo, hi)
    V0 = -Z / np.sqrt(X**2 + Y**2 + (zeta / Z) ** 2)
    (x,) = axes((n,), (-L,), (L,))
    tmid = (np.arange(nsteps) + 0.5) * dt
    abar = np.stack([dt * laser_vector_potential(x, t, E0, lam) for t in tmid])  # midpoint rule
    psi0 = dirac_packet(N, lo, hi, (40.0, 0.0), sigma_f, sigma_s)
    return Workload(name="dirac2d_softcore_%d" % n, equation="dirac", n=N, xmin=lo, xmax=hi, dt=dt,
                    nsteps=nsteps, V0=V0, psi0=psi0, abar_y=abar,
                    meta=dict(Z=Z, zeta=zeta, E0=E0, lam=lam))


# ---------------------------------------------------------------- batched --

def control_batch(seed=5, count=64, nsteps=400, dt=0.05, namp=200, sizes_1d=(9, 13),
                  sizes_2d=(8, 10)):
    """Independent control problems of uneven size.  The first half are 1-D
    (N = 2^U{9..13} on [-100, 100), V = -1/sqrt(x^2+2)), the second half 2-D
    (N^2, N = 2^U{8..10} on [-50, 50)^2, V = -1/sqrt(r^2+0.6257)).  psi0 is a
    sigma = 1 Gaussian at the origin, the target the same packet moved +1 along x.
    The control is ``namp`` amplitudes ~ U[-0.05, 0.05] along x, each held for
    nsteps/namp steps.  Returns (workloads, targets, control)."""
    rng = np.random.default_rng(seed)
    half = count // 2
    e1 = rng.integers(sizes_1d[0], sizes_1d[1] + 1, size=half)
    e2 = rng.integers(sizes_2d[0], sizes_2d[1] + 1, size=count - half)
    control = rng.uniform(-0.05, 0.05, size=namp)
    hold = nsteps // namp
    amp_per_step = np.repeat(control, hold)
    out, targets = [], []
    for e in e1:
        N = (int(2**e),)
        lo, hi = (-100.0,), (100.0,)
        (x,) = axes(N, lo, hi)
        eb = np.zeros((nsteps, 1))
        eb[:, 0] = dt * amp_per_step
        out.append(Workload(name="b1d_%d" % N[0], equation="schrodinger", n=N, xmin=lo, xmax=hi,
                            dt=dt, nsteps=nsteps, V0=-1.0 / np.sqrt(x**2 + 2.0),
                            psi0=gaussian(N, lo, hi, (0.0,), 1.0, (0.0,)), ebar=eb))
        targets.append(gaussian(N, lo, hi, (1.0,), 1.0, (0.0,)))
    for e in e2:
        N = (int(2**e), int(2**e))
        lo, hi = (-50.0, -50.0), (50.0, 50.0)
        X, Y = mesh(N, lo, hi)
        eb = np.zeros((nsteps, 2))
        eb[:, 0] = dt * amp_per_step
        out.append(Workload(name="b2d_%d" % N[0], equation="schrodinger", n=N, xmin=lo, xmax=hi,
                            dt=dt, nsteps=nsteps, V0=-1.0 / np.sqrt(X**2 + Y**2 + 0.6257),
                            psi0=gaussian(N, lo, hi, (0.0, 0.0), 1.0, (0.0, 0.0)), ebar=eb))
        targets.append(gaussian(N, lo, hi, (1.0, 0.0), 1.0, (0.0, 0.0)))
    return out, targets, dict(control=control, hold=hold, dt=dt)
