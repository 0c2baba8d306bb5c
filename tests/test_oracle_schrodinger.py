"""Pins for the oracle's Schroedinger split step (Sec. 2.1-2.2).

Each pin is fixed by mathematics, not by the oracle:
  * Gaussian packets in a quadratic plus linear potential stay Gaussian under
    every factor of the Strang step, so the exact result of the DISCRETE-TIME
    map (no splitting error at all) follows from the Heller parameter
    recurrence, derived here from the free Schroedinger equation;
  * the "shadow" harmonic-oscillator ground state, the exact fixed point of
    that map, only picks up a phase exp(-i theta/2) per step;
  * unitarity and time reversibility of the step;
  * on tiny grids the step is compared with the matrix exponential of the
    discretised Hamiltonian: local error O(tau^3), global error O(tau^2)
    (eq. U_split).
"""
import cmath
import math

import numpy as np
import pytest
import scipy.linalg

from paper_1012_3911_amd import workloads as W


# ------------------------------------------------------------ Heller Gaussian --
# psi(x) = exp(i [a (x-q)^2 + p (x-q) + g]),   hbar = m = 1.
# Kick by exp(-i (u x^2 + e x)):  a -= u, p -= 2 u q + e, g -= u q^2 + e q
# Free drift for time t (i psi_t = -psi_xx/2):  a' = a/(1+2at), q' = q+pt,
#   g' = g + p^2 t/2 + (i/2) log(1+2at),  p' = p.

class Heller:
    def __init__(self, a, q, p, g):
        self.a, self.q, self.p, self.g = complex(a), float(q), float(p), complex(g)

    def kick(self, quad, lin):
        """Multiply by exp(-i (quad x^2 + lin x))."""
        q = self.q
        self.a -= quad
        self.p -= 2 * quad * q + lin
        self.g -= quad * q * q + lin * q

    def drift(self, t):
        a, q, p, g = self.a, self.q, self.p, self.g
        self.a = a / (1 + 2 * a * t)
        self.q = q + p * t
        self.g = g + p * p * t / 2 + 0.5j * cmath.log(1 + 2 * a * t)

    def values(self, x):
        d = x - self.q
        return np.exp(1j * (self.a * d * d + self.p * d + self.g))


def heller_from_gaussian(x0, sigma, k0, norm):
    # norm * exp(-(x-x0)^2/(4 s^2) + i k0 x)
    return Heller(1j / (4 * sigma**2), x0, k0, k0 * x0 - 1j * math.log(norm))


def discrete_norm_factor(n, xmin, xmax, x0, sigma, k0):
    (x,) = W.axes((n,), (xmin,), (xmax,))
    g = np.exp(-((x - x0) ** 2) / (4 * sigma**2))
    return 1.0 / math.sqrt(np.sum(np.abs(g) ** 2) * (xmax - xmin) / n)


def heller_run(h, omega2, ebar, dt, nsteps):
    """Exact discrete Strang map: half kick, drift, half kick with V = omega2 x^2/2 + x E(t)."""
    for s in range(nsteps):
        e = 0.0 if ebar is None else ebar[s]
        h.kick(dt * omega2 / 4, e / 2)
        h.drift(dt)
        h.kick(dt * omega2 / 4, e / 2)
    return h


def rel_l2(a, b):
    return float(np.linalg.norm((a - b).ravel()) / np.linalg.norm(b.ravel()))


def test_heller_harmonic_1d_full_config(orc):
    """1-D N=1024 harmonic packet, tau = 0.01, 1000 steps (the c128 parity workload)."""
    wl = W.harmonic_1d()
    psi = orc.schrodinger(wl.psi0, wl.n, wl.xmin, wl.xmax, wl.dt, wl.V0, wl.ebar, nsteps=wl.nsteps)
    m = wl.meta
    nf = discrete_norm_factor(wl.n[0], wl.xmin[0], wl.xmax[0], m["x0"], m["sigma"], m["k0"])
    h = heller_run(heller_from_gaussian(m["x0"], m["sigma"], m["k0"], nf), 1.0, None, wl.dt, wl.nsteps)
    (x,) = W.axes(wl.n, wl.xmin, wl.xmax)
    err = rel_l2(psi, h.values(x))
    assert err < 5e-13, err


def test_heller_with_dipole_field_1d(orc):
    """Linear potential x.E(t) pins the field term of the half step (sign, the 1/2, x_j)."""
    n, L, dt, ns = 512, 40.0, 0.02, 300
    (x,) = W.axes((n,), (-L,), (L,))
    psi0 = W.gaussian((n,), (-L,), (L,), (1.5,), 1.3, (0.7,))
    t = (np.arange(ns) + 0.5) * dt
    ebar = (dt * 0.3 * np.sin(0.9 * t))[:, None]
    V0 = 0.25 * x**2  # omega^2 = 0.5
    psi = orc.schrodinger(psi0, (n,), (-L,), (L,), dt, V0, ebar, nsteps=ns)
    nf = discrete_norm_factor(n, -L, L, 1.5, 1.3, 0.7)
    h = heller_run(heller_from_gaussian(1.5, 1.3, 0.7, nf), 0.5, ebar[:, 0], dt, ns)
    assert rel_l2(psi, h.values(x)) < 5e-13


def test_heller_separable_3d_anisotropic(orc):
    """A product of 1-D Gaussians in a separable quadratic potential stays a product:
    pins the axis order, per-axis box lengths and the multi-axis kinetic phase."""
    n = (64, 32, 32)
    lo = (-8.0, -9.0, -6.5)
    hi = (8.0, 9.0, 6.5)
    w2 = (1.0, 0.5, 2.0)
    x0 = (0.5, -0.8, 0.2)
    k0 = (0.4, -0.3, 0.25)
    sig = tuple(1.0 / math.sqrt(2.0 * math.sqrt(w)) for w in w2)  # ground-state widths
    dt, ns = 0.02, 60
    t = (np.arange(ns) + 0.5) * dt
    ebar = np.stack([dt * 0.2 * np.cos(t), dt * 0.1 * np.sin(2 * t), dt * 0.05 * np.ones(ns)], axis=1)
    X = W.mesh(n, lo, hi)
    V0 = sum(0.5 * w2[a] * X[a] ** 2 for a in range(3))
    factors = []
    for a in range(3):
        (xa,) = W.axes((n[a],), (lo[a],), (hi[a],))
        nf = discrete_norm_factor(n[a], lo[a], hi[a], x0[a], sig[a], k0[a])
        factors.append((xa, heller_from_gaussian(x0[a], sig[a], k0[a], nf)))
    vals = [h.values(xa) for xa, h in factors]
    psi0 = vals[2][:, None, None] * vals[1][None, :, None] * vals[0][None, None, :]
    psi = orc.schrodinger(psi0, n, lo, hi, dt, V0, ebar, nsteps=ns)
    ev = [heller_run(h, w2[a], ebar[:, a], dt, ns).values(xa) for a, (xa, h) in enumerate(factors)]
    ref = ev[2][:, None, None] * ev[1][None, :, None] * ev[0][None, None, :]
    # grids resolve the packet to ~1e-9 (box tails and spectral cut), not to machine precision
    assert rel_l2(psi, ref) < 1e-8


def test_shadow_ground_state(orc):
    """psi_s = (s/pi)^(1/4) exp(-s x^2/2), s = sqrt(1 - tau^2/4), is the exact fixed
    point of the Strang map for V = x^2/2; each step multiplies it by exp(-i theta/2),
    cos(theta) = 1 - tau^2/2."""
    n, L, dt, ns = 1024, 50.0, 0.01, 1000
    (x,) = W.axes((n,), (-L,), (L,))
    s = math.sqrt(1 - dt * dt / 4)
    theta = math.acos(1 - dt * dt / 2)
    psi_s = (s / math.pi) ** 0.25 * np.exp(-s * x**2 / 2) + 0j
    psi = orc.schrodinger(psi_s, (n,), (-L,), (L,), dt, 0.5 * x**2, None, nsteps=ns)
    assert rel_l2(psi, psi_s * np.exp(-1j * ns * theta / 2)) < 5e-13


def test_unitarity_and_reversal_2d(orc):
    wl = W.softcore_2d_laser(n=64, nsteps=120, L=20.0)
    psi, norms = orc.schrodinger(wl.psi0, wl.n, wl.xmin, wl.xmax, wl.dt, wl.V0, wl.ebar,
                                 nsteps=wl.nsteps, return_norms=True)
    assert np.max(np.abs(norms / norms[0] - 1)) < 1e-13
    back = orc.schrodinger(psi, wl.n, wl.xmin, wl.xmax, wl.dt, wl.V0, wl.ebar,
                           nsteps=wl.nsteps, direction=-1)
    assert rel_l2(back, wl.psi0) < 1e-12
    # the step really moved the state
    assert rel_l2(psi, wl.psi0) > 1e-2


def _dense_step_matrix(orc, n, L, dt, V0):
    N = n
    S = np.zeros((N, N), complex)
    for j in range(N):
        e = np.zeros(N, complex)
        e[j] = 1
        S[:, j] = orc.schrodinger(e, (n,), (-L,), (L,), dt, V0, None, nsteps=1)
    return S


def _dense_hamiltonian(n, L, V0):
    k = 2 * np.pi * np.fft.fftfreq(n, d=2 * L / n)
    F = np.exp(-2j * np.pi * np.outer(np.arange(n), np.arange(n)) / n)
    T = np.conj(F).T @ np.diag(k**2 / 2) @ F / n
    return T + np.diag(V0)


def test_local_and_global_order(orc):
    """Strang splitting (eq. U_split): local error tau^3, global tau^2, against
    expm(-i tau H) of the discretised Hamiltonian."""
    n, L = 32, 6.0
    (x,) = W.axes((n,), (-L,), (L,))
    V0 = 0.5 * x**2 + 0.3 * np.cos(x)
    H = _dense_hamiltonian(n, L, V0)
    taus = np.array([0.04, 0.02, 0.01, 0.005])
    loc = []
    for tau in taus:
        S = _dense_step_matrix(orc, n, L, tau, V0)
        loc.append(np.linalg.norm(S - scipy.linalg.expm(-1j * tau * H), 2))
    slope = np.polyfit(np.log(taus), np.log(loc), 1)[0]
    assert abs(slope - 3.0) < 0.15, slope
    T = 0.4
    psi0 = W.gaussian((n,), (-L,), (L,), (0.3,), 0.8, (0.5,))
    exact = scipy.linalg.expm(-1j * T * H) @ psi0
    glob = []
    for tau in taus:
        m = int(round(T / tau))
        psi = orc.schrodinger(psi0, (n,), (-L,), (L,), tau, V0, None, nsteps=m)
        glob.append(np.linalg.norm(psi - exact))
    slope = np.polyfit(np.log(taus), np.log(glob), 1)[0]
    assert abs(slope - 2.0) < 0.1, slope


def test_step_resume_is_exact(orc):
    """Steps are Markov in (psi, step index): 40 steps = 25 then 15 starting at step 25."""
    wl = W.softcore_2d_laser(n=32, nsteps=40, L=16.0)
    a = orc.schrodinger(wl.psi0, wl.n, wl.xmin, wl.xmax, wl.dt, wl.V0, wl.ebar, nsteps=40)
    b = orc.schrodinger(wl.psi0, wl.n, wl.xmin, wl.xmax, wl.dt, wl.V0, wl.ebar, nsteps=25)
    b = orc.schrodinger(b, wl.n, wl.xmin, wl.xmax, wl.dt, wl.V0, wl.ebar, step0=25, nsteps=15)
    assert np.array_equal(a, b)


def test_norm_overlap(orc):
    n, lo, hi = (16, 8), (-2.0, -1.0), (2.0, 3.0)
    rng = np.random.default_rng(0)
    a = rng.standard_normal((8, 16)) + 1j * rng.standard_normal((8, 16))
    b = rng.standard_normal((8, 16)) + 1j * rng.standard_normal((8, 16))
    dv = (4 / 16) * (4 / 8)
    assert abs(orc.norm(a, n, lo, hi) - dv * np.sum(np.abs(a) ** 2)) < 1e-12
    assert abs(orc.overlap(a, b, n, lo, hi) - dv * np.vdot(a, b)) < 1e-12


# ------------------------------------------------------ free Gaussian (Sec. 5.1) --

def test_free_packet_spreads_as_the_closed_form(orc):
    """A free Gaussian packet (the paper's free-packet experiment, Sec. 5.1,
    in its /4 width convention): with V = 0 every Strang step is the exact
    spectral propagator, so after t the state is the textbook free packet,
    centre x0 + hbar k0 t / m and |psi|^2 standard deviation
    sigma sqrt(1 + (hbar t / (2 m sigma^2))^2), with the complex amplitude
    (sigma^2 / s)^(1/2) exp(-(x - x0 - k0 t)^2 / (4 s) + i k0 x - i k0^2 t / 2),
    s = sigma^2 + i t / 2 (hbar = m = 1)."""
    N, L, sigma, x0, k0, dt, S = 4096, 200.0, 1.0, -20.0, 2.0, 0.01, 1000
    x = -L + 2 * L / N * np.arange(N)
    A = (2 * np.pi * sigma ** 2) ** -0.25
    psi0 = A * np.exp(-(x - x0) ** 2 / (4 * sigma ** 2) + 1j * k0 * x)
    out = orc.schrodinger(psi0, (N,), (-L,), (L,), dt, np.zeros(N), None, nsteps=S)
    t = dt * S
    s = sigma ** 2 + 0.5j * t
    exact = A * np.sqrt(sigma ** 2 / s) * np.exp(-(x - x0 - k0 * t) ** 2 / (4 * s) + 1j * k0 * x - 0.5j * k0 ** 2 * t)
    assert np.linalg.norm(out - exact) / np.linalg.norm(exact) < 1e-11
    rho = np.abs(out) ** 2
    rho /= rho.sum()
    centre = (x * rho).sum()
    width = math.sqrt(((x - centre) ** 2 * rho).sum())
    assert abs(centre - (x0 + k0 * t)) < 1e-9
    assert abs(width - sigma * math.sqrt(1 + (t / (2 * sigma ** 2)) ** 2)) < 1e-9
