"""Pins of the oracle's velocity-gauge step (the dipole-approximation split
with the vector potential in the momentum-space factor, eq. SE_K).

With A(0) = 0 and E = -dA/dt the velocity-gauge state equals
exp(i q A(t).x / hbar) times the length-gauge state (a gauge transformation,
exact for the Schroedinger equation); both splittings converge to it at
second order in tau, so their difference must fall fourfold when tau halves
(a state held in a harmonic well, far from the box edge).
With A = 0 the two steps coincide."""
import numpy as np

import oracle as orc

Q = -1.0


def _fields(S, dt, A0=0.5, w=0.5):
    t = dt * np.arange(S + 1)
    A = A0 * np.sin(w * t)
    abar = (A0 / w) * (np.cos(w * t[:-1]) - np.cos(w * t[1:]))
    a2bar = A0 ** 2 * (dt / 2 - (np.sin(2 * w * t[1:]) - np.sin(2 * w * t[:-1])) / (4 * w))
    ebar = -(A[1:] - A[:-1])  # int E dt with E = -dA/dt
    return A, abar, a2bar, ebar


def _gauge_gap(ndim, dt, T=10.0):
    S = int(round(T / dt))
    N, L = (128, 10.0) if ndim == 1 else (64, 8.0)
    n, lo, hi = (N,) * ndim, (-L,) * ndim, (L,) * ndim
    ax = -L + 2 * L / N * np.arange(N)
    X = np.meshgrid(*([ax] * ndim), indexing="ij")[::-1]  # x first
    r2 = sum(x ** 2 for x in X)
    # a harmonic well keeps the state far from the box edge, where the
    # length gauge's x.E is discontinuous on the periodic grid
    V0 = 0.5 * r2
    psi0 = np.exp(-r2 / 2 + 0.3j * X[0]).astype(complex)
    A, abar, a2bar, ebar = _fields(S, dt)
    pol = np.zeros(ndim)
    pol[0] = 1.0  # field along x
    psi_l = orc.schrodinger(psi0, n, lo, hi, dt, V0, ebar[:, None] * pol[None, :], nsteps=S)
    psi_v = orc.schrodinger_velocity(psi0, n, lo, hi, dt, V0, abar[:, None] * pol[None, :], a2bar, nsteps=S,
                                     charge=Q)
    gauge = np.exp(1j * Q * A[-1] * X[0])
    return np.linalg.norm(psi_v - gauge * psi_l) / np.linalg.norm(psi_l)


def test_gauge_equivalence_second_order_1d():
    e1, e2 = _gauge_gap(1, 0.05), _gauge_gap(1, 0.025)
    assert e1 < 2e-3
    assert 3.6 < e1 / e2 < 4.4, (e1, e2)


def test_gauge_equivalence_second_order_2d():
    e1, e2 = _gauge_gap(2, 0.05), _gauge_gap(2, 0.025)
    assert 3.6 < e1 / e2 < 4.4, (e1, e2)


def test_zero_vector_potential_is_the_length_gauge():
    N, L, dt, S = 128, 10.0, 0.02, 20
    x = -L + 2 * L / N * np.arange(N)
    psi0 = np.exp(-(x - 1) ** 2 + 0.5j * x)
    V0 = 0.5 * x ** 2
    a = orc.schrodinger(psi0, (N,), (-L,), (L,), dt, V0, None, nsteps=S)
    b = orc.schrodinger_velocity(psi0, (N,), (-L,), (L,), dt, V0, np.zeros((S, 1)), np.zeros(S), nsteps=S)
    assert np.array_equal(a, b)
