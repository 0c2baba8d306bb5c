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


# ------------------------------------------------------- velocity-gauge gradient --

def _vg_problem(n, S=12, dt=0.05, seed=0):
    ndim = len(n)
    L = 6.0
    lo, hi = (-L,) * ndim, (L,) * ndim
    axes = [-L + 2 * L / m * np.arange(m) for m in n]
    X = np.meshgrid(*axes[::-1], indexing="ij")[::-1]
    r2 = sum(x ** 2 for x in X)
    V0 = 0.4 * r2 - 1.0 / np.sqrt(r2 + 1.0)
    psi0 = np.exp(-r2 / 2 + 0.5j * X[0]).astype(complex)
    psi0 /= np.sqrt(orc.norm(psi0, n, lo, hi))
    target = np.exp(-((X[0] - 0.4) ** 2 + sum(x ** 2 for x in X[1:])) / 2).astype(complex)
    rng = np.random.default_rng(seed)
    abar = dt * rng.uniform(-0.8, 0.8, size=(S, ndim))
    a2bar = dt * rng.uniform(0.0, 0.5, size=S)
    return n, lo, hi, dt, S, V0, psi0, target, abar, a2bar


def _vg_loss(p, abar, a2bar, V0=None):
    n, lo, hi, dt, S, V, psi0, target, _, _ = p
    psiT = orc.schrodinger_velocity(psi0, n, lo, hi, dt, V if V0 is None else V0, abar, a2bar, nsteps=S)
    dv = np.prod([(hi[a] - lo[a]) / n[a] for a in range(len(n))])
    ov = dv * np.vdot(target, psiT)
    return abs(ov) ** 2, psiT, 2 * ov * target * dv


def test_velocity_gradient_matches_central_differences():
    """dL/dAbar_{n,a}, dL/dA2bar_n and dL/dV0 of |<target|psi_T>|^2 from the
    stored trajectory against central differences of the forward run (1-D
    and 2-D, every step and axis of Abar, several steps of A2bar and points of V0)."""
    for n in ((64,), (32, 16)):
        p = _vg_problem(n)
        _, lo, hi, dt, S, V0, psi0, target, abar, a2bar = p
        L0, psiT, gT = _vg_loss(p, abar, a2bar)
        _, da, da2, dV = orc.schrodinger_velocity_adjoint(psi0, gT, n, lo, hi, dt, V0, abar, a2bar, nsteps=S)
        h = 1e-6
        for j in range(S):
            for a in range(len(n)):
                ap, am = abar.copy(), abar.copy()
                ap[j, a] += h
                am[j, a] -= h
                fd = (_vg_loss(p, ap, a2bar)[0] - _vg_loss(p, am, a2bar)[0]) / (2 * h)
                assert abs(fd - da[j, a]) < 1e-7 * max(1.0, np.abs(da).max()), (n, j, a, fd, da[j, a])
        # A2bar enters each step as a global phase: a phase-blind loss does not see it
        assert np.abs(da2).max() < 1e-12 * np.abs(da).max()
        for j in (0, S // 2, S - 1):
            ap, am = a2bar.copy(), a2bar.copy()
            ap[j] += h
            am[j] -= h
            fd = (_vg_loss(p, abar, ap)[0] - _vg_loss(p, abar, am)[0]) / (2 * h)
            assert abs(fd - da2[j]) < 1e-7
        flat = V0.ravel()
        for i in (0, flat.size // 3, flat.size // 2 + 1):
            vp, vm = flat.copy(), flat.copy()
            vp[i] += h
            vm[i] -= h
            fd = (_vg_loss(p, abar, a2bar, vp.reshape(V0.shape))[0] -
                  _vg_loss(p, abar, a2bar, vm.reshape(V0.shape))[0]) / (2 * h)
            assert abs(fd - dV.ravel()[i]) < 1e-7 * max(1.0, np.abs(dV).max()), (n, i)
        assert abs(dV.sum()) < 1e-10 * np.abs(dV).sum()  # global-phase invariance


def test_velocity_adjoint_state_is_the_transpose_of_the_run():
    """The returned adjoint at step 0 is S^dagger applied to gT: for any state d,
    <g0 | d> = <gT | S d> (the run is linear), exactly to rounding."""
    p = _vg_problem((32, 16), seed=3)
    n, lo, hi, dt, S, V0, psi0, target, abar, a2bar = p
    rng = np.random.default_rng(11)
    gT = rng.normal(size=psi0.shape) + 1j * rng.normal(size=psi0.shape)
    d = rng.normal(size=psi0.shape) + 1j * rng.normal(size=psi0.shape)
    g0, _, _, _ = orc.schrodinger_velocity_adjoint(psi0, gT, n, lo, hi, dt, V0, abar, a2bar, nsteps=S)
    Sd = orc.schrodinger_velocity(d, n, lo, hi, dt, V0, abar, a2bar, nsteps=S)
    lhs, rhs = np.vdot(g0, d), np.vdot(gT, Sd)
    assert abs(lhs - rhs) < 1e-12 * abs(rhs)


def test_velocity_gradient_phase_sensitive_loss():
    """L = Re <target|psi_T> sees the global phase each step's A2bar adds:
    dL/dA2bar_n and dL/dAbar_{n,a} against central differences."""
    p = _vg_problem((32, 16), seed=5)
    n, lo, hi, dt, S, V0, psi0, target, abar, a2bar = p
    dv = np.prod([(hi[a] - lo[a]) / n[a] for a in range(2)])

    def loss(ab, a2):
        psiT = orc.schrodinger_velocity(psi0, n, lo, hi, dt, V0, ab, a2, nsteps=S)
        return float(np.real(dv * np.vdot(target, psiT)))

    _, da, da2, _ = orc.schrodinger_velocity_adjoint(psi0, dv * target, n, lo, hi, dt, V0, abar, a2bar, nsteps=S)
    assert np.abs(da2).max() > 1e-3
    h = 1e-6
    for j in range(S):
        ap, am = a2bar.copy(), a2bar.copy()
        ap[j] += h
        am[j] -= h
        assert abs((loss(abar, ap) - loss(abar, am)) / (2 * h) - da2[j]) < 1e-8
        bp, bm = abar.copy(), abar.copy()
        bp[j, 1] += h
        bm[j, 1] -= h
        assert abs((loss(bp, a2bar) - loss(bm, a2bar)) / (2 * h) - da[j, 1]) < 1e-8
