"""Pins for the oracle's stored-trajectory gradient.

Loss L = |<target|psi_T>|^2 of a final-state overlap, differentiated with
respect to the per-step field integrals Ebar_n, the static potential V0 and
the initial state.  Pins:
  * central finite differences of the oracle's forward run;
  * sum_x dL/dV0(x) = 0 exactly: a constant shift of V0 only changes the
    global phase of psi_T, which L ignores;
  * an affine field change: d/ds L(Ebar + s dE) equals <dL/dEbar, dE>.
"""
import numpy as np
import pytest

from paper_1012_3911_amd import workloads as W


def loss_and_grad(psiT, target, dv):
    """L = |dv sum conj(t) psi|^2 and g = 2 dL/dconj(psi) = 2 ov * t dv."""
    ov = dv * np.vdot(target, psiT)
    return abs(ov) ** 2, 2 * ov * target * dv


def small_problem(ndim):
    if ndim == 1:
        n, lo, hi = (64,), (-12.0,), (12.0,)
    else:
        n, lo, hi = (16, 8), (-8.0, -6.0), (8.0, 6.0)
    X = W.mesh(n, lo, hi)
    r2 = sum(x**2 for x in X)
    V0 = -1.0 / np.sqrt(r2 + 1.0)
    psi0 = W.gaussian(n, lo, hi, (0.0,) * ndim, 1.0, (0.2,) + (0.0,) * (ndim - 1))
    target = W.gaussian(n, lo, hi, (0.8,) + (0.0,) * (ndim - 1), 1.0, (0.0,) * ndim)
    ns, dt = 24, 0.05
    rng = np.random.default_rng(ndim)
    ebar = dt * rng.uniform(-0.3, 0.3, size=(ns, ndim))
    return n, lo, hi, V0, psi0, target, ns, dt, ebar


def run_loss(orc, n, lo, hi, dt, V0, ebar, psi0, target, ns):
    psiT = orc.schrodinger(psi0, n, lo, hi, dt, V0, ebar, nsteps=ns)
    dv = float(np.prod([(b - a) / m for a, b, m in zip(lo, hi, n)]))
    return loss_and_grad(psiT, target, dv)


@pytest.mark.parametrize("ndim", [1, 2])
def test_adjoint_vs_finite_differences(orc, ndim):
    n, lo, hi, V0, psi0, target, ns, dt, ebar = small_problem(ndim)
    L0, gT = run_loss(orc, n, lo, hi, dt, V0, ebar, psi0, target, ns)
    g0, dE, dV = orc.schrodinger_adjoint(psi0, gT, n, lo, hi, dt, V0, ebar, nsteps=ns)
    h = 1e-6
    rng = np.random.default_rng(11)
    # field integrals
    for _ in range(6):
        s, a = rng.integers(ns), rng.integers(ndim)
        ep, em = ebar.copy(), ebar.copy()
        ep[s, a] += h
        em[s, a] -= h
        fd = (run_loss(orc, n, lo, hi, dt, V0, ep, psi0, target, ns)[0]
              - run_loss(orc, n, lo, hi, dt, V0, em, psi0, target, ns)[0]) / (2 * h)
        assert abs(fd - dE[s, a]) <= 1e-8 + 1e-6 * abs(fd), (fd, dE[s, a])
    # potential values
    flat = V0.ravel()
    for _ in range(6):
        i = rng.integers(flat.size)
        vp, vm = flat.copy(), flat.copy()
        vp[i] += h
        vm[i] -= h
        fd = (run_loss(orc, n, lo, hi, dt, vp.reshape(V0.shape), ebar, psi0, target, ns)[0]
              - run_loss(orc, n, lo, hi, dt, vm.reshape(V0.shape), ebar, psi0, target, ns)[0]) / (2 * h)
        assert abs(fd - dV.ravel()[i]) <= 1e-9 + 1e-6 * abs(fd), (fd, dV.ravel()[i])
    # initial state: dL = Re <g0, dpsi0>
    for _ in range(4):
        i = rng.integers(psi0.size)
        for d in (1.0, 1j):
            pp, pm = psi0.copy().ravel(), psi0.copy().ravel()
            pp[i] += h * d
            pm[i] -= h * d
            fd = (run_loss(orc, n, lo, hi, dt, V0, ebar, pp.reshape(psi0.shape), target, ns)[0]
                  - run_loss(orc, n, lo, hi, dt, V0, ebar, pm.reshape(psi0.shape), target, ns)[0]) / (2 * h)
            an = float(np.real(np.conj(g0.ravel()[i]) * d))
            assert abs(fd - an) <= 1e-8 + 1e-6 * abs(fd), (fd, an)


@pytest.mark.parametrize("ndim", [1, 2])
def test_potential_gradient_sums_to_zero(orc, ndim):
    n, lo, hi, V0, psi0, target, ns, dt, ebar = small_problem(ndim)
    L0, gT = run_loss(orc, n, lo, hi, dt, V0, ebar, psi0, target, ns)
    _, _, dV = orc.schrodinger_adjoint(psi0, gT, n, lo, hi, dt, V0, ebar, nsteps=ns)
    assert abs(dV.sum()) < 1e-12 * np.abs(dV).sum() * 10
    assert np.abs(dV).max() > 1e-6  # nontrivial


def test_directional_field_derivative(orc):
    n, lo, hi, V0, psi0, target, ns, dt, ebar = small_problem(1)
    L0, gT = run_loss(orc, n, lo, hi, dt, V0, ebar, psi0, target, ns)
    _, dE, _ = orc.schrodinger_adjoint(psi0, gT, n, lo, hi, dt, V0, ebar, nsteps=ns)
    d = np.random.default_rng(2).standard_normal(ebar.shape) * dt
    h = 1e-5
    fd = (run_loss(orc, n, lo, hi, dt, V0, ebar + h * d, psi0, target, ns)[0]
          - run_loss(orc, n, lo, hi, dt, V0, ebar - h * d, psi0, target, ns)[0]) / (2 * h)
    assert abs(fd - np.sum(dE * d)) < 1e-6 * abs(fd) + 1e-9
