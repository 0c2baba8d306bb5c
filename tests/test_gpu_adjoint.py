"""GPU adjoint against the oracle's stored-trajectory gradient and finite differences.

The library walks psi and the adjoint back with the exact inverse step; the
oracle stores the FP64 forward trajectory instead (a different algorithm).
Loss: L = |<target|psi_T>|^2.  Tolerances: complex128 1e-11 relative,
complex64 1e-4 relative (the gradient target), FD 1e-4."""
import numpy as np
import pytest

from paper_1012_3911_amd import workloads as W
from gpu_util import make_grid, rel_l2, to_device

pytestmark = pytest.mark.gpu


def problem(ndim, n=None):
    if ndim == 1:
        n, lo, hi = n or (256,), (-20.0,), (20.0,)
    elif ndim == 2:
        n, lo, hi = n or (128, 64), (-12.8, -9.6), (12.8, 9.6)
    else:
        n, lo, hi = n or (64, 64, 64), (-9.6, -9.6, -9.6), (9.6, 9.6, 9.6)
    X = W.mesh(n, lo, hi)
    r2 = sum(x**2 for x in X)
    V0 = -1.0 / np.sqrt(r2 + 1.0)
    psi0 = W.gaussian(n, lo, hi, (0.0,) * ndim, 1.0, (0.3,) + (0.0,) * (ndim - 1))
    target = W.gaussian(n, lo, hi, (0.7,) + (0.0,) * (ndim - 1), 1.0, (0.0,) * ndim)
    ns, dt = 24, 0.05
    rng = np.random.default_rng(ndim)
    ebar = dt * rng.uniform(-0.3, 0.3, size=(ns, ndim))
    wl = W.Workload("adj", "schrodinger", n, lo, hi, dt, ns, V0, psi0, ebar=ebar)
    return wl, target


def loss_grad(psiT, target, dv):
    ov = dv * np.vdot(target, psiT)
    return abs(ov) ** 2, 2 * ov * target * dv


def oracle_grads(orc, wl, target):
    psiT = orc.schrodinger(wl.psi0, wl.n, wl.xmin, wl.xmax, wl.dt, wl.V0, wl.ebar, nsteps=wl.nsteps)
    L, gT = loss_grad(psiT, target, wl.dv)
    g0, dE, dV = orc.schrodinger_adjoint(wl.psi0, gT, wl.n, wl.xmin, wl.xmax, wl.dt, wl.V0, wl.ebar,
                                         nsteps=wl.nsteps)
    return psiT, gT, g0, dE, dV


def gpu_grads(wl, psiT, gT, dtype):
    import torch

    g = make_grid(wl, dtype)
    psi = to_device(psiT, dtype)
    gv = to_device(gT, dtype)
    dE, dV = g.adjoint(psi, gv, 0, wl.nsteps)
    torch.cuda.synchronize()
    out = (psi.cpu().numpy().astype(np.complex128), gv.cpu().numpy().astype(np.complex128),
           dE.cpu().numpy(), dV.cpu().numpy())
    g.close()
    return out


@pytest.mark.parametrize("dtype", ["c128", "c64"])
@pytest.mark.parametrize("ndim", [1, 2, 3])
def test_adjoint_matches_oracle(orc, ndim, dtype):
    wl, target = problem(ndim)
    psiT, gT, g0, dE, dV = oracle_grads(orc, wl, target)
    if dtype == "c64":
        # feed the c64 path the c64-rounded forward result
        psiT = psiT.astype(np.complex64).astype(np.complex128)
    p0, gg0, gdE, gdV = gpu_grads(wl, psiT, gT, dtype)
    tol = 1e-11 if dtype == "c128" else 1e-4
    assert rel_l2(p0, wl.psi0) < (1e-12 if dtype == "c128" else 1e-5)
    assert rel_l2(gg0, g0) < tol
    assert np.linalg.norm(gdE - dE) / np.linalg.norm(dE) < tol
    assert np.linalg.norm((gdV - dV).ravel()) / np.linalg.norm(dV.ravel()) < tol
    # global-phase invariance: sum_x dL/dV0 = 0
    assert abs(gdV.sum()) < 1e-6 * np.abs(gdV).sum()


def test_adjoint_finite_differences_gpu():
    """Central differences of the GPU forward (complex128) against the GPU adjoint."""
    import torch

    wl, target = problem(2)
    g = make_grid(wl, "c128")

    def loss(ebar):
        g.set_field(ebar)
        psi = to_device(wl.psi0, "c128")
        g.propagate(psi, 0, wl.nsteps)
        torch.cuda.synchronize()
        return loss_grad(psi.cpu().numpy(), target, wl.dv)

    L0, gT = loss(wl.ebar)
    g.set_field(wl.ebar)
    psi = to_device(wl.psi0, "c128")
    g.propagate(psi, 0, wl.nsteps)
    gv = to_device(gT, "c128")
    dE, dV = g.adjoint(psi, gv, 0, wl.nsteps)
    dE = dE.cpu().numpy()
    h = 1e-6
    for s, a in [(0, 0), (5, 1), (11, 0), (23, 1)]:
        ep, em = wl.ebar.copy(), wl.ebar.copy()
        ep[s, a] += h
        em[s, a] -= h
        fd = (loss(ep)[0] - loss(em)[0]) / (2 * h)
        assert abs(fd - dE[s, a]) <= 1e-4 * abs(fd) + 1e-9, (s, a, fd, dE[s, a])
    g.close()


@pytest.mark.parametrize("dtype", ["c128", "c64"])
def test_autograd_control_gradient(orc, dtype):
    """torch.autograd through SplitStep: gradient of |<target|psi_T>|^2 with respect to a
    piecewise-constant control (amplitudes held 2 steps) and V0, against the oracle."""
    import torch
    from paper_1012_3911_amd import autograd as AG

    wl, target = problem(1, n=(512,))
    nsteps = wl.nsteps
    amps = torch.tensor(np.random.default_rng(3).uniform(-0.05, 0.05, nsteps // 2), dtype=torch.float64,
                        requires_grad=True)
    V0 = torch.tensor(wl.V0, dtype=torch.float64, device="cuda", requires_grad=True)
    grid = make_grid(wl, dtype)
    ebar = (wl.dt * amps.repeat_interleave(2)).reshape(nsteps, 1)
    psi0 = to_device(wl.psi0, dtype)
    psiT = AG.propagate(psi0, ebar, V0, grid)
    tt = to_device(target, dtype)
    ov = wl.dv * torch.sum(tt.conj() * psiT)
    L = (ov.real ** 2 + ov.imag ** 2)
    L.backward()
    # oracle: chain rule dL/damp_k = dt * (dL/dEbar_{2k} + dL/dEbar_{2k+1})
    e_np = ebar.detach().numpy()
    wl.ebar = e_np
    _, _, _, dE, dV = oracle_grads(orc, wl, target)
    ref_amp = wl.dt * (dE[0::2, 0] + dE[1::2, 0])
    tol = 1e-9 if dtype == "c128" else 1e-4
    got = amps.grad.numpy()
    assert np.linalg.norm(got - ref_amp) / np.linalg.norm(ref_amp) < tol
    gv = V0.grad.cpu().numpy()
    assert np.linalg.norm(gv - dV) / np.linalg.norm(dV) < tol
    grid.close()


@pytest.mark.parametrize("dtype", ["c128", "c64"])
def test_adjoint_after_autotune(orc, dtype):
    """The autotuner picks the reverse sweep's two-state shapes separately from
    the forward ones; the gradient must not depend on that choice."""
    import torch

    wl, target = problem(2, n=(256, 128))
    psiT, gT, g0, dE, dV = oracle_grads(orc, wl, target)
    if dtype == "c64":
        psiT = psiT.astype(np.complex64).astype(np.complex128)
    g = make_grid(wl, dtype)
    g.autotune(2)
    psi = to_device(psiT, dtype)
    gv = to_device(gT, dtype)
    gdE, gdV = g.adjoint(psi, gv, 0, wl.nsteps)
    torch.cuda.synchronize()
    tol = 1e-11 if dtype == "c128" else 1e-4
    assert rel_l2(gv.cpu().numpy(), g0) < tol
    assert np.linalg.norm(gdE.cpu().numpy() - dE) / np.linalg.norm(dE) < tol
    assert np.linalg.norm((gdV.cpu().numpy() - dV).ravel()) / np.linalg.norm(dV.ravel()) < tol
    g.close()


def test_autograd_two_forward_calls_on_one_grid(orc):
    """Two differentiable runs with different controls on ONE grid before a single
    backward: each run's gradient must be taken with the potential and field that
    run used (the grid's tables are re-installed), matching the oracle."""
    import torch
    from paper_1012_3911_amd import autograd as AG

    wl, target = problem(1, n=(512,))
    ns = wl.nsteps
    grid = make_grid(wl, "c128")
    rng = np.random.default_rng(7)
    e1 = torch.tensor(rng.uniform(-0.02, 0.02, (ns, 1)), dtype=torch.float64, requires_grad=True)
    e2 = torch.tensor(rng.uniform(-0.02, 0.02, (ns, 1)), dtype=torch.float64, requires_grad=True)
    V1 = torch.tensor(wl.V0, dtype=torch.float64, device="cuda", requires_grad=True)
    V2 = torch.tensor(0.5 * wl.V0, dtype=torch.float64, device="cuda", requires_grad=True)
    psi0 = to_device(wl.psi0, "c128")
    tt = to_device(target, "c128")
    L = 0.0
    for e, V in ((e1, V1), (e2, V2)):
        psiT = AG.propagate(psi0, e, V, grid)
        ov = wl.dv * torch.sum(tt.conj() * psiT)
        L = L + ov.real ** 2 + ov.imag ** 2
    L.backward()
    for e, V, vscale in ((e1, V1, 1.0), (e2, V2, 0.5)):
        wl.ebar = e.detach().numpy()
        wl.V0 = vscale * problem(1, n=(512,))[0].V0
        _, _, _, dE, dV = oracle_grads(orc, wl, target)
        assert np.linalg.norm(e.grad.numpy() - dE) / np.linalg.norm(dE) < 1e-9
        assert np.linalg.norm(V.grad.cpu().numpy() - dV) / np.linalg.norm(dV) < 1e-9
    grid.close()
