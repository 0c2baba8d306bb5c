"""1-D two-component Dirac runs on the GPU (one work-group per line) against
the oracle's 1-D Dirac step: a bound packet in a soft-core well driven by a
travelling vector potential A_1(x, t)."""
import numpy as np
import pytest

import oracle as orc
from paper_1012_3911_amd import workloads as W
from gpu_util import make_grid, rel_l2, to_device

pytestmark = pytest.mark.gpu

C = 137.036


def _wl(N, S, dt=2e-4, L=10.0, A0=30.0):
    x = -L + 2 * L / N * np.arange(N)
    V0 = -1.0 / np.sqrt(x ** 2 + 1.0)
    up = np.exp(-x ** 2 / 2 + 1.5j * x)
    psi0 = np.stack([up, 0.004 * (1.5 - 1j * x) * np.exp(-x ** 2 / 2)]).astype(complex)
    t = dt * (np.arange(S) + 0.5)
    abar = dt * A0 * np.sin(0.8 * x[None, :] - 40.0 * t[:, None])  # midpoint rule
    wl = W.Workload("d1", "dirac", (N,), (-L,), (L,), dt, S, V0, psi0, abar_y=abar, c=C)
    return wl


@pytest.mark.parametrize("dtype,N,S,tol", [("c128", 1024, 200, 1e-12), ("c64", 1024, 200, 1e-5),
                                           ("c128", 64, 50, 1e-12), ("c128", 8192, 20, 1e-12),
                                           ("c128", 4096, 20, 1e-12)])
def test_dirac1d_matches_oracle(dtype, N, S, tol):
    import torch

    wl = _wl(N, S)
    g = make_grid(wl, dtype)
    psi = to_device(wl.psi0, dtype)
    g.propagate(psi, 0, S)
    torch.cuda.synchronize()
    p0 = wl.psi0.astype(np.complex64).astype(complex) if dtype == "c64" else wl.psi0
    ref = orc.dirac1d(p0, (N,), wl.xmin, wl.xmax, wl.dt, wl.V0, wl.abar_y, nsteps=S, c=C)
    err = rel_l2(psi.cpu().numpy(), ref)
    print("dirac1d %s N=%d %d steps: rel L2 vs oracle %.3e" % (dtype, N, S, err), flush=True)
    assert err < tol
    if dtype == "c128":
        assert abs(g.norm(psi) / g.norm(to_device(wl.psi0, dtype)) - 1) < 1e-12
    g.close()


def test_dirac1d_steps_from_an_offset():
    """A run of steps 30..59 equals the oracle's steps 30..59 of the same
    vector-potential table."""
    import torch

    wl = _wl(512, 60)
    g = make_grid(wl, "c128")
    psi = to_device(wl.psi0, "c128")
    g.propagate(psi, 30, 30)
    torch.cuda.synchronize()
    ref = orc.dirac1d(wl.psi0, (512,), wl.xmin, wl.xmax, wl.dt, wl.V0, wl.abar_y, step0=30, nsteps=30, c=C)
    assert rel_l2(psi.cpu().numpy(), ref) < 1e-12
    g.close()


def test_free_positive_energy_packet_group_velocity():
    """The GPU run of a free positive-energy packet moves its centre of mass
    by S tau <c^2 p / E> (complex128)."""
    import torch
    from test_oracle_dirac1d import _positive_energy_packet

    N, L, c, dt, S = 1024, 40.0, 5.0, 0.01, 400
    x, k, E, psi0 = _positive_energy_packet(N, L, 2.0, 0.6, c)
    wl = W.Workload("free", "dirac", (N,), (-L,), (L,), dt, S, np.zeros(N), psi0, abar_y=None, c=c)
    g = make_grid(wl, "c128")
    psi = to_device(psi0, "c128")
    g.propagate(psi, 0, S)
    torch.cuda.synchronize()
    out = psi.cpu().numpy()
    rho0, rho1 = np.sum(np.abs(psi0) ** 2, axis=0), np.sum(np.abs(out) ** 2, axis=0)
    shift = np.sum(x * rho1) / np.sum(rho1) - np.sum(x * rho0) / np.sum(rho0)
    w = np.sum(np.abs(np.fft.fft(psi0, axis=1)) ** 2, axis=0)
    vg = np.sum(w * c * c * k / E) / np.sum(w)
    assert abs(shift - S * dt * vg) < 1e-9
    g.close()
