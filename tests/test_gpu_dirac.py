"""GPU parity of the 2-D Dirac 4-spinor split step against the FP64 oracle.

Workload: soft-core nucleus (Z = 20), a laser pulse with A along y travelling
along x (per-step integrals of A_y(x, t)), a positive-energy spin-up packet.
Tolerances: complex128 <= 1e-12 relative L2, complex64 <= 1e-5."""
import numpy as np
import pytest

from paper_1012_3911_amd import workloads as W
from gpu_util import gpu_run, make_grid, oracle_run, rel_l2, to_device

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("dtype", ["c128", "c64"])
def test_dirac_small(orc, dtype):
    wl = W.dirac_softcore_laser(n=128, nsteps=40)
    ref = oracle_run(orc, wl)
    got = gpu_run(wl, dtype)
    assert rel_l2(got, ref) < (1e-12 if dtype == "c128" else 1e-5)


@pytest.mark.parametrize("dtype", ["c128", "c64"])
def test_dirac_long_potential_phase(orc, dtype):
    """A step forty times the workload's: the row pass's potential phase
    |tau V0 / hbar| reaches 0.2 near the nucleus (5e-3 at the workload's step),
    against the oracle."""
    wl = W.dirac_softcore_laser(n=128, nsteps=12, dt=4e-4)
    assert wl.dt * np.abs(wl.V0).max() > 0.125
    ref = oracle_run(orc, wl)
    got = gpu_run(wl, dtype)
    assert rel_l2(got, ref) < (1e-12 if dtype == "c128" else 1e-5)


@pytest.mark.parametrize("dtype", ["c128", "c64"])
def test_dirac_anisotropic(orc, dtype):
    """nx != ny and unequal box lengths pin the k_x/k_y and plane indexing."""
    wl = W.dirac_softcore_laser(n=128, nsteps=16)
    n, lo, hi = (256, 64), (-2.0, -1.0), (2.0, 1.0)
    X, Y = W.mesh(n, lo, hi)
    wl.n, wl.xmin, wl.xmax = n, lo, hi
    wl.V0 = -20.0 / np.sqrt(X**2 + Y**2 + (0.791 / 20) ** 2)
    wl.psi0 = W.dirac_packet(n, lo, hi, (40.0, -15.0), 60.0, 30.0)
    (x,) = W.axes((n[0],), (lo[0],), (hi[0],))
    tmid = (np.arange(wl.nsteps) + 0.5) * wl.dt
    wl.abar_y = np.stack([wl.dt * W.laser_vector_potential(x, t) for t in tmid])
    ref = oracle_run(orc, wl)
    got = gpu_run(wl, dtype)
    assert rel_l2(got, ref) < (1e-12 if dtype == "c128" else 1e-5)


def test_dirac_unfused_and_stepwise():
    from paper_1012_3911_amd import sfo

    wl = W.dirac_softcore_laser(n=128, nsteps=8)
    a = gpu_run(wl, "c128")
    b = gpu_run(wl, "c128", flags=sfo.UNFUSED)
    c = gpu_run(wl, "c128", stepwise=True)
    assert rel_l2(a, b) < 1e-14 and rel_l2(a, c) < 1e-14


@pytest.mark.parametrize("dtype", ["c128", "c64"])
def test_dirac_every_tile_shape(orc, dtype):
    """Every row and column tile shape of the Dirac passes (four planes per
    work-group, or one coupled pair (1,4) / (2,3); radix 8 or 16) gives the
    oracle's result on an anisotropic grid with the vector potential, and the
    autotuner picks one of them."""
    import torch
    from paper_1012_3911_amd import sfo

    wl = W.dirac_softcore_laser(n=128, nsteps=12)
    n, lo, hi = (512, 256), (-4.0, -2.0), (4.0, 2.0)
    X, Y = W.mesh(n, lo, hi)
    wl.n, wl.xmin, wl.xmax = n, lo, hi
    wl.V0 = -20.0 / np.sqrt(X**2 + Y**2 + (0.791 / 20) ** 2)
    wl.psi0 = W.dirac_packet(n, lo, hi, (40.0, -15.0), 60.0, 30.0)
    (x,) = W.axes((n[0],), (lo[0],), (hi[0],))
    tmid = (np.arange(wl.nsteps) + 0.5) * wl.dt
    wl.abar_y = np.stack([wl.dt * W.laser_vector_potential(x, t) for t in tmid])
    ref = oracle_run(orc, wl)
    tol = 1e-12 if dtype == "c128" else 1e-5
    g = make_grid(wl, dtype)
    tried = []
    for r in range(8):
        for c in range(8):
            try:
                g.plan = (r, c, 0)
            except sfo.SfoError:
                continue
            psi = to_device(wl.psi0, dtype)
            g.propagate(psi, 0, wl.nsteps)
            torch.cuda.synchronize()
            err = rel_l2(psi.cpu().numpy(), ref)
            print("dirac shapes (%d, %d): rel L2 vs oracle %.3e" % (r, c, err), flush=True)
            assert err < tol, (r, c, err)
            tried.append((r, c))
    assert len(tried) >= 20, tried
    g.autotune(3)
    assert tuple(g.plan[:2]) in tried
    psi = to_device(wl.psi0, dtype)
    g.propagate(psi, 0, wl.nsteps)
    torch.cuda.synchronize()
    assert rel_l2(psi.cpu().numpy(), ref) < tol
    g.close()
