"""sfo_adjoint_noalloc: the reverse sweep with its moment partials in the
library's static per-device scratch array instead of a buffer the handle
allocates.  It runs the kernels of sfo_adjoint in the same order, so on the
same inputs its outputs (recomputed psi(0), the adjoint at step 0, dL/dEbar,
dL/dV0) must equal sfo_adjoint's bit for bit.  Checked on calls in a row on
one device, each smaller than the one before (the array keeps the previous
call's contents), and the refusal of a run whose partials exceed the array."""
import numpy as np
import pytest

from paper_1012_3911_amd import workloads as W
from gpu_util import make_grid, to_device

pytestmark = pytest.mark.gpu


def _problem(n, nsteps, seed):
    ndim = len(n)
    lo = tuple(-0.1 * n[a] for a in range(ndim))
    hi = tuple(0.1 * n[a] for a in range(ndim))
    X = W.mesh(n, lo, hi)
    V0 = -1.0 / np.sqrt(sum(x ** 2 for x in X) + 1.0)
    psi0 = W.gaussian(n, lo, hi, (0.0,) * ndim, 1.0, (0.4,) + (0.0,) * (ndim - 1))
    target = W.gaussian(n, lo, hi, (0.6,) + (0.0,) * (ndim - 1), 1.0, (0.0,) * ndim)
    dt = 0.05
    rng = np.random.default_rng(seed)
    ebar = dt * rng.uniform(-0.2, 0.2, size=(nsteps, ndim))
    return W.Workload("noalloc", "schrodinger", n, lo, hi, dt, nsteps, V0, psi0, ebar=ebar), target


def _sweep(wl, target, dtype, noalloc):
    import torch

    g = make_grid(wl, dtype)
    psi = to_device(wl.psi0, dtype)
    g.propagate(psi, 0, wl.nsteps)
    torch.cuda.synchronize()
    ov = wl.dv * np.vdot(target, psi.cpu().numpy().astype(np.complex128))
    gv = to_device(2 * ov * target * wl.dv, dtype)
    if noalloc:
        de = torch.zeros((wl.nsteps, wl.ndim), dtype=torch.float64, device="cuda")
        dv = torch.zeros(wl.n[::-1], dtype=torch.float64, device="cuda")
        g.adjoint_noalloc(psi, gv, 0, wl.nsteps, de, dv)
    else:
        de, dv = g.adjoint(psi, gv, 0, wl.nsteps)
    torch.cuda.synchronize()
    out = [psi.cpu().numpy(), gv.cpu().numpy(), de.cpu().numpy(), dv.cpu().numpy()]
    g.close()
    return out


CALLS = [((256, 128), 40, "c64"), ((128, 64), 12, "c64"), ((512,), 30, "c128"), ((256,), 8, "c128")]


def test_noalloc_adjoint_equals_adjoint_on_calls_in_a_row():
    for i, (n, nsteps, dtype) in enumerate(CALLS):
        print("noalloc call %d: grid %s, %d steps, %s" % (i, n, nsteps, dtype), flush=True)
        wl, target = _problem(n, nsteps, seed=i)
        ref = _sweep(wl, target, dtype, noalloc=False)
        got = _sweep(wl, target, dtype, noalloc=True)
        for name, a, b in zip(("psi0", "g0", "dL/dEbar", "dL/dV0"), got, ref):
            assert a.shape == b.shape, (i, name)
            assert np.array_equal(a, b), (i, name, float(np.abs(a - b).max()))
        assert np.abs(ref[2]).max() > 0 and np.abs(ref[3]).max() > 0


def test_noalloc_adjoint_refuses_runs_beyond_the_scratch_array():
    import torch

    from paper_1012_3911_amd import sfo

    wl, _ = _problem((256,), 4, seed=9)
    g = make_grid(wl, "c128")
    g.set_field(None)  # no table: every step is in range
    psi = to_device(wl.psi0, "c128")
    gv = to_device(wl.psi0, "c128")
    nsteps = 1 << 20  # 3 (nsteps + 1) doubles > 2^21
    # full-size output, so that nothing could be written out of bounds even if the check were missing
    de = torch.zeros((nsteps, 1), dtype=torch.float64, device="cuda")
    with pytest.raises(sfo.SfoError) as ei:
        g.adjoint_noalloc(psi, gv, 0, nsteps, de)
    assert ei.value.status == sfo.SFO_E_UNSUPPORTED
    assert "scratch" in str(ei.value)
    g.close()
