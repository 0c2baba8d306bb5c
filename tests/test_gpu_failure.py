"""Failure detection forced from the host (no kernel is made to fail):
non-finite values in a state reported by sfo_norm / sfo_overlap, the norm
watch of a handle, and device allocation failures injected with
SFO_FAIL_ALLOC=<n> (the n-th allocation of one ABI call fails before the
runtime is asked), which must leave nothing allocated and the library usable."""
import os

import numpy as np
import pytest

from paper_1012_3911_amd import workloads as W
from gpu_util import make_grid, to_device

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("dtype", ["c128", "c64"])
@pytest.mark.parametrize("bad", [float("nan"), float("inf")])
def test_nonfinite_state_is_reported(dtype, bad):
    from paper_1012_3911_amd import sfo

    wl = W.softcore_2d_laser(n=128, nsteps=4, L=20.0)
    g = make_grid(wl, dtype)
    psi = to_device(wl.psi0, dtype)
    good = g.norm(psi)
    assert np.isfinite(good)
    psi[77, 13] = complex(bad, 0.0)
    with pytest.raises(sfo.SfoError) as ei:
        g.norm(psi)
    assert ei.value.status == sfo.SFO_E_NUMERIC
    with pytest.raises(sfo.SfoError) as ei:
        g.overlap(to_device(wl.psi0, dtype), psi)
    assert ei.value.status == sfo.SFO_E_NUMERIC
    g.close()


def test_norm_watch():
    from paper_1012_3911_amd import sfo

    wl = W.softcore_2d_laser(n=256, nsteps=100, L=40.0)
    for dtype, tol in (("c128", 1e-12), ("c64", 1e-6)):
        g = make_grid(wl, dtype)
        psi = to_device(wl.psi0, dtype)
        n0 = g.norm(psi)
        g.set_norm_watch(n0, tol)
        g.propagate(psi, 0, wl.nsteps)
        assert abs(g.norm(psi) / n0 - 1) <= tol  # a unitary run stays inside the band
        psi.mul_(1.0 + 100 * tol)
        with pytest.raises(sfo.SfoError) as ei:
            g.norm(psi)
        assert ei.value.status == sfo.SFO_E_NUMERIC and "drifted" in str(ei.value)
        g.set_norm_watch(0.0, 0.0)  # off
        g.norm(psi)
        for ref, t in ((-1.0, 1e-6), (1.0, -1e-6), (float("nan"), 1e-6), (1.0, float("inf"))):
            with pytest.raises(sfo.SfoError) as ei:
                g.set_norm_watch(ref, t)
            assert ei.value.status == sfo.SFO_E_INVALID
        g.close()


def _free_bytes():
    import torch

    torch.cuda.synchronize()
    return torch.cuda.mem_get_info()[0]


def test_injected_allocation_failures_leave_nothing_behind(orc):
    import torch

    from paper_1012_3911_amd import sfo

    wl = W.softcore_2d_laser(n=256, nsteps=6, L=40.0)
    # load every code object and the library's per-device state first
    g = make_grid(wl, "c64")
    psi = to_device(wl.psi0, "c64")
    g.propagate(psi, 0, wl.nsteps)
    g.adjoint(psi, (0.5 * psi).contiguous(), 0, wl.nsteps)
    g.close()
    del psi
    torch.cuda.empty_cache()
    free0 = _free_bytes()
    try:
        # grid creation: fail each of its allocations in turn until one passes them all
        created_at = None
        for k in range(1, 64):
            os.environ["SFO_FAIL_ALLOC"] = str(k)
            try:
                g = sfo.Grid(wl.n, wl.xmin, wl.xmax, wl.dt, dtype="c64")
            except sfo.SfoError as e:
                assert e.status == sfo.SFO_E_NOMEM, str(e)
                continue
            created_at = k
            g.close()
            break
        print("sfo_create_grid makes %d device allocations" % (created_at - 1), flush=True)
        assert created_at is not None and created_at > 3
        # the first reverse sweep allocates its partial slots: make that fail, then succeed.
        # Loss |<target|psi_T>|^2 with the target the initial packet moved along x (a loss
        # of the norm alone would have an identically zero field gradient).
        os.environ.pop("SFO_FAIL_ALLOC")
        g = make_grid(wl, "c128")
        psi = to_device(wl.psi0, "c128")
        g.propagate(psi, 0, wl.nsteps)
        target = W.gaussian(wl.n, wl.xmin, wl.xmax, (1.0, 0.0), 1.0, (0.0, 0.0))
        ov = wl.dv * np.vdot(target, psi.cpu().numpy())
        gT = 2 * ov * target * wl.dv
        gv = to_device(gT, "c128")
        os.environ["SFO_FAIL_ALLOC"] = "1"
        with pytest.raises(sfo.SfoError) as ei:
            g.adjoint(psi.clone(), gv.clone(), 0, wl.nsteps)
        assert ei.value.status == sfo.SFO_E_NOMEM
        # a table upload fails and leaves the previous table in place
        with pytest.raises(sfo.SfoError) as ei:
            g.set_field(np.zeros_like(wl.ebar))
        assert ei.value.status == sfo.SFO_E_NOMEM
        os.environ.pop("SFO_FAIL_ALLOC")
        dE, dV = g.adjoint(psi, gv, 0, wl.nsteps)
        torch.cuda.synchronize()
        psiT = orc.schrodinger(wl.psi0, wl.n, wl.xmin, wl.xmax, wl.dt, wl.V0, wl.ebar, nsteps=wl.nsteps)
        rgT = 2 * (wl.dv * np.vdot(target, psiT)) * target * wl.dv
        _, rdE, _ = orc.schrodinger_adjoint(wl.psi0, rgT, wl.n, wl.xmin, wl.xmax, wl.dt, wl.V0, wl.ebar,
                                            nsteps=wl.nsteps)
        assert np.linalg.norm(rdE) > 1e-6
        assert np.linalg.norm(dE.cpu().numpy() - rdE) <= 1e-10 * np.linalg.norm(rdE)
        g.close()
        del psi, gv, dE, dV
        torch.cuda.empty_cache()
    finally:
        os.environ.pop("SFO_FAIL_ALLOC", None)
    # nothing the failed calls allocated is still held
    assert _free_bytes() >= free0 - (4 << 20)
