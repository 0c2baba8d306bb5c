"""GPU parity of the Schroedinger split step against the FP64 oracle.

Every test calls the HIP library through its C ABI (paper_1012_3911_amd.sfo)
and compares with the oracle element by element on the same seeded inputs.
Tolerances: complex128 <= 1e-12 relative L2 (the accuracy target of the
complex128 path); complex64 <= 1e-5 relative L2 after the whole run with a
norm drift <= 1e-6 (the target stated for the FP32-storage path).
"""
import math

import numpy as np
import pytest

from paper_1012_3911_amd import workloads as W
from gpu_util import gpu_run, make_grid, oracle_run, rel_l2, to_device

pytestmark = pytest.mark.gpu

C128_TOL = 1e-12
C64_TOL = 1e-5
C64_DRIFT = 1e-6


def _rand_state(shape, seed):
    rng = np.random.default_rng(seed)
    return rng.standard_normal(shape) + 1j * rng.standard_normal(shape)


@pytest.mark.parametrize("dtype", ["c128", "c64"])
@pytest.mark.parametrize("shape", [(64,), (1024,), (4096,), (64, 128), (256, 64), (4096, 64), (64, 64, 128),
                                   (128, 64, 64)])
def test_fft_parity(orc, dtype, shape):
    import torch
    from paper_1012_3911_amd import sfo

    n = shape[::-1]
    g = sfo.Grid(n, [-1.0] * len(n), [1.0] * len(n), 0.01, dtype=dtype)
    a = _rand_state(shape, sum(shape))
    for sign in (-1, 1):
        t = to_device(a, dtype)
        g.fft(t, sign)
        torch.cuda.synchronize()
        ref = orc.fft(a.astype(np.complex64).astype(np.complex128) if dtype == "c64" else a, sign)
        err = rel_l2(t.cpu().numpy(), ref)
        tol = 2e-15 * math.log2(a.size) if dtype == "c128" else 2e-7 * math.log2(a.size)
        assert err < tol, (sign, err)
    g.close()


def test_1d_harmonic_full_c128(orc):
    """1-D N=1024 harmonic packet, tau = 0.01, 1000 steps in complex128."""
    wl = W.harmonic_1d()
    ref = oracle_run(orc, wl)
    got = gpu_run(wl, "c128")
    assert rel_l2(got, ref) < C128_TOL


def test_1d_harmonic_c64(orc):
    wl = W.harmonic_1d(nsteps=400)
    ref = oracle_run(orc, wl)
    got = gpu_run(wl, "c64")
    assert rel_l2(got, ref) < C64_TOL
    n0, n1 = orc.norm(wl.psi0, wl.n, wl.xmin, wl.xmax), orc.norm(got, wl.n, wl.xmin, wl.xmax)
    assert abs(n1 / n0 - 1) < C64_DRIFT


@pytest.mark.parametrize("n", [64, 512, 2048, 8192])
@pytest.mark.parametrize("dtype", ["c128", "c64"])
def test_1d_sizes_with_field(orc, n, dtype):
    wl = W.control_batch(count=2, nsteps=40, namp=20, sizes_1d=(9, 9))[0][0]
    # rebuild on a grid of n points with the same box and field
    L = 100.0
    (x,) = W.axes((n,), (-L,), (L,))
    wl.n, wl.V0 = (n,), -1.0 / np.sqrt(x**2 + 2.0)
    wl.psi0 = W.gaussian((n,), (-L,), (L,), (0.0,), 4.0, (0.3,))
    ref = oracle_run(orc, wl)
    got = gpu_run(wl, dtype)
    assert rel_l2(got, ref) < (C128_TOL if dtype == "c128" else C64_TOL)


@pytest.mark.parametrize("dtype", ["c128", "c64"])
@pytest.mark.parametrize("n", [(256, 256), (128, 64), (64, 512)])
def test_2d_softcore_laser(orc, dtype, n):
    wl = W.softcore_2d_laser(n=256, nsteps=200, L=25.6)
    if n != (256, 256):
        lo, hi = (-25.6, -12.8), (25.6, 12.8)
        X, Y = W.mesh(n, lo, hi)
        wl.n, wl.xmin, wl.xmax = n, lo, hi
        wl.V0 = -1.0 / np.sqrt(X**2 + Y**2 + 1.0)
        wl.psi0 = W.gaussian(n, lo, hi, (0.0, 0.0), 0.8, (0.5, -0.2))
        wl.ebar[:, 1] = 0.5 * wl.ebar[:, 0]
    ref = oracle_run(orc, wl)
    got = gpu_run(wl, dtype)
    err = rel_l2(got, ref)
    assert err < (C128_TOL if dtype == "c128" else C64_TOL), err
    if dtype == "c64":
        n0 = orc.norm(wl.psi0, wl.n, wl.xmin, wl.xmax)
        n1 = orc.norm(got, wl.n, wl.xmin, wl.xmax)
        assert abs(n1 / n0 - 1) < C64_DRIFT


@pytest.mark.parametrize("dtype", ["c128", "c64"])
def test_3d_wells(orc, dtype):
    wl = W.wells_3d(n=64, nsteps=30)
    # anisotropic variant of the same physics
    n, lo, hi = (64, 64, 128), (-20.0, -20.0, -40.0), (20.0, 20.0, 40.0)
    X, Y, Z = W.mesh(n, lo, hi)
    c, d, w = wl.meta["centres"], wl.meta["depths"], wl.meta["widths"]
    V0 = np.zeros(X.shape)
    for j in range(len(d)):
        V0 -= d[j] * np.exp(-((X - c[j, 0]) ** 2 + (Y - c[j, 1]) ** 2 + (Z - c[j, 2]) ** 2) / (2 * w[j] ** 2))
    wl.n, wl.xmin, wl.xmax, wl.V0 = n, lo, hi, V0
    wl.psi0 = W.gaussian(n, lo, hi, (1.0, -0.5, 0.0), 1.0, (0.2, 0.0, -0.3))
    wl.ebar = np.tile([[0.001, -0.0005, 0.0002]], (wl.nsteps, 1))
    ref = oracle_run(orc, wl)
    got = gpu_run(wl, dtype)
    assert rel_l2(got, ref) < (C128_TOL if dtype == "c128" else C64_TOL)


@pytest.mark.parametrize("dtype", ["c128", "c64"])
def test_every_tile_shape(orc, dtype):
    """Every row-pass and column-pass tile shape the planner may choose gives the oracle's
    result (anisotropic 256 x 512 grid, 20 steps); autotune picks one of them."""
    import torch
    from paper_1012_3911_amd import sfo

    n, lo, hi = (256, 512), (-25.6, -51.2), (25.6, 51.2)
    X, Y = W.mesh(n, lo, hi)
    wl = W.Workload("t", "schrodinger", n, lo, hi, 0.02, 20, -1.0 / np.sqrt(X**2 + Y**2 + 1.0),
                    W.gaussian(n, lo, hi, (0.5, -0.5), 0.9, (0.3, 0.1)),
                    ebar=np.tile([[0.002, -0.001]], (20, 1)))
    ref = oracle_run(orc, wl)
    tol = C128_TOL if dtype == "c128" else C64_TOL
    g = make_grid(wl, dtype)
    base = g.plan

    def sweep():
        # the reverse sweep with the forced shapes (a single-state column shape with
        # line pairs hands the two-state passes its plain equivalent)
        psi = to_device(ref, dtype)
        gv = to_device(wl.psi0, dtype)
        dE, dV = g.adjoint(psi, gv, 0, wl.nsteps)
        torch.cuda.synchronize()
        return dE.cpu().numpy(), dV.cpu().numpy()

    dE0, dV0 = sweep()
    tried = 0
    for kind in (0, 1):
        for v in range(32):
            p = list(base)
            p[kind] = v
            try:
                g.plan = p
            except sfo.SfoError:
                continue
            psi = to_device(wl.psi0, dtype)
            g.propagate(psi, 0, wl.nsteps)
            torch.cuda.synchronize()
            err = rel_l2(psi.cpu().numpy(), ref)
            assert err < tol, (kind, v, err)
            dE, dV = sweep()
            gtol = 1e-12 if dtype == "c128" else 1e-4
            assert np.linalg.norm(dE - dE0) <= gtol * np.linalg.norm(dE0), (kind, v)
            assert np.linalg.norm(dV - dV0) <= gtol * np.linalg.norm(dV0), (kind, v)
            tried += 1
    assert tried >= 16
    g.plan = base
    chosen = g.autotune(3)
    psi = to_device(wl.psi0, dtype)
    g.propagate(psi, 0, wl.nsteps)
    torch.cuda.synchronize()
    assert rel_l2(psi.cpu().numpy(), ref) < tol, chosen
    g.close()


@pytest.mark.parametrize("dtype", ["c128", "c64"])
def test_persistent_column_shapes(orc, dtype):
    """The column shapes whose work-groups walk several column groups (the next
    group's loads, or its copy into LDS, in flight while the current group
    transforms) on a grid wide enough that every work-group takes two or more
    groups (2048 columns): the oracle's result after 12 steps, and the plain
    shape's result (the same arithmetic) to rounding."""
    import torch
    from paper_1012_3911_amd import sfo

    n, lo, hi = (2048, 512), (-102.4, -25.6), (102.4, 25.6)
    X, Y = W.mesh(n, lo, hi)
    wl = W.Workload("t", "schrodinger", n, lo, hi, 0.02, 12, -1.0 / np.sqrt(X**2 + Y**2 + 1.0),
                    W.gaussian(n, lo, hi, (3.0, -0.5), 1.5, (0.4, 0.2)),
                    ebar=np.tile([[0.003, -0.002]], (12, 1)))
    ref = oracle_run(orc, wl)
    tol = C128_TOL if dtype == "c128" else C64_TOL
    g = make_grid(wl, dtype)
    base = list(g.plan)
    plain = None
    tried = []
    for v in range(48):
        try:
            g.plan = (base[0], v, 0)
        except sfo.SfoError:
            continue
        psi = to_device(wl.psi0, dtype)
        g.propagate(psi, 0, wl.nsteps)
        torch.cuda.synchronize()
        got = psi.cpu().numpy()
        err = rel_l2(got, ref)
        print("column shape %d: rel L2 vs oracle %.3e" % (v, err), flush=True)
        assert err < tol, (v, err)
        if v == 0:
            plain = got
        elif plain is not None and dtype == "c128":
            assert rel_l2(got, plain) < 1e-13, v
        tried.append(v)
    assert 0 in tried and len(tried) >= 12
    g.close()


@pytest.mark.parametrize("ndim", [1, 2, 3])
def test_step_equals_propagate(orc, ndim):
    if ndim == 1:
        wl = W.harmonic_1d(n=512, nsteps=12)
    elif ndim == 2:
        wl = W.softcore_2d_laser(n=128, nsteps=12, L=20.0)
    else:
        wl = W.wells_3d(n=64, nsteps=6)
    a = gpu_run(wl, "c128", step0=3, nsteps=wl.nsteps - 3)
    b = gpu_run(wl, "c128", step0=3, nsteps=wl.nsteps - 3, stepwise=True)
    assert rel_l2(a, b) < 1e-14
    ref = oracle_run(orc, wl, step0=3, nsteps=wl.nsteps - 3)
    assert rel_l2(a, ref) < C128_TOL


@pytest.mark.parametrize("ndim", [2, 3])
def test_unfused_equals_fused(ndim):
    from paper_1012_3911_amd import sfo

    wl = W.softcore_2d_laser(n=128, nsteps=10, L=20.0) if ndim == 2 else W.wells_3d(n=64, nsteps=5)
    a = gpu_run(wl, "c128")
    b = gpu_run(wl, "c128", flags=sfo.UNFUSED)
    assert rel_l2(a, b) < 1e-14


@pytest.mark.parametrize("dtype", ["c128", "c64"])
def test_norm_overlap(orc, dtype):
    n, lo, hi = (256, 128), (-3.0, -2.0), (5.0, 2.0)
    a = _rand_state((128, 256), 1)
    b = _rand_state((128, 256), 2)
    wl = W.Workload("r", "schrodinger", n, lo, hi, 0.01, 1, np.zeros((128, 256)), a)
    g = make_grid(wl, dtype)
    if dtype == "c64":
        a = a.astype(np.complex64).astype(np.complex128)
        b = b.astype(np.complex64).astype(np.complex128)
    ta, tb = to_device(a, dtype), to_device(b, dtype)
    assert abs(g.norm(ta) / orc.norm(a, n, lo, hi) - 1) < 1e-13
    ov = g.overlap(ta, tb)
    ref = orc.overlap(a, b, n, lo, hi)
    assert abs(ov - ref) < 1e-13 * abs(ref) + 1e-13 * math.sqrt(orc.norm(a, n, lo, hi) * orc.norm(b, n, lo, hi))
    g.close()


def test_resume_and_reversal_device(orc):
    """Markov in (psi, step): 30 = 17 + 13 steps; forward then backward by the adjoint's inverse
    step is covered in the adjoint tests."""
    wl = W.softcore_2d_laser(n=128, nsteps=30, L=20.0)
    a = gpu_run(wl, "c128")
    b = gpu_run(wl, "c128", nsteps=17)
    b = gpu_run(wl, "c128", step0=17, nsteps=13, psi0=b)
    assert rel_l2(a, b) < 1e-14


def test_time_pass_reports_the_current_shapes():
    """sfo_time_pass: positive durations for the row and column passes of a
    2-D grid, refused for a 1-D grid (which has no separate passes)."""
    from paper_1012_3911_amd import sfo

    n, lo, hi = (256, 128), (-10.0, -10.0), (10.0, 10.0)
    wl = W.Workload("t", "schrodinger", n, lo, hi, 0.02, 1, np.zeros(n[::-1]), np.ones(n[::-1], complex))
    g = make_grid(wl, "c64")
    for kind in (sfo.KERNEL_ROW, sfo.KERNEL_COLUMN):
        ms = g.time_pass(kind, 5)
        assert 0.0 < ms < 100.0
    with pytest.raises(sfo.SfoError):
        g.time_pass(sfo.KERNEL_ZCOLUMN, 5)
    g.close()
    w1 = W.Workload("l", "schrodinger", (256,), (-5.0,), (5.0,), 0.01, 1, np.zeros(256), np.ones(256, complex))
    g1 = make_grid(w1, "c64")
    with pytest.raises(sfo.SfoError):
        g1.time_pass(sfo.KERNEL_ROW, 5)
    g1.close()


@pytest.mark.parametrize("n", [(256, 128), (64, 64, 128)])
def test_time_pass_in_step(n):
    """sfo_time_pass with SFO_TIME_IN_STEP: per-dispatch durations of each pass
    within steps of the pass sequence (2-D and 3-D), positive, and together
    no longer than a whole step of the same sequence (which also holds the
    gaps between launches)."""
    import torch
    from paper_1012_3911_amd import sfo

    lo, hi = (-10.0,) * len(n), (10.0,) * len(n)
    shape = n[::-1]
    wl = W.Workload("t", "schrodinger", n, lo, hi, 0.02, 1, np.zeros(shape), np.ones(shape, complex))
    g = make_grid(wl, "c64")
    kinds = [sfo.KERNEL_ROW, sfo.KERNEL_COLUMN] + ([sfo.KERNEL_ZCOLUMN] if len(n) == 3 else [])
    per = {k: g.time_pass(k, 20, in_step=True) for k in kinds}
    assert all(0.0 < v < 100.0 for v in per.values()), per
    psi = torch.ones(shape, dtype=torch.complex64, device="cuda")
    g.propagate(psi, 0, 1)
    torch.cuda.synchronize()
    t0 = torch.cuda.Event(enable_timing=True)
    t1 = torch.cuda.Event(enable_timing=True)
    t0.record()
    for _ in range(20):
        g.propagate(psi, 0, 1)
    t1.record()
    torch.cuda.synchronize()
    step_ms = t0.elapsed_time(t1) / 20
    # a 3-D step runs the y-pass twice; the timed y-pass is the forward one
    passes = sum(per.values()) + (per[sfo.KERNEL_COLUMN] if len(n) == 3 else 0.0)
    assert passes < 1.5 * step_ms + 0.05, (per, step_ms)
    with pytest.raises(sfo.SfoError):
        g.time_pass(sfo.KERNEL_ROW, 5000, in_step=True)
    g.close()
