"""Batched runs (grouped launches under a HIP graph) against the oracle.

Every problem of a batch (uneven 1-D and 2-D sizes, each with its own box,
time step, potential and field table) must match the FP64 oracle run of that
problem alone, forward and in the reverse sweep, to the single-grid
tolerances: complex128 1e-12 relative L2 (forward) / 1e-11 (gradients),
complex64 1e-5 (forward) / 1e-4 (gradients).  HIP graph replays must
reproduce the directly launched result bit for bit.
"""
import numpy as np
import pytest

from paper_1012_3911_amd import workloads as W
from gpu_util import make_grid, oracle_run, rel_l2, to_device

pytestmark = pytest.mark.gpu

FWD_TOL = {"c128": 1e-12, "c64": 1e-5}
GRAD_TOL = {"c128": 1e-11, "c64": 1e-4}


def mixed_problems(seed=11, nsteps=40):
    """Uneven sizes, one problem per shape: 1-D 256 .. 8192 points, 2-D square
    and rectangular grids of 128 .. 1024 points per axis."""
    rng = np.random.default_rng(seed)
    shapes = [(256,), (8192,), (1024,), (128, 128), (256, 128), (128, 512), (1024, 128), (512, 256)]
    out = []
    for i, n in enumerate(shapes):
        nd = len(n)
        half = rng.uniform(8.0, 30.0, size=nd)
        lo, hi = tuple(-h for h in half), tuple(half)
        X = W.mesh(n, lo, hi) if nd > 1 else W.axes(n, lo, hi)
        r2 = sum(x**2 for x in X)
        V0 = -rng.uniform(0.5, 2.0) / np.sqrt(r2 + rng.uniform(0.5, 2.0))
        k0 = tuple(rng.uniform(-1.0, 1.0, size=nd))
        psi0 = W.gaussian(n, lo, hi, (0.0,) * nd, 1.0, k0)
        dt = float(rng.uniform(0.01, 0.05))
        ebar = dt * rng.uniform(-0.2, 0.2, size=(nsteps, nd))
        out.append(W.Workload("mix%d" % i, "schrodinger", n, lo, hi, dt, nsteps, V0, psi0, ebar=ebar))
    return out


def run_batch(wls, dtype, step0, nsteps, graph=True):
    import torch

    from paper_1012_3911_amd import sfo

    grids = [make_grid(wl, dtype) for wl in wls]
    psis = [to_device(wl.psi0, dtype) for wl in wls]
    b = sfo.Batch(grids, graph=graph)
    b.propagate(psis, step0, nsteps)
    b.check()
    torch.cuda.synchronize()
    out = [p.cpu().numpy().astype(np.complex128) for p in psis]
    b.close()
    for g in grids:
        g.close()
    return out


@pytest.mark.parametrize("dtype", ["c128", "c64"])
def test_batch_forward_matches_oracle(orc, dtype):
    wls = mixed_problems()
    step0, ns = 5, 30
    got = run_batch(wls, dtype, step0, ns)
    for wl, g in zip(wls, got):
        ref = oracle_run(orc, wl, nsteps=ns, step0=step0)
        err = rel_l2(g, ref)
        print("%-6s %-12s rel L2 %.2e" % (dtype, wl.n, err), flush=True)
        assert err < FWD_TOL[dtype], (wl.n, err)


@pytest.mark.parametrize("dtype", ["c128", "c64"])
def test_batch_autotune_matches_oracle(orc, dtype):
    """sfo_batch_autotune picks the grouped launches' shapes (forward runs and
    reverse sweep) on scratch states: the caller's states are untouched by the
    tuning, every problem still matches the oracle forward, and the tuned
    reverse sweep's gradients equal the untuned batch's to rounding."""
    import torch

    from paper_1012_3911_amd import sfo

    wls = mixed_problems()
    step0, ns = 5, 30
    grids = [make_grid(wl, dtype) for wl in wls]
    psis = [to_device(wl.psi0, dtype) for wl in wls]
    before = [p.clone() for p in psis]
    b = sfo.Batch(grids)
    b.autotune(2)
    torch.cuda.synchronize()
    for p, q in zip(psis, before):
        assert torch.equal(p, q)
    b.propagate(psis, step0, ns)
    b.check()
    torch.cuda.synchronize()
    for wl, p in zip(wls, psis):
        ref = oracle_run(orc, wl, nsteps=ns, step0=step0)
        err = rel_l2(p.cpu().numpy(), ref)
        print("tuned batch %-6s %-12s rel L2 %.2e" % (dtype, wl.n, err), flush=True)
        assert err < FWD_TOL[dtype], (wl.n, err)
    gs = [to_device(0.5 * wl.psi0, dtype) for wl in wls]
    d1, _ = b.adjoint([p.clone() for p in psis], [g_.clone() for g_ in gs], step0, ns, want_dV0=False)
    b.close()
    b2 = sfo.Batch(grids)
    d2, _ = b2.adjoint([p.clone() for p in psis], [g_.clone() for g_ in gs], step0, ns, want_dV0=False)
    b2.check()
    torch.cuda.synchronize()
    tol = 1e-12 if dtype == "c128" else 1e-5
    for x, y in zip(d1, d2):
        x, y = x.cpu().numpy(), y.cpu().numpy()
        assert np.linalg.norm(x - y) <= tol * np.linalg.norm(y)
    b2.close()
    for g in grids:
        g.close()


def test_batch_single_problem_and_zero_steps(orc):
    wls = mixed_problems()[3:4]
    got = run_batch(wls, "c128", 0, 0)
    assert np.array_equal(got[0], wls[0].psi0.astype(np.complex128))
    got = run_batch(wls, "c128", 0, 1)
    assert rel_l2(got[0], oracle_run(orc, wls[0], nsteps=1)) < 1e-13


def test_batch_graph_replays_match_direct_launch():
    """A captured graph, replayed several times with other work and
    synchronisations in between, gives the directly launched result exactly."""
    import torch

    from paper_1012_3911_amd import sfo

    wls = mixed_problems()
    direct = run_batch(wls, "c64", 0, 20, graph=False)
    grids = [make_grid(wl, "c64") for wl in wls]
    b = sfo.Batch(grids, graph=True)
    other = to_device(wls[3].psi0, "c64")
    for rep in range(3):
        psis = [to_device(wl.psi0, "c64") for wl in wls]
        b.propagate(psis, 0, 20)
        grids[3].propagate(other, 0, 7)  # eager work between replays
        b.check()
        torch.cuda.synchronize()
        for i, (p, d) in enumerate(zip(psis, direct)):
            assert np.array_equal(p.cpu().numpy().astype(np.complex128), d), (rep, i)
    b.close()
    for g in grids:
        g.close()


def adjoint_problems():
    wls = mixed_problems(seed=12, nsteps=24)
    targets = []
    for wl in wls:
        nd = wl.ndim
        targets.append(W.gaussian(wl.n, wl.xmin, wl.xmax, (0.7,) + (0.0,) * (nd - 1), 1.0, (0.0,) * nd))
    return wls, targets


@pytest.mark.parametrize("dtype", ["c128", "c64"])
def test_batch_adjoint_matches_oracle(orc, dtype):
    import torch

    from paper_1012_3911_amd import sfo

    wls, targets = adjoint_problems()
    ns = 24
    refs, psiTs, gTs = [], [], []
    for wl, tg in zip(wls, targets):
        psiT = orc.schrodinger(wl.psi0, wl.n, wl.xmin, wl.xmax, wl.dt, wl.V0, wl.ebar, nsteps=ns)
        ov = wl.dv * np.vdot(tg, psiT)
        gT = 2 * ov * tg * wl.dv
        refs.append(orc.schrodinger_adjoint(wl.psi0, gT, wl.n, wl.xmin, wl.xmax, wl.dt, wl.V0, wl.ebar,
                                            nsteps=ns))
        if dtype == "c64":
            psiT = psiT.astype(np.complex64).astype(np.complex128)
        psiTs.append(psiT)
        gTs.append(gT)
    grids = [make_grid(wl, dtype) for wl in wls]
    psis = [to_device(p, dtype) for p in psiTs]
    gs = [to_device(g, dtype) for g in gTs]
    b = sfo.Batch(grids)
    dEs, dVs = b.adjoint(psis, gs, 0, ns)
    b.check()
    torch.cuda.synchronize()
    tol = GRAD_TOL[dtype]
    for i, (wl, (g0, dE, dV)) in enumerate(zip(wls, refs)):
        p0 = psis[i].cpu().numpy().astype(np.complex128)
        gg = gs[i].cpu().numpy().astype(np.complex128)
        gdE, gdV = dEs[i].cpu().numpy(), dVs[i].cpu().numpy()
        errs = (rel_l2(p0, wl.psi0), rel_l2(gg, g0), np.linalg.norm(gdE - dE) / np.linalg.norm(dE),
                np.linalg.norm((gdV - dV).ravel()) / np.linalg.norm(dV.ravel()))
        print("%-6s %-12s psi0 %.1e g0 %.1e dE %.1e dV %.1e" % ((dtype, wl.n) + errs), flush=True)
        assert errs[0] < FWD_TOL[dtype], (wl.n, errs)
        assert max(errs[1:]) < tol, (wl.n, errs)
    b.close()
    for g in grids:
        g.close()


def test_batch_adjoint_equals_single_grid_adjoint():
    """The batched reverse sweep and the single-grid one agree (c128)."""
    import torch

    from paper_1012_3911_amd import sfo

    wls, targets = adjoint_problems()
    wls, targets = wls[:1] + wls[4:6], targets[:1] + targets[4:6]
    grids = [make_grid(wl, "c128") for wl in wls]
    rng = np.random.default_rng(3)
    states = [(rng.standard_normal(wl.psi0.shape) + 1j * rng.standard_normal(wl.psi0.shape)) * 1e-2 + wl.psi0
              for wl in wls]
    adjs = [t * 0.5 for t in targets]
    ps = [to_device(s, "c128") for s in states]
    gs = [to_device(a, "c128") for a in adjs]
    b = sfo.Batch(grids)
    dEs, dVs = b.adjoint(ps, gs, 2, 20)
    b.check()
    for i, g in enumerate(grids):
        p1, g1 = to_device(states[i], "c128"), to_device(adjs[i], "c128")
        dE1, dV1 = g.adjoint(p1, g1, 2, 20)
        torch.cuda.synchronize()
        assert rel_l2(ps[i].cpu().numpy(), p1.cpu().numpy()) < 1e-13
        assert rel_l2(gs[i].cpu().numpy(), g1.cpu().numpy()) < 1e-13
        assert np.linalg.norm((dEs[i] - dE1).cpu().numpy()) <= 1e-12 * np.linalg.norm(dE1.cpu().numpy())
        assert np.linalg.norm((dVs[i] - dV1).cpu().numpy()) <= 1e-12 * np.linalg.norm(dV1.cpu().numpy())
    b.close()
    for g in grids:
        g.close()


def test_batch_rejects_unsupported():
    from paper_1012_3911_amd import sfo

    ok = make_grid(mixed_problems()[3], "c64")
    cube = W.Workload("c", "schrodinger", (64, 64, 64), (-5.0,) * 3, (5.0,) * 3, 0.01, 1,
                      np.zeros((64, 64, 64)), np.ones((64, 64, 64), complex))
    dirac = W.Workload("d", "dirac", (64, 64), (-1.0, -1.0), (1.0, 1.0), 1e-5, 1,
                       np.zeros((64, 64)), np.ones((4, 64, 64), complex), abar_y=np.zeros((1, 64)))
    for wl, dtype, status in ((cube, "c64", sfo.SFO_E_UNSUPPORTED), (dirac, "c64", sfo.SFO_E_UNSUPPORTED),
                              (mixed_problems()[0], "c128", sfo.SFO_E_INVALID)):
        g = make_grid(wl, dtype)
        with pytest.raises(sfo.SfoError) as ei:
            sfo.Batch([ok, g])
        assert ei.value.status == status
        g.close()
    ok.close()


def test_batch_small_grids_and_repeated_shapes(orc):
    """Grids below the usual tile sizes (64-point lines, 64 x 64) and several
    problems of one shape in one group, against the oracle."""
    wls = []
    rng = np.random.default_rng(21)
    for n in ((64,), (64, 64), (64, 64), (128, 64), (64,)):
        nd = len(n)
        lo, hi = (-8.0,) * nd, (8.0,) * nd
        X = W.mesh(n, lo, hi) if nd > 1 else W.axes(n, lo, hi)
        V0 = -1.0 / np.sqrt(sum(x**2 for x in X) + rng.uniform(0.5, 2.0))
        psi0 = W.gaussian(n, lo, hi, (0.0,) * nd, 1.0, tuple(rng.uniform(-1, 1, size=nd)))
        ebar = 0.02 * rng.uniform(-0.2, 0.2, size=(12, nd))
        wls.append(W.Workload("s", "schrodinger", n, lo, hi, 0.02, 12, V0, psi0, ebar=ebar))
    got = run_batch(wls, "c128", 0, 12)
    for wl, g in zip(wls, got):
        assert rel_l2(g, oracle_run(orc, wl, nsteps=12)) < 1e-12


def test_control_batch_full_size(orc):
    """The 64-problem control batch (1-D 512..8192, 2-D 256^2..1024^2,
    complex64, 400 steps) in one batched call: norm conservation for every
    problem and oracle parity for the smallest and largest of each kind."""
    import torch

    from paper_1012_3911_amd import sfo

    wls, targets, ctl = W.control_batch()
    grids = [make_grid(wl, "c64") for wl in wls]
    psis = [to_device(wl.psi0, "c64") for wl in wls]
    n0 = [g.norm(p) for g, p in zip(grids, psis)]
    b = sfo.Batch(grids)
    b.autotune(3)  # the grouped launches' shapes, as the benchmark runs them
    b.propagate(psis, 0, wls[0].nsteps)
    b.check()
    torch.cuda.synchronize()
    for g, p, a in zip(grids, psis, n0):
        assert abs(g.norm(p) / a - 1) < 1e-5
    pick = set()
    for nd in (1, 2):
        idx = [i for i, wl in enumerate(wls) if wl.ndim == nd]
        pick.add(min(idx, key=lambda i: wls[i].npoints))
        pick.add(max(idx, key=lambda i: wls[i].npoints))
    for i in sorted(pick):
        ref = oracle_run(orc, wls[i])
        err = rel_l2(psis[i].cpu().numpy(), ref)
        print("control batch problem %d %s rel L2 %.2e" % (i, wls[i].n, err), flush=True)
        assert err < 1e-5
    b.close()
    for g in grids:
        g.close()


def _amp_grad(dE, dt, hold):
    """dL/d(amplitude k) from dL/dEbar: Ebar_s,x = dt * amp_k for the `hold` steps of piece k."""
    return dt * dE[:, 0].reshape(-1, hold).sum(axis=1)


def _overlap_grad(psiT, target, dv):
    ov = dv * np.vdot(target, psiT)
    return abs(ov) ** 2, 2 * ov * target * dv


def test_control_batch_full_size_gradient(orc):
    """Gradient of |<target|psi(T)>|^2 with respect to the 200 control amplitudes for
    every problem of the 64-problem control batch (complex64, 400 steps, one batched
    forward call and one batched reverse sweep, grids and grouped launches autotuned
    as the benchmark runs them).  Checked: the norm of every problem after the forward run (drift <= 1e-6);
    the largest 2-D problem against the complex128 single-grid adjoint and against
    central differences of the complex128 forward run at 4 amplitudes; one 8192-point
    line and one 256^2 problem against the oracle's stored-trajectory gradient
    (all <= 1e-4 relative)."""
    import torch

    from paper_1012_3911_amd import sfo

    wls, targets, ctl = W.control_batch()
    dt, hold, amps = ctl["dt"], ctl["hold"], ctl["control"]
    S = wls[0].nsteps
    grids = []
    for wl in wls:
        g = make_grid(wl, "c64")
        g.autotune(3)
        grids.append(g)
    psis = [to_device(wl.psi0, "c64") for wl in wls]
    n0 = [g.norm(p) for g, p in zip(grids, psis)]
    b = sfo.Batch(grids)
    b.autotune(3)
    b.propagate(psis, 0, S)
    b.check()
    drifts = [g.norm(p) / a - 1 for g, p, a in zip(grids, psis, n0)]
    worst = int(np.argmax(np.abs(drifts)))
    print("control batch: worst norm drift %.2e (problem %d, %s)" % (drifts[worst], worst, wls[worst].n),
          flush=True)
    gs = []
    for wl, t, p in zip(wls, targets, psis):
        _, gT = _overlap_grad(p.cpu().numpy().astype(np.complex128), t, wl.dv)
        gs.append(to_device(gT, "c64"))
    des, _ = b.adjoint(psis, gs, 0, S, want_dV0=False)
    b.check()
    torch.cuda.synchronize()
    grads = [_amp_grad(d.cpu().numpy(), dt, hold) for d in des]
    b.close()
    for g in grids:
        g.close()

    def rel(a, ref):
        return float(np.linalg.norm(a - ref) / np.linalg.norm(ref))

    # largest 2-D problem: complex128 single-grid adjoint and central differences
    i2 = max((i for i, wl in enumerate(wls) if wl.ndim == 2), key=lambda i: wls[i].npoints)
    wl = wls[i2]
    g = make_grid(wl, "c128")

    def forward(ebar):
        g.set_field(ebar)
        psi = to_device(wl.psi0, "c128")
        g.propagate(psi, 0, S)
        torch.cuda.synchronize()
        return psi

    psi = forward(wl.ebar)
    L0, gT = _overlap_grad(psi.cpu().numpy(), targets[i2], wl.dv)
    dE, _ = g.adjoint(psi, to_device(gT, "c128"), 0, S, want_dV0=False)
    ref128 = _amp_grad(dE.cpu().numpy(), dt, hold)
    e128 = rel(grads[i2], ref128)
    print("problem %d %s: batch c64 gradient vs single-grid c128 adjoint %.2e" % (i2, wl.n, e128), flush=True)
    assert e128 < 1e-4
    h = 1e-5
    scale = np.abs(ref128).max()
    for k in (0, 57, 123, 199):
        e_p, e_m = wl.ebar.copy(), wl.ebar.copy()
        e_p[k * hold:(k + 1) * hold, 0] += dt * h
        e_m[k * hold:(k + 1) * hold, 0] -= dt * h
        Lp = _overlap_grad(forward(e_p).cpu().numpy(), targets[i2], wl.dv)[0]
        Lm = _overlap_grad(forward(e_m).cpu().numpy(), targets[i2], wl.dv)[0]
        fd = (Lp - Lm) / (2 * h)
        print("  amplitude %d: FD %.6e  batch %.6e  c128 adjoint %.6e" % (k, fd, grads[i2][k], ref128[k]),
              flush=True)
        assert abs(fd - grads[i2][k]) <= 1e-4 * max(abs(fd), 1e-2 * scale), (k, fd, grads[i2][k])
        assert abs(fd - ref128[k]) <= 1e-6 * max(abs(fd), 1e-2 * scale), (k, fd, ref128[k])
    g.close()

    # an 8192-point line and a 256^2 grid against the oracle's stored-trajectory gradient
    picks = [next(i for i, w in enumerate(wls) if w.n == (8192,)), next(i for i, w in enumerate(wls) if w.n == (256, 256))]
    for i in picks:
        wl = wls[i]
        psiT = oracle_run(orc, wl)
        _, gT = _overlap_grad(psiT, targets[i], wl.dv)
        _, dE, _ = orc.schrodinger_adjoint(wl.psi0, gT, wl.n, wl.xmin, wl.xmax, wl.dt, wl.V0, wl.ebar, nsteps=S)
        e = rel(grads[i], _amp_grad(dE, dt, hold))
        print("problem %d %s: batch c64 gradient vs oracle %.2e" % (i, wl.n, e), flush=True)
        assert e < 1e-4
    assert max(abs(d) for d in drifts) < 1e-6, drifts[worst]


def test_batch_adjoint_after_plan_change():
    """The batch's captured reverse-sweep graph holds launches of the member grids'
    tile shapes (grid sizes and the partial-slot stride of the row pass).  Forcing
    other shapes on the grids between two reverse sweeps must give the same
    gradients (complex128, 1e-12), i.e. the batch re-captures instead of replaying."""
    import torch

    from paper_1012_3911_amd import sfo

    wls = mixed_problems(nsteps=12)
    grids = [make_grid(wl, "c128") for wl in wls]
    b = sfo.Batch(grids)

    def sweep():
        psis = [to_device(wl.psi0, "c128") for wl in wls]
        b.propagate(psis, 0, 12)
        gs = [(0.5 * p).contiguous() for p in psis]
        des, dvs = b.adjoint(psis, gs, 0, 12)
        b.check()
        torch.cuda.synchronize()
        return [d.cpu().numpy() for d in des], [d.cpu().numpy() for d in dvs]

    dE0, dV0 = sweep()
    alts = {}
    for i, (wl, g) in enumerate(zip(wls, grids)):
        if wl.ndim != 2:
            continue
        base = g.plan
        ok = []
        for v in range(16):
            if v == base[0]:
                continue
            try:
                g.plan = (v, base[1], base[2])
                ok.append(v)
            except sfo.SfoError:
                pass
        g.plan = base
        alts[i] = (base, ok)
    changed = 0
    for trial in range(3):
        for i, (base, ok) in alts.items():
            if ok:
                grids[i].plan = (ok[trial % len(ok)], base[1], base[2])
                changed += 1
        dE1, dV1 = sweep()
        for i in range(len(wls)):
            assert np.linalg.norm(dE1[i] - dE0[i]) <= 1e-12 * np.linalg.norm(dE0[i]), (trial, i)
            assert np.linalg.norm((dV1[i] - dV0[i]).ravel()) <= 1e-12 * np.linalg.norm(dV0[i].ravel()), (trial, i)
    assert changed > 0
    b.close()
    for g in grids:
        g.close()
