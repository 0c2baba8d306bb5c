"""Parity with the FP64 oracle over the full length of the 2-D, 3-D and Dirac
workloads, at their full sizes, in the launch configuration the benchmark
times (autotuned tile shapes).

The 4096^2 grid (the largest square grid, which the benchmark times beside
the 2-D workload) runs a 100-step pulse of the same workload.

Each workload is advanced in chunks; the oracle state, the complex128 GPU
state and the complex64 GPU state are carried from chunk to chunk (module
cache), so every checkpoint compares all three after the same number of
steps, element by element, and the last checkpoint is the whole run.  The
oracle runs on the host's cores (OpenMP); each chunk is sized to stay well
inside a couple of minutes.

Targets (the whole-run accuracy the path is built to): complex128 <= 1e-12
relative L2; complex64 <= 1e-5 relative L2; complex64 norm drift <= 1e-6;
complex128 norm drift <= 1e-12.

The reverse sweep at the sizes where the two-state pass kernels run with
2048- and 1024-point lines (500 steps, the length of the 2-D workload) is
compared with the oracle's gradient from a stored FP64 trajectory
(complex128 1e-11, complex64 1e-4 relative)."""
import numpy as np
import pytest

from paper_1012_3911_amd import workloads as W
from gpu_util import make_grid, oracle_run, rel_l2, to_device

pytestmark = pytest.mark.gpu

C128_TOL = 1e-12
C64_TOL = 1e-5
C64_DRIFT = 1e-6
C128_DRIFT = 1e-12


class FullRun:
    """One workload advanced on the oracle and on the GPU (c128 and c64)."""

    def __init__(self, orc, wl, dtypes=("c128", "c64"), autotune=True):
        self.orc, self.wl = orc, wl
        self.step = 0
        self.ref = np.array(wl.psi0, dtype=np.complex128)
        self.grids, self.psi, self.n0 = {}, {}, {}
        for d in dtypes:
            g = make_grid(wl, d)
            if autotune:
                g.autotune(3)
            p = to_device(wl.psi0, d)
            self.grids[d], self.psi[d], self.n0[d] = g, p, g.norm(p)

    def advance_to(self, step):
        import torch

        assert step >= self.step
        ns = step - self.step
        if ns:
            for d, g in self.grids.items():
                g.propagate(self.psi[d], self.step, ns)
            self.ref = oracle_run(self.orc, self.wl, step0=self.step, nsteps=ns, psi0=self.ref)
            torch.cuda.synchronize()
            self.step = step

    def check(self, tag):
        out = {}
        for d, g in self.grids.items():
            got = self.psi[d].cpu().numpy()
            err = rel_l2(got, self.ref)
            drift = g.norm(self.psi[d]) / self.n0[d] - 1
            out[d] = (err, drift)
            print("%s step %d %s: rel L2 vs oracle %.3e, norm drift %.2e" % (tag, self.step, d, err, drift),
                  flush=True)
        for d, (err, drift) in out.items():
            if d == "c128":
                assert err < C128_TOL, (d, self.step, err)
                assert abs(drift) < C128_DRIFT, (d, self.step, drift)
            else:
                assert err < C64_TOL, (d, self.step, err)
                assert abs(drift) < C64_DRIFT, (d, self.step, drift)

    def close(self):
        import torch

        for g in self.grids.values():
            g.close()
        self.grids, self.psi = {}, {}
        torch.cuda.empty_cache()


_RUNS = {}


def _run(orc, key, make):
    r = _RUNS.get(key)
    if r is None:
        for k in list(_RUNS):  # one full-size workload resident at a time
            _RUNS.pop(k).close()
        r = _RUNS[key] = FullRun(orc, make())
    return r


@pytest.fixture(scope="module", autouse=True)
def _release():
    yield
    for k in list(_RUNS):
        _RUNS.pop(k).close()


@pytest.mark.parametrize("step", [100, 200, 300, 400, 500])
def test_2d_softcore_laser_2048sq_500_steps(orc, step):
    """2048^2 soft-core atom with the dipole laser term, tau = 0.02, 500 steps."""
    r = _run(orc, "2d", W.softcore_2d_laser)
    r.advance_to(step)
    r.check("2d 2048^2")


@pytest.mark.parametrize("step", [50, 100])
def test_2d_softcore_laser_4096sq_100_steps(orc, step):
    """4096^2 soft-core atom with the dipole laser term (the largest square grid:
    256 MiB of complex128 state, the tile shapes that stream from HBM), tau = 0.02,
    a 100-step pulse."""
    r = _run(orc, "2d4096", lambda: W.softcore_2d_laser(n=4096, nsteps=100))
    r.advance_to(step)
    r.check("2d 4096^2")


@pytest.mark.parametrize("step", [50, 100, 150, 200])
def test_3d_wells_256cube_200_steps(orc, step):
    """256^3 sum of 8 random Gaussian wells, tau = 0.01, 200 steps."""
    r = _run(orc, "3d", W.wells_3d)
    r.advance_to(step)
    r.check("3d 256^3")


@pytest.mark.parametrize("step", [100, 200])
def test_dirac_1024sq_200_steps(orc, step):
    """2-D Dirac 4-spinor 1024^2, Z = 20 soft core, laser A_y(x, t), tau = 1e-5, 200 steps."""
    r = _run(orc, "dirac", W.dirac_softcore_laser)
    r.advance_to(step)
    r.check("dirac 1024^2")


# ------------------------------------------------ reverse sweep at full line lengths --

def _adjoint_problem(n, nsteps=500, dt=0.02):
    """A soft-core atom on an anisotropic box with a random dipole field; the loss is
    |<target|psi_T>|^2 with the target the initial packet moved along x."""
    dx = (0.05, 0.2) if n[0] > n[1] else (0.2, 0.05)
    lo = tuple(-0.5 * n[a] * dx[a] for a in range(2))
    hi = tuple(0.5 * n[a] * dx[a] for a in range(2))
    X, Y = W.mesh(n, lo, hi)
    V0 = -1.0 / np.sqrt(X**2 + Y**2 + 1.0)
    psi0 = W.gaussian(n, lo, hi, (0.0, 0.0), 1.0, (0.3, -0.2))
    target = W.gaussian(n, lo, hi, (0.5, 0.0), 1.0, (0.0, 0.0))
    rng = np.random.default_rng(sum(n))
    ebar = dt * rng.uniform(-0.1, 0.1, size=(nsteps, 2))
    return W.Workload("adj", "schrodinger", n, lo, hi, dt, nsteps, V0, psi0, ebar=ebar), target


@pytest.mark.parametrize("n", [(2048, 128), (128, 2048), (1024, 128), (128, 1024)])
def test_adjoint_500_steps_long_lines(orc, n):
    """sfo_adjoint over 500 steps on grids whose row or column lines hold 2048 or
    1024 points, after autotuning (as the benchmark runs the reverse sweep),
    against the oracle's stored-trajectory gradient."""
    import torch

    wl, target = _adjoint_problem(n)
    psiT = orc.schrodinger(wl.psi0, wl.n, wl.xmin, wl.xmax, wl.dt, wl.V0, wl.ebar, nsteps=wl.nsteps)
    ov = wl.dv * np.vdot(target, psiT)
    gT = 2 * ov * target * wl.dv
    g0, dE, dV = orc.schrodinger_adjoint(wl.psi0, gT, wl.n, wl.xmin, wl.xmax, wl.dt, wl.V0, wl.ebar,
                                         nsteps=wl.nsteps)
    for dtype, tol, ptol in (("c128", 1e-11, 1e-12), ("c64", 1e-4, 1e-5)):
        g = make_grid(wl, dtype)
        g.autotune(2)
        # the c64 sweep starts from its own forward result, as it would after a c64 forward run
        psi = to_device(wl.psi0, dtype)
        g.propagate(psi, 0, wl.nsteps)
        gv = to_device(gT, dtype)
        gdE, gdV = g.adjoint(psi, gv, 0, wl.nsteps)
        torch.cuda.synchronize()
        e_psi = rel_l2(psi.cpu().numpy(), wl.psi0)
        e_g = rel_l2(gv.cpu().numpy(), g0)
        e_dE = float(np.linalg.norm(gdE.cpu().numpy() - dE) / np.linalg.norm(dE))
        e_dV = float(np.linalg.norm((gdV.cpu().numpy() - dV).ravel()) / np.linalg.norm(dV.ravel()))
        print("adjoint %s %s 500 steps: psi0 %.2e g0 %.2e dL/dEbar %.2e dL/dV0 %.2e plan %s"
              % (n, dtype, e_psi, e_g, e_dE, e_dV, g.plan), flush=True)
        g.close()
        assert e_psi < ptol, (dtype, e_psi)
        assert e_g < tol, (dtype, e_g)
        assert e_dE < tol, (dtype, e_dE)
        assert e_dV < tol, (dtype, e_dV)
