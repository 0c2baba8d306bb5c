#!/usr/bin/env python3
"""Benchmark: split-step grid-point updates/s of the Fourier split-operator hot path.

Workload: 2-D Schroedinger, 2048 x 2048 periodic grid on [-100, 100)^2 a.u.,
soft-core Coulomb V0 = -1/sqrt(r^2+1) plus the dipole term x.E(t) of a
sin^2-envelope pulse (E0 = 0.05, omega = 0.057), Gaussian initial state,
tau = 0.02, 500 steps per run (the field table repeats every 500 steps).
Seeded synthetic inputs (no dataset), state resident in HBM.

A "step" is one Strang step of the whole grid: the row pass (inverse
x-transform, merged potential factor, forward x-transform) and the column
pass (forward y-transform, kinetic factor, inverse y-transform).  `value` is
the complex128 path, the paper's precision (FP64 storage, butterflies,
phases and reductions); the complex64 path (FP32 storage and butterflies,
FP64 phases and reductions) and the paper's unfused five-launch complex128
step are reported beside it under `paths`, each fused path with its own
roofline block, and so are the forward run plus reverse sweep (adjoint) of
the same workload and the 64-problem batched control workload (forward,
and forward + reverse sweep).

Roofline: the dominant pass's algorithmic bytes per launch divided by its
average launch duration within steps of the propagation's pass sequence,
each launch timestamped by its own dispatch (start/stop events of the
launch, on the grid's stream); back-to-back launches of one pass, which read
their own output partly from cache, are reported beside it.  `traffic` is
the HBM bytes per launch measured with rocprofv3 counters for the same
kernel sources (null otherwise).

Prints ONE JSON line.  --gpus N with N > 1 is refused: the library runs on
one GPU.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X published HBM3E bandwidth

# HBM bytes per launch of the 2048 x 2048 passes, from two rocprofv3 --pmc
# runs (FETCH_SIZE, WRITE_SIZE) scaled by what the same counters read for a
# plain 512 MiB device copy (FETCH_SIZE x 2, WRITE_SIZE x 1); keyed by
# precision, then pass and tile-shape number.  Valid only for the kernel
# sources they were taken on: a different fingerprint reports null.
# the kernels' code and their tile-shape table (the dispatch files only choose among them)
TRAFFIC_SOURCES = ["fft_engine.h", "pass_kernels.h"]
TRAFFIC_TABLE = ("sfo_impl.h", b"struct RowVariant {", b"constexpr int kNumColVariants")
_KIB = 1024
MEASURED_TRAFFIC = {
    "sources_sha256": "1284db5b488a12aa1ab452bbee0d52b4194078c930b7c3b07c609f47e6fb5bd4",
    # pass/shape: (FETCH_SIZE KiB, WRITE_SIZE KiB) per dispatch as read; the pipelined
    # column shapes that differ only in groups per work-group share one kernel and one entry;
    # shapes whose kernel spills registers (never tuned in) have none
    "c64": {
        "row/0": (24726, 32768), "row/1": (24724, 32768), "row/2": (24718, 32768), "row/3": (24726, 32768),
        "row/4": (24722, 32768), "row/5": (24698, 32768), "row/6": (24698, 32768), "row/7": (24702, 32768),
        "row/8": (24691, 32768), "row/9": (24688, 32768), "row/10": (24720, 32768), "row/11": (24723, 32768),
        "row/12": (24720, 32768), "row/13": (24702, 32768), "row/14": (24726, 32768), "row/15": (24723, 32768),
        "row/16": (24720, 32768), "row/17": (24702, 32768), "row/18": (24735, 32768), "row/19": (24746, 32768),
        "column/0": (16657, 32798), "column/1": (16658, 32776), "column/2": (16658, 33258),
        "column/4": (16658, 32776), "column/5": (16660, 33191), "column/7": (16768, 32810),
        "column/8": (16626, 36052), "column/9": (16808, 32769), "column/10": (16816, 32768),
        "column/11": (16808, 32769), "column/12": (16816, 32768), "column/13": (16840, 32768),
        "column/14": (16856, 32768), "column/15": (16840, 32768), "column/16": (16856, 32768),
        "column/17": (16660, 33378), "column/18": (16654, 33006), "column/19": (16657, 33040),
        "column/20": (16655, 33428), "column/21": (16659, 33596), "column/22": (16866, 32769),
    },
    "c128": {
        "row/0": (49616, 65536), "row/1": (49432, 65536), "row/2": (49558, 65536), "row/3": (49598, 65536),
        "row/4": (49613, 65536), "row/5": (49384, 65536), "row/6": (49464, 65536), "row/7": (49388, 65536),
        "row/8": (49376, 65536), "row/9": (49449, 65536), "row/10": (49627, 65536), "row/11": (49435, 65536),
        "row/12": (49585, 65536), "row/13": (49394, 65536), "row/14": (49328, 65536), "row/15": (49322, 65536),
        "row/16": (49332, 65536), "row/17": (49288, 65536), "row/18": (49340, 65536), "row/19": (49342, 65536),
        "column/1": (33466, 76738), "column/2": (34058, 91756), "column/4": (33462, 77112),
        "column/5": (33910, 89643), "column/7": (33373, 65765), "column/8": (33382, 87118),
        "column/10": (33367, 69558), "column/12": (33367, 69558), "column/14": (33433, 65779),
        "column/16": (33433, 65779), "column/18": (33185, 65709), "column/19": (33185, 66244),
        "column/20": (33300, 79756), "column/21": (35456, 83055), "column/22": (33282, 69437),
    },
}
FETCH_SCALE, WRITE_SCALE = 2.0, 1.0  # plain-copy calibration of the two counters


def measured_traffic(dtype, kind, variant):
    v = MEASURED_TRAFFIC.get(dtype, {}).get("%s/%d" % (kind, variant))
    if v is None:
        return None
    return (FETCH_SCALE * v[0] + WRITE_SCALE * v[1]) * _KIB


def sources_fingerprint():
    import hashlib

    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_1012_3911_amd", "csrc")
    for f in TRAFFIC_SOURCES:
        with open(os.path.join(csrc, f), "rb") as fh:
            h.update(fh.read())
    f, first, last = TRAFFIC_TABLE
    with open(os.path.join(csrc, f), "rb") as fh:
        t = fh.read()
    h.update(t[t.index(first):t.index(last)])
    return h.hexdigest()


def parse():
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=1000)
    p.add_argument("--warmup", type=int, default=100)
    p.add_argument("--n", type=int, default=2048, help="grid points per axis")
    p.add_argument("--cpu-seconds", type=float, default=12.0, help="time budget of the oracle sample")
    p.add_argument("--no-cpu", action="store_true")
    p.add_argument("--only", choices=["c64", "c128", "all"], default="all")
    p.add_argument("--no-batch", action="store_true", help="skip the 64-problem batched control line")
    p.add_argument("--copy-calibration", action="store_true",
                   help="only run a plain 512 MiB device copy (the reference kernel for HBM counters)")
    p.add_argument("--other-workloads", action="store_true",
                   help="only run the other workloads (1-D harmonic, 1-D Dirac, 3-D wells, 2-D Dirac)")
    p.add_argument("--library-fft", action="store_true",
                   help="only time the torch.fft (hipFFT/rocFFT) split step of the workload (a comparison point)")
    p.add_argument("--batch-only", action="store_true",
                   help="only run the 64-problem batched control line (forward, forward + reverse sweep)")
    return p.parse_args()


def run_steps(g, psi, steps, period):
    """Propagate `steps` Strang steps, restarting the field table every `period` steps."""
    done = 0
    while done < steps:
        k = min(period, steps - done)
        g.propagate(psi, 0, k)
        done += k


def bench_path(wl, dtype, flags, steps, warmup):
    import torch
    from paper_1012_3911_amd import sfo

    g = sfo.Grid(wl.n, wl.xmin, wl.xmax, wl.dt, dtype=dtype, flags=flags)
    g.set_potential(wl.V0)
    g.set_field(wl.ebar)
    plan = g.autotune(20)
    psi = torch.from_numpy(wl.psi0).to("cuda").to(g.torch_dtype).contiguous()
    n0 = g.norm(psi)
    run_steps(g, psi, warmup, wl.nsteps)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    run_steps(g, psi, steps, wl.nsteps)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    # one more full run from psi0 for the accuracy figures (untimed)
    psi.copy_(torch.from_numpy(wl.psi0).to("cuda").to(g.torch_dtype))
    g.propagate(psi, 0, wl.nsteps)
    drift = g.norm(psi) / n0 - 1
    final = psi.cpu().numpy()
    # per-kernel durations: within steps of the pass sequence, each launch
    # timestamped by its own dispatch (the figure the roofline uses); back to
    # back launches of one pass (which finds its own output partly in cache);
    # and the timed sequence again with an event pair around every launch
    # (which adds the dispatch gap to each)
    # (fused paths only: the unfused step launches other kernels)
    kern = kern_b2b = kern_ev = None
    if not flags:
        kinds = (("row", sfo.KERNEL_ROW), ("column", sfo.KERNEL_COLUMN))
        kern = {name: g.time_pass(kind, 200, in_step=True) for name, kind in kinds}
        kern_b2b = {name: g.time_pass(kind, 200) for name, kind in kinds}
        g.profile(True)
        run_steps(g, psi, min(steps, 2 * wl.nsteps), wl.nsteps)
        kern_ev = {name: g.profile_read(kind) for name, kind in kinds}
        g.profile(False)
    fa = None
    if not flags:
        # forward run + reverse sweep (state, adjoint and both gradients) of the same workload
        gT = (0.5 * psi).contiguous()
        g.propagate(psi, 0, wl.nsteps)
        g.adjoint(psi, gT, 0, wl.nsteps)
        reps = 2
        torch.cuda.synchronize()
        ta = time.perf_counter()
        for _ in range(reps):
            g.propagate(psi, 0, wl.nsteps)
            g.adjoint(psi, gT, 0, wl.nsteps)
        torch.cuda.synchronize()
        fa = (time.perf_counter() - ta) / reps
    g.close()
    del psi
    torch.cuda.empty_cache()
    return dict(seconds=t1 - t0, drift=drift, final=final, kernels=kern, kernels_b2b=kern_b2b, kernels_ev=kern_ev,
                plan=plan, fwd_adj_seconds=fa)


def bench_batch(reps=3):
    """The 64-problem control batch (1-D 512..8192, 2-D 256^2..1024^2,
    complex64, 400 steps): one batched forward call, and forward + reverse
    sweep, timed over whole runs."""
    import torch
    from paper_1012_3911_amd import sfo, workloads as W

    wls, targets, _ = W.control_batch()
    S = wls[0].nsteps
    grids = []
    for wl in wls:
        g = sfo.Grid(wl.n, wl.xmin, wl.xmax, wl.dt, dtype="c64")
        g.set_potential(wl.V0)
        g.set_field(wl.ebar)
        g.autotune(10)  # tuned once per shape; later grids of that shape reuse the plan
        grids.append(g)
    psis = [torch.from_numpy(wl.psi0).to("cuda").to(torch.complex64).contiguous() for wl in wls]
    gs = [torch.from_numpy(t).to("cuda").to(torch.complex64).contiguous() for t in targets]
    b = sfo.Batch(grids)
    b.autotune(10)  # shapes of the grouped launches (one launch covers a group's problems)
    b.propagate(psis, 0, S)
    b.adjoint(psis, gs, 0, S)
    b.check()
    t0 = time.perf_counter()
    for _ in range(reps):
        b.propagate(psis, 0, S)
    b.check()
    t1 = time.perf_counter()
    for _ in range(reps):
        b.propagate(psis, 0, S)
        b.adjoint(psis, gs, 0, S)
    b.check()
    t2 = time.perf_counter()
    pts = sum(wl.npoints for wl in wls)
    b.close()
    for g in grids:
        g.close()
    return {"problems": len(wls), "steps": S, "points": pts,
            "fwd_ms_per_run": 1e3 * (t1 - t0) / reps, "fwd_updates_per_s": pts * S * reps / (t1 - t0),
            "fwd_adjoint_ms_per_run": 1e3 * (t2 - t1) / reps,
            "fwd_adjoint_updates_per_s": pts * S * reps / (t2 - t1)}


def bench_config(wl, dtype, runs=2):
    """Whole runs of one of the other workloads (1-D harmonic oscillator, 3-D
    wells, 2-D Dirac): ms per step, updates/s, and for the multi-pass grids
    the byte model per step (state read and written once per pass, plus one
    potential read) over the step time."""
    import torch
    from paper_1012_3911_amd import sfo

    g = sfo.Grid(wl.n, wl.xmin, wl.xmax, wl.dt, dtype=dtype, equation=wl.equation, mass=wl.mass,
                 charge=wl.charge, c=wl.c, hbar=wl.hbar)
    g.set_potential(wl.V0)
    if wl.equation == "dirac":
        g.set_vector_potential(wl.abar_y)
    else:
        g.set_field(wl.ebar)
    plan = list(g.autotune(5)) if wl.ndim >= 2 else None
    tdt = torch.complex64 if dtype == "c64" else torch.complex128
    psi = torch.from_numpy(wl.psi0).to("cuda").to(tdt).contiguous()
    g.propagate(psi, 0, min(wl.nsteps, 10))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(runs):
        g.propagate(psi, 0, wl.nsteps)
    torch.cuda.synchronize()
    t = (time.perf_counter() - t0) / (runs * wl.nsteps)
    g.close()
    del psi
    torch.cuda.empty_cache()
    npts = wl.npoints
    s = 8 if dtype == "c64" else 16
    v = 4 if dtype == "c64" else 8
    if wl.ndim == 1:
        step_bytes = None  # 1-D: the line stays on chip for the whole run
    elif wl.equation == "dirac":
        step_bytes = npts * (2 * 2 * 4 * s + v)  # row + column pass over 4 components, potential
    elif wl.ndim == 3:
        step_bytes = npts * (4 * 2 * s + v)  # x, y, z, y^-1 passes, potential
    else:
        step_bytes = npts * (2 * 2 * s + v)
    out = {"grid": list(wl.n), "dtype": dtype, "steps_per_run": wl.nsteps, "ms_per_step": 1e3 * t,
           "updates_per_s": npts / t, "plan": plan}
    if step_bytes:
        out["byte_model_gbs"] = step_bytes / t / 1e9
        out["byte_model_frac"] = step_bytes / t / 1e9 / HBM_PEAK_GBS
    return out


def bench_configs():
    import numpy as np
    from paper_1012_3911_amd import workloads as W

    def dirac_1d(N=4096, S=1000, dt=2e-4, L=10.0):
        # a bound packet in a soft-core well driven by a travelling A_1(x, t), complex128
        x = -L + 2 * L / N * np.arange(N)
        psi0 = np.stack([np.exp(-x ** 2 / 2 + 1.5j * x), 0.004 * (1.5 - 1j * x) * np.exp(-x ** 2 / 2)])
        t = dt * (np.arange(S) + 0.5)
        abar = dt * 30.0 * np.sin(0.8 * x[None, :] - 40.0 * t[:, None])
        return W.Workload("dirac1d", "dirac", (N,), (-L,), (L,), dt, S, -1.0 / np.sqrt(x ** 2 + 1.0),
                          psi0.astype(complex), abar_y=abar)

    res = {}
    for name, make, dtype, runs in (("1d_harmonic 1024 c128", lambda: W.harmonic_1d(), "c128", 5),
                                    ("1d_dirac 4096 c128", dirac_1d, "c128", 2),
                                    ("3d_wells 256^3 c64", lambda: W.wells_3d(), "c64", 2),
                                    ("2d_dirac_softcore_laser 1024^2 c128", lambda: W.dirac_softcore_laser(), "c128", 2)):
        res[name] = bench_config(make(), dtype, runs)
        print("# %s %.4f ms/step  %.3e updates/s" % (name, res[name]["ms_per_step"], res[name]["updates_per_s"]),
              file=sys.stderr, flush=True)
    return res


def bench_autocorrelation(runs=2):
    """The eigenstate method on the 2048^2 complex64 grid of the main
    workload with its field switched off: a 500-step autocorrelation run
    (the overlap with the entry state fused into the k-space pass) against a
    plain 500-step run, and the windowed spectrum at 2000 energies."""
    import torch
    from paper_1012_3911_amd import sfo, workloads as W

    wl = W.softcore_2d_laser()
    g = sfo.Grid(wl.n, wl.xmin, wl.xmax, wl.dt, dtype="c64")
    g.set_potential(wl.V0)
    g.set_field(None)
    g.autotune(5)
    psi = torch.from_numpy(wl.psi0).to("cuda").to(torch.complex64).contiguous()
    g.autocorrelation(psi, 10)
    g.propagate(psi, 0, 10)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(runs):
        chi = g.autocorrelation(psi, wl.nsteps)
    torch.cuda.synchronize()
    t_chi = (time.perf_counter() - t0) / (runs * wl.nsteps)
    t0 = time.perf_counter()
    for _ in range(runs):
        g.propagate(psi, 0, wl.nsteps)
    torch.cuda.synchronize()
    t_plain = (time.perf_counter() - t0) / (runs * wl.nsteps)
    E = torch.linspace(-1.0, 1.0, 2000, dtype=torch.float64, device="cuda")
    g.spectrum(chi, E)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    g.spectrum(chi, E)
    torch.cuda.synchronize()
    t_spec = time.perf_counter() - t0
    g.close()
    del psi
    torch.cuda.empty_cache()
    npts = wl.npoints
    step_bytes = npts * (2 * 2 * 8 + 4 + 8)  # two passes, potential, the reference read in the k-space pass
    return {"grid": list(wl.n), "dtype": "c64", "steps_per_run": wl.nsteps, "ms_per_step": 1e3 * t_chi,
            "updates_per_s": npts / t_chi, "ms_per_step_without_chi": 1e3 * t_plain,
            "byte_model_gbs": step_bytes / t_chi / 1e9, "byte_model_frac": step_bytes / t_chi / 1e9 / HBM_PEAK_GBS,
            "spectrum_ms_2000_energies": 1e3 * t_spec}


def bench_overall(steps=128, reps=3):
    """The paper's "overall" figure: the time to propagate `steps` steps
    including the copies of the state from host memory before the first step
    and back after the last, on the 2048^2 complex64 workload; pinned and
    pageable host buffers.  Context only: `value` has the state resident."""
    import numpy as np
    import torch
    from paper_1012_3911_amd import sfo, workloads as W

    wl = W.softcore_2d_laser()
    g = sfo.Grid(wl.n, wl.xmin, wl.xmax, wl.dt, dtype="c64")
    g.set_potential(wl.V0)
    g.set_field(wl.ebar)
    g.autotune(5)
    dev = torch.empty(wl.psi0.shape, dtype=torch.complex64, device="cuda")
    out = {"grid": list(wl.n), "dtype": "c64", "steps": steps}
    for kind in ("pinned", "pageable"):
        host = torch.from_numpy(wl.psi0.astype(np.complex64))
        if kind == "pinned":
            host = host.pin_memory()
        back = torch.empty_like(host, pin_memory=(kind == "pinned"))
        best = None
        for _ in range(reps + 1):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            dev.copy_(host, non_blocking=True)
            g.propagate(dev, 0, steps)
            back.copy_(dev, non_blocking=True)
            torch.cuda.synchronize()
            t = time.perf_counter() - t0
            best = t if best is None else min(best, t)
        out[kind] = {"ms": 1e3 * best, "updates_per_s": wl.npoints * steps / best}
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    g.propagate(dev, 0, steps)
    torch.cuda.synchronize()
    out["resident_ms"] = 1e3 * (time.perf_counter() - t0)
    g.close()
    del dev
    torch.cuda.empty_cache()
    return out


def bench_beyond_mall(steps=40):
    """2-D 4096 x 4096 complex128 (256 MiB of state, beyond the 256 MiB
    Infinity Cache once the potential is counted): the passes stream from HBM."""
    import torch
    from paper_1012_3911_amd import sfo, workloads as W

    wl = W.softcore_2d_laser(n=4096, nsteps=steps)
    g = sfo.Grid(wl.n, wl.xmin, wl.xmax, wl.dt, dtype="c128")
    g.set_potential(wl.V0)
    g.set_field(wl.ebar)
    plan = g.autotune(5)
    psi = torch.from_numpy(wl.psi0).to("cuda").to(torch.complex128).contiguous()
    g.propagate(psi, 0, 5)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    g.propagate(psi, 0, steps)
    torch.cuda.synchronize()
    t = (time.perf_counter() - t0) / steps
    kern = {name: g.time_pass(kind, 50, in_step=True)
            for name, kind in (("row", sfo.KERNEL_ROW), ("column", sfo.KERNEL_COLUMN))}
    g.close()
    del psi
    torch.cuda.empty_cache()
    npts = wl.n[0] * wl.n[1]
    alg = {"row": npts * (2 * 16 + 8), "column": npts * 2 * 16}
    return {"grid": list(wl.n), "dtype": "c128", "ms_per_step": 1e3 * t, "updates_per_s": npts / t, "plan": list(plan),
            "kernels": {k: {"avg_us": 1e3 * v, "gbs": alg[k] / (v * 1e-3) / 1e9,
                            "frac": alg[k] / (v * 1e-3) / 1e9 / HBM_PEAK_GBS} for k, v in kern.items()}}


def bench_library_fft(wl, steps=500, warmup=50, check_steps=20):
    """An external point of comparison, not the product path: the same
    Strang steps written with the vendor FFT library behind torch.fft
    (hipFFT/rocFFT) and torch elementwise products, adjacent potential halves
    merged, factors precomputed once.  Each step is a forward and an inverse
    2-D transform, the kinetic product and the merged potential product.
    After `check_steps` steps from psi0 its complex128 result is compared with
    the sfo complex128 path, to show that both compute the same steps."""
    import numpy as np
    import torch
    from paper_1012_3911_amd import sfo

    Ny, Nx = wl.n
    dx = [(wl.xmax[a] - wl.xmin[a]) / wl.n[a] for a in range(2)]
    x = wl.xmin[0] + dx[0] * np.arange(Nx)
    kx = 2 * np.pi * np.fft.fftfreq(Nx, d=dx[0])
    ky = 2 * np.pi * np.fft.fftfreq(Ny, d=dx[1])
    half_v = np.exp(-0.5j * wl.dt * wl.V0)
    kin = np.exp(-0.5j * wl.dt * (ky[:, None] ** 2 + kx[None, :] ** 2))
    half_x = np.exp(-0.5j * np.outer(wl.ebar[:, 0], x))  # (nsteps, Nx)
    nxt = np.roll(np.arange(wl.nsteps), -1)
    out = {"what": "torch.fft (hipFFT/rocFFT) split step, merged halves", "grid": [Ny, Nx]}
    for dtype, tdt in (("c64", torch.complex64), ("c128", torch.complex128)):
        dev = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to("cuda").to(tdt)
        V1, V2, K = dev(half_v), dev(half_v * half_v), dev(kin)
        X1, X2 = dev(half_x), dev(half_x * half_x[nxt])
        psi = dev(wl.psi0)
        buf = torch.empty_like(psi)

        def run(psi, n0, count):
            # opening half of step n0, then per step: transforms, kinetic factor,
            # closing half merged with the next step's opening half
            psi.mul_(V1).mul_(X1[n0 % wl.nsteps])
            for j in range(count):
                n = (n0 + j) % wl.nsteps
                torch.fft.fft2(psi, out=buf)
                buf.mul_(K)
                torch.fft.ifft2(buf, out=psi)
                if j + 1 < count:
                    psi.mul_(V2).mul_(X2[n])
                else:
                    psi.mul_(V1).mul_(X1[n])
            return psi

        run(psi, 0, warmup)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        run(psi, 0, steps)
        torch.cuda.synchronize()
        t = (time.perf_counter() - t0) / steps
        out[dtype] = {"ms_per_step": 1e3 * t, "updates_per_s": Ny * Nx / t}
        if dtype == "c128":
            psi.copy_(dev(wl.psi0))
            run(psi, 0, check_steps)
            g = sfo.Grid(wl.n, wl.xmin, wl.xmax, wl.dt, dtype="c128")
            g.set_potential(wl.V0)
            g.set_field(wl.ebar)
            ours = dev(wl.psi0)
            g.propagate(ours, 0, check_steps)
            torch.cuda.synchronize()
            out["c128_rel_l2_vs_sfo_after_%d_steps" % check_steps] = float(
                torch.linalg.vector_norm(psi - ours) / torch.linalg.vector_norm(ours))
            g.close()
            del ours
        del V1, V2, K, X1, X2, psi, buf
        torch.cuda.empty_cache()
    return out


def copy_calibration():
    """A plain device copy of known size: the HBM counters of this kernel
    calibrate FETCH_SIZE / WRITE_SIZE of the split-step kernels."""
    import torch

    nbytes = 512 << 20
    src = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(5):
        dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes_read": nbytes, "copy_bytes_written": nbytes, "launches": 5}))


def cpu_baseline(wl, budget, threads=None):
    """The FP64 oracle as it stands, on the host cores, over a bounded number of steps."""
    import numpy as np

    import oracle

    oracle.build(force=False)
    all_cores = oracle.num_threads()
    if threads:
        oracle.set_num_threads(threads)
    cores = oracle.num_threads()
    psi = wl.psi0.copy()
    steps = 0
    t0 = time.perf_counter()
    while True:
        psi = oracle.schrodinger(psi, wl.n, wl.xmin, wl.xmax, wl.dt, wl.V0, wl.ebar, step0=steps, nsteps=1)
        steps += 1
        el = time.perf_counter() - t0
        if el >= budget or steps >= wl.nsteps:
            break
    pts = int(np.prod(wl.n))
    if threads:
        oracle.set_num_threads(all_cores)
    return dict(value=pts * steps / el, unit="grid-point updates/s", cores=cores, kind="oracle",
                sample="%d of %d steps of the same %dx%d workload, FP64 radix-2, OpenMP over lines, %.1f s"
                       % (steps, wl.nsteps, wl.n[0], wl.n[1], el))


def main():
    args = parse()
    if args.gpus != 1:
        print("bench.py runs on one GPU only (got --gpus %d); the library has no multi-GPU sharding"
              % args.gpus, file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch

    from paper_1012_3911_amd import sfo, workloads as W

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    if args.copy_calibration:
        copy_calibration()
        return
    if args.other_workloads:
        print(json.dumps(bench_configs()))
        return
    if args.batch_only:
        print(json.dumps(bench_batch(reps=1)))
        return
    wl = W.softcore_2d_laser(n=args.n)
    if args.library_fft:
        print(json.dumps(bench_library_fft(wl, steps=args.steps, warmup=args.warmup)))
        return
    npts = wl.n[0] * wl.n[1]
    res = {}
    paths = [("c128", 0), ("c64", 0), ("c128_unfused", sfo.UNFUSED)]
    if args.only != "all":
        paths = [p for p in paths if p[0] == args.only]
    for name, flags in paths:
        dtype = name.split("_")[0]
        res[name] = bench_path(wl, dtype, flags, args.steps, args.warmup)
        print("# %-13s %.3f ms/step  %.3e updates/s  norm drift %.2e" % (
            name, 1e3 * res[name]["seconds"] / args.steps, npts * args.steps / res[name]["seconds"],
            res[name]["drift"]), file=sys.stderr, flush=True)

    def path_report(name, r):
        """ms/step, updates/s, plan and, for a fused path, per-pass timings and the
        roofline block of its dominant pass."""
        dt_ = name.split("_")[0]
        ms_ = 1e3 * r["seconds"] / args.steps
        rep = {"ms_per_step": ms_, "updates_per_s": npts * args.steps / r["seconds"], "plan": list(r["plan"])}
        if r["kernels"] is None:
            return rep
        bytes_state = npts * (8 if dt_ == "c64" else 16)
        bytes_v0 = npts * (4 if dt_ == "c64" else 8)
        # algorithmic bytes per launch: column pass reads and writes the state once;
        # row pass additionally reads V0
        alg = {"column": 2 * bytes_state, "row": 2 * bytes_state + bytes_v0}
        kstats = {}
        for k, avg in r["kernels"].items():
            cnt, tot = r["kernels_ev"][k]
            kstats[k] = dict(avg_us=1e3 * avg, gbs=alg[k] / (avg * 1e-3) / 1e9, launches_per_step=1,
                             timing="in-step, per-dispatch timestamps",
                             avg_us_back_to_back=1e3 * r["kernels_b2b"][k],
                             avg_us_event_per_launch=1e3 * tot / cnt if cnt else None)
        dom = max(kstats, key=lambda k: kstats[k]["avg_us"])
        achieved = kstats[dom]["gbs"]
        variant = {"row": rep["plan"][0], "column": rep["plan"][1]}[dom]
        traffic = None
        if wl.n == (2048, 2048) and sources_fingerprint() == MEASURED_TRAFFIC["sources_sha256"]:
            traffic = measured_traffic(dt_, dom, variant)
        rep["roofline"] = {
            "bound": "hbm",
            "kernel": ("k_colpass" if dom == "column" else "k_xpass") + " (tile shape %d)" % variant,
            "achieved": achieved,
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS,
            "traffic": traffic,
            "algorithmic_bytes": alg[dom],
        }
        step_bytes = alg["row"] + alg["column"]
        rep["step_model_gbs"] = step_bytes / (ms_ * 1e-3) / 1e9
        rep["step_model_frac"] = step_bytes / (ms_ * 1e-3) / 1e9 / HBM_PEAK_GBS
        rep["kernels"] = kstats
        if r.get("fwd_adj_seconds"):
            # each grid point is advanced once and walked back once per step
            rep["fwd_adjoint"] = {"updates_per_s": npts * wl.nsteps / r["fwd_adj_seconds"],
                                  "ms_per_step": 1e3 * r["fwd_adj_seconds"] / wl.nsteps,
                                  "note": "forward run + reverse sweep with dL/dEbar and dL/dV0, %s" % dt_}
        return rep

    reports = {k: path_report(k, v) for k, v in res.items()}
    # the headline is the paper's precision, complex128, when it was run
    head = "c128" if "c128" in res else list(res)[0]
    hdtype = head.split("_")[0]
    r, hr = res[head], reports[head]
    ms = hr["ms_per_step"]
    value = hr["updates_per_s"]
    err_vs_c128 = None
    if "c64" in res and "c128" in res:
        a, b = res["c64"]["final"].astype(np.complex128), res["c128"]["final"]
        err_vs_c128 = float(np.linalg.norm(a - b) / np.linalg.norm(b))
    out = {
        "metric": "split-step grid-point updates/s (fwd, fwd+adjoint) at stated err; % HBM BW",
        "value": value,
        "unit": "grid-point updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": hdtype,
        "data": "synthetic",
        "config": {
            "workload": "2d_schrodinger_softcore_laser %dx%d %s fwd%s" % (
                wl.n[0], wl.n[1], hdtype, " unfused" if head.endswith("unfused") else ""),
            "grid": list(wl.n), "box": [wl.xmin[0], wl.xmax[0]], "dt": wl.dt, "steps_per_run": wl.nsteps,
            "field": "x.E(t), E0=0.05, omega=0.057, sin^2 envelope over the run",
        },
        "roofline": hr.get("roofline"),
        "step_model_gbs": hr.get("step_model_gbs"),
        "step_model_frac": hr.get("step_model_frac"),
        "kernels": hr.get("kernels"),
        "accuracy": {"c64_norm_drift_per_run": res.get("c64", {}).get("drift"),
                     "c64_rel_l2_vs_c128_after_run": err_vs_c128,
                     "c128_norm_drift_per_run": res.get("c128", {}).get("drift")},
        "paths": {k: v for k, v in reports.items() if k != head},
    }
    if hr.get("fwd_adjoint"):
        out["fwd_adjoint"] = hr["fwd_adjoint"]
    if not args.no_batch:
        out["batch"] = bench_batch()
        print("# batch fwd %.2f ms/run, fwd+adjoint %.2f ms/run" % (out["batch"]["fwd_ms_per_run"],
              out["batch"]["fwd_adjoint_ms_per_run"]), file=sys.stderr, flush=True)
    if not args.no_batch:
        out["beyond_mall"] = bench_beyond_mall()
        print("# 4096^2 c128 %.3f ms/step" % out["beyond_mall"]["ms_per_step"], file=sys.stderr, flush=True)
        out["other_workloads"] = bench_configs()
        out["overall_with_transfers"] = bench_overall()
        print("# overall 128 steps incl. host copies: pinned %.2f ms, pageable %.2f ms, resident %.2f ms" % (
            out["overall_with_transfers"]["pinned"]["ms"], out["overall_with_transfers"]["pageable"]["ms"],
            out["overall_with_transfers"]["resident_ms"]), file=sys.stderr, flush=True)
        out["autocorrelation"] = bench_autocorrelation()
        print("# autocorrelation 2048^2 c64 %.4f ms/step (plain run %.4f)" % (
            out["autocorrelation"]["ms_per_step"], out["autocorrelation"]["ms_per_step_without_chi"]),
            file=sys.stderr, flush=True)
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(wl, args.cpu_seconds)
        one = cpu_baseline(wl, args.cpu_seconds, threads=1)
        out["cpu_baseline_one_core"] = {"value": one["value"], "cores": one["cores"], "sample": one["sample"]}
    print(json.dumps(out))


if __name__ == "__main__":
    main()
