"""Pins of the oracle's autocorrelation spectrum (the paper's eigenstate
section: chi(t), its windowed transform chi~(E), the windowed eigenfunction).

Each pin is fixed by something other than the oracle: closed forms of the
window's transform, the exact quasi-energies of the Strang map of the
harmonic oscillator, a dense diagonalisation of the discrete Hamiltonian, and
the soft-core ground state energy the paper quotes."""
import numpy as np

import oracle as orc


def test_window_transform_closed_form():
    """For chi = exp(-i E0 t): chi~(E0) = T, chi~(E0 +- 2 pi/T) = -T/2 and
    chi~(E0 + 2 pi k/T) = 0 for |k| >= 2 (the discrete sums of the window are
    exact), which fixes the window and the sign of the exponent."""
    S, dt, E0 = 1000, 0.01, 3.7
    T = S * dt
    chi = np.exp(-1j * E0 * dt * np.arange(S))
    Es = E0 + 2 * np.pi / T * np.array([0, 1, -1, 2, -3, 7])
    sp = orc.spectrum(chi, dt, Es)
    want = np.array([T, -T / 2, -T / 2, 0, 0, 0])
    assert np.max(np.abs(sp - want)) < 1e-10 * T
    # the opposite sign of E would be far from T
    assert abs(orc.spectrum(chi, dt, [-E0])[0]) < 1e-3 * T


def test_harmonic_quasi_energies():
    """V = x^2/2: the Strang map rotates phase space by theta, cos theta =
    1 - tau^2/2, so its eigenstates have quasi-energies (2n+1) theta / (2 tau)
    (hbar = m = 1).  A displaced Gaussian shows peaks at n = 0..3."""
    N, L, dt, S = 128, 10.0, 0.05, 4000
    x = -L + 2 * L / N * np.arange(N)
    psi0 = np.exp(-(x - 1.5) ** 2 / 2).astype(complex)
    chi, _ = orc.autocorrelation(psi0, (N,), (-L,), (L,), dt, x ** 2 / 2, S)
    theta = np.arccos(1 - dt ** 2 / 2)
    for n in range(4):
        En = (2 * n + 1) * theta / (2 * dt)
        E = np.linspace(En - 0.15, En + 0.15, 301)
        peak = orc.peak_energy(E, orc.spectrum(chi, dt, E))
        assert abs(peak - En) < 2e-4, (n, peak, En)


def _softcore_1d(N=256, L=30.0, zeta=1.4133):
    x = -L + 2 * L / N * np.arange(N)
    V = -1.0 / np.sqrt(x ** 2 + zeta ** 2)
    dx = 2 * L / N
    k = 2 * np.pi * np.fft.fftfreq(N, dx)
    F = np.fft.fft(np.eye(N), axis=0)
    Tk = np.linalg.inv(F) @ np.diag(k ** 2 / 2) @ F
    H = (Tk + Tk.conj().T) / 2 + np.diag(V)
    w, vec = np.linalg.eigh(H)
    return x, V, dx, w, vec


def test_softcore_ground_state():
    """1-D soft-core potential, zeta = 1.4133, Z = 1: the lowest peak of the
    spectrum agrees with the lowest eigenvalue of the discrete Hamiltonian
    (dense diagonalisation) to the splitting error, and with the paper's
    statement that this zeta gives the 3-D Coulomb ground state energy -1/2."""
    N, L, dt, S = 256, 30.0, 0.05, 4000
    x, V, dx, w, _ = _softcore_1d(N, L)
    psi0 = np.exp(-x ** 2 / 2).astype(complex)
    chi, _ = orc.autocorrelation(psi0, (N,), (-L,), (L,), dt, V, S)
    E = np.linspace(-0.7, -0.3, 401)
    peak = orc.peak_energy(E, orc.spectrum(chi, dt, E))
    assert abs(peak - w[0]) < 1e-4
    assert abs(peak + 0.5) < 2e-3


def test_softcore_eigenfunction():
    """The windowed eigenfunction at the ground state energy is the ground
    eigenvector of the discrete Hamiltonian."""
    N, L, dt, S = 256, 30.0, 0.05, 4000
    x, V, dx, w, vec = _softcore_1d(N, L)
    psi0 = np.exp(-x ** 2 / 2).astype(complex)
    pe = orc.eigenfunction(psi0, (N,), (-L,), (L,), dt, V, S, w[0])
    g = vec[:, 0] / np.sqrt(dx)
    assert abs(np.sum(np.conj(g) * pe) * dx) > 0.999
