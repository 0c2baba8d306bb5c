"""Pins of the oracle's 1-D two-component Dirac step (alpha_1 = sigma_x,
beta = sigma_z): dense matrix exponentials of the discrete Hamiltonian
H = c alpha_1 (p - q A) + m c^2 beta + V on a small line (scipy's expm, not
the oracle's arithmetic), for the free case (the split is exact there) and
for the local error of one step with a potential and a constant vector
potential (third order in tau), and unitarity."""
import numpy as np
import scipy.linalg as sla

import oracle as orc

N, L, C, M, Q = 32, 4.0, 10.0, 1.0, -1.0


def _hamiltonian(V, A=0.0):
    dx = 2 * L / N
    k = 2 * np.pi * np.fft.fftfreq(N, dx)
    F = np.fft.fft(np.eye(N), axis=0)
    P = np.linalg.inv(F) @ np.diag(k) @ F  # hbar = 1
    P = (P + P.conj().T) / 2
    sx = np.array([[0, 1], [1, 0]])
    sz = np.array([[1, 0], [0, -1]])
    return C * np.kron(sx, P - Q * A * np.eye(N)) + M * C * C * np.kron(sz, np.eye(N)) + np.kron(np.eye(2), np.diag(V))


def _state():
    x = -L + 2 * L / N * np.arange(N)
    rng = np.random.default_rng(7)
    psi = np.stack([np.exp(-x ** 2) * (1 + 0.3j * x), 0.2 * np.exp(-(x - 0.5) ** 2)]).astype(complex)
    psi += 0.01 * (rng.standard_normal((2, N)) + 1j * rng.standard_normal((2, N)))
    return x, psi


def test_free_steps_equal_the_exponential():
    x, psi0 = _state()
    dt, S = 0.002, 25
    out = orc.dirac1d(psi0, N, -L, L, dt, np.zeros(N), None, nsteps=S, mass=M, charge=Q, c=C)
    ref = sla.expm(-1j * S * dt * _hamiltonian(np.zeros(N))) @ psi0.reshape(-1)
    assert np.linalg.norm(out.reshape(-1) - ref) / np.linalg.norm(ref) < 1e-11


def test_local_error_third_order_with_potential_and_vector_potential():
    x, psi0 = _state()
    V = -2.0 / np.sqrt(x ** 2 + 0.5)
    A = 0.7
    errs = []
    for dt in (0.004, 0.002):
        abar = np.full((1, N), A * dt)
        out = orc.dirac1d(psi0, N, -L, L, dt, V, abar, nsteps=1, mass=M, charge=Q, c=C)
        ref = sla.expm(-1j * dt * _hamiltonian(V, A)) @ psi0.reshape(-1)
        errs.append(np.linalg.norm(out.reshape(-1) - ref) / np.linalg.norm(ref))
    assert 7.0 < errs[0] / errs[1] < 9.0, errs


def test_norm_is_conserved():
    x, psi0 = _state()
    V = -2.0 / np.sqrt(x ** 2 + 0.5)
    abar = 0.01 * np.sin(np.arange(200)[:, None] * 0.1 + x[None, :])
    out = orc.dirac1d(psi0, N, -L, L, 0.003, V, abar, nsteps=200, mass=M, charge=Q, c=C)
    n0, n1 = np.sum(np.abs(psi0) ** 2), np.sum(np.abs(out) ** 2)
    assert abs(n1 / n0 - 1) < 1e-13


def _positive_energy_packet(N, L, p0, sigma, c, m=1.0):
    """A free packet of positive-energy states only: in momentum space each
    component of g(p) (Gaussian around p0) along the eigenvector of
    H(p) = c p sigma_x + m c^2 sigma_z with eigenvalue +E(p)."""
    x = -L + 2 * L / N * np.arange(N)
    k = 2 * np.pi * np.fft.fftfreq(N, 2 * L / N)
    E = np.sqrt(m ** 2 * c ** 4 + c ** 2 * k ** 2)
    g = np.exp(-((k - p0) ** 2) / (4 * sigma ** 2)) * np.exp(-1j * k * x[0])
    v0, v1 = E + m * c * c, c * k  # unnormalised eigenvector of +E
    nrm = np.sqrt(v0 ** 2 + v1 ** 2)
    psi = np.stack([np.fft.ifft(g * v0 / nrm), np.fft.ifft(g * v1 / nrm)])
    return x, k, E, psi


def test_free_positive_energy_packet_moves_with_its_group_velocity():
    """A free positive-energy packet has d<x>/dt = <c^2 p / E> exactly (no
    Zitterbewegung without negative-energy components): the centre of mass
    after S steps is <x>_0 + S tau <c^2 p/E>, the mean taken over |psi~(p)|^2."""
    Nn, Ln, c = 1024, 40.0, 5.0
    x, k, E, psi0 = _positive_energy_packet(Nn, Ln, 2.0, 0.6, c)
    dt, S = 0.01, 400
    out = orc.dirac1d(psi0, Nn, -Ln, Ln, dt, np.zeros(Nn), None, nsteps=S, c=c)
    rho0, rho1 = np.sum(np.abs(psi0) ** 2, axis=0), np.sum(np.abs(out) ** 2, axis=0)
    xm0, xm1 = np.sum(x * rho0) / np.sum(rho0), np.sum(x * rho1) / np.sum(rho1)
    w = np.sum(np.abs(np.fft.fft(psi0, axis=1)) ** 2, axis=0)
    vg = np.sum(w * c * c * k / E) / np.sum(w)
    assert abs((xm1 - xm0) - S * dt * vg) < 1e-9
    assert abs(xm1 - xm0) > 5.0  # it did move
