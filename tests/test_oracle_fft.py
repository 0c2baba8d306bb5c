"""Pins for the oracle's own FFT (the DFT that replaces the Fourier transform, Sec. 2.1).

The oracle's radix-2 transform is compared with the O(N^2) definition of the
DFT written out as a sum, with inverse-after-forward, with Parseval's identity
and with numpy.fft as a second, independent library."""
import numpy as np
import pytest


def brute_dft(a, sign):
    """out[m] = sum_j a[j] exp(sign 2 pi i j m / N) along every axis, by definition."""
    out = np.asarray(a, np.complex128)
    for ax in range(out.ndim):
        n = out.shape[ax]
        j = np.arange(n)
        W = np.exp(sign * 2j * np.pi * np.outer(j, j) / n)
        out = np.moveaxis(np.tensordot(W, np.moveaxis(out, ax, 0), axes=(1, 0)), 0, ax)
    return out


def rand_c(rng, shape):
    return rng.standard_normal(shape) + 1j * rng.standard_normal(shape)


@pytest.mark.parametrize("shape", [(1,), (2,), (4,), (8,), (64,), (16, 8), (4, 32), (8, 4, 2), (2, 8, 16)])
@pytest.mark.parametrize("sign", [-1, 1])
def test_fft_matches_definition(orc, shape, sign):
    rng = np.random.default_rng(sum(shape) + sign)
    a = rand_c(rng, shape)
    got = orc.fft(a, sign)
    ref = brute_dft(a, sign)
    assert np.max(np.abs(got - ref)) <= 1e-14 * max(1.0, np.max(np.abs(ref))) * np.prod(shape) ** 0.5


@pytest.mark.parametrize("shape", [(1024,), (64, 128), (16, 8, 32)])
def test_fft_inverse_parseval_numpy(orc, shape):
    rng = np.random.default_rng(7)
    a = rand_c(rng, shape)
    f = orc.fft(a, -1)
    back = orc.fft(f, +1) / a.size
    assert np.max(np.abs(back - a)) < 1e-14 * np.sqrt(np.log2(a.size) + 1) * 10
    # Parseval: sum |F|^2 = N sum |a|^2
    assert abs(np.sum(np.abs(f) ** 2) / (a.size * np.sum(np.abs(a) ** 2)) - 1) < 1e-14
    ref = np.fft.fftn(a)
    assert np.max(np.abs(f - ref)) / np.max(np.abs(ref)) < 1e-14


def test_fft_components_independent(orc):
    rng = np.random.default_rng(3)
    a = rand_c(rng, (4, 8, 16))
    got = orc.fft(a, -1, ncomp=4)
    for c in range(4):
        assert np.max(np.abs(got[c] - brute_dft(a[c], -1))) < 1e-12


def test_fft_single_mode(orc):
    """A pure mode exp(2 pi i m j / N) lands entirely on bin m with weight N."""
    n = 32
    j = np.arange(n)
    for m in (0, 1, 5, 16, 31):
        a = np.exp(2j * np.pi * m * j / n)
        f = orc.fft(a, -1)
        expect = np.zeros(n, complex)
        expect[m] = n
        assert np.max(np.abs(f - expect)) < 1e-12
