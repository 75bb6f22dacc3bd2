"""Pins for the oracle's radix-2 FFT (the transforms of section 4).

Checked against things other than the oracle itself: a brute-force DFT
whose angles are reduced exactly as 2 pi ((k n) mod N) / N, Parseval's
identity, the closed-form spectrum of a pure tone, numpy.fft, and the
inverse-of-forward identity.
"""
import numpy as np
import pytest

from oracle import oracle as O


def brute_dft(x, sign=-1):
    n = len(x)
    k = np.arange(n)
    kn = np.outer(k, k) % n                      # exact integer angle reduction
    w = np.exp(sign * 2j * np.pi * kn / n)
    return w @ x


@pytest.mark.parametrize("n", [1, 2, 4, 8, 16, 32, 64, 128, 256])
def test_fft_matches_brute_force_dft(n):
    r = np.random.default_rng(n)
    x = r.standard_normal(n) + 1j * r.standard_normal(n)
    for sign in (-1, +1):
        got = O.fft(x, sign)
        ref = brute_dft(x, sign)
        assert np.max(np.abs(got - ref)) <= 1e-13 * max(1.0, np.max(np.abs(ref)))


@pytest.mark.parametrize("n", [16, 256, 2048, 4096])
def test_parseval(n):
    r = np.random.default_rng(100 + n)
    x = r.standard_normal(n) + 1j * r.standard_normal(n)
    X = O.fft(x)
    lhs = np.sum(np.abs(x) ** 2)
    rhs = np.sum(np.abs(X) ** 2) / n
    assert abs(lhs - rhs) <= 1e-13 * lhs


@pytest.mark.parametrize("n,k0,psi", [(2048, 411, 0.3), (4096, 1000, -1.2), (64, 5, 2.0)])
def test_pure_tone(n, k0, psi):
    t = np.arange(n)
    x = np.cos(2 * np.pi * k0 * t / n + psi)
    X = O.fft(x)
    expect = np.zeros(n, complex)
    expect[k0] = n / 2 * np.exp(1j * psi)
    expect[n - k0] = n / 2 * np.exp(-1j * psi)
    assert np.max(np.abs(X - expect)) <= 1e-12 * n


@pytest.mark.parametrize("n", [2048, 4096])
def test_fft_matches_numpy(n):
    r = np.random.default_rng(7 + n)
    x = r.standard_normal(n) + 1j * r.standard_normal(n)
    X = O.fft(x)
    ref = np.fft.fft(x)
    assert np.max(np.abs(X - ref)) <= 1e-13 * np.max(np.abs(ref))
    xi = O.fft(X, +1) / n
    assert np.max(np.abs(xi - x)) <= 1e-14 * np.max(np.abs(x)) * np.log2(n)


def test_fft_rejects_non_power_of_two():
    with pytest.raises(ValueError):
        O.fft(np.ones(12))
