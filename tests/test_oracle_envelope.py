"""Pins for the oracle's Hilbert envelope (section 4: envelope = magnitude
of the analytic signal; section 2: its maximum times the station).

Closed forms: the Hilbert transform of cos is sin, so a pure tone has a
constant envelope equal to its amplitude; an amplitude-modulated tone
A (1 + m cos(w_m t)) cos(w_c t) (all components strictly between DC and
Nyquist, carrier above the modulation) has envelope A (1 + m cos(w_m t));
scipy.signal.hilbert computes the analytic signal by the same definition.
"""
import numpy as np
import pytest

from oracle import oracle as O


@pytest.mark.parametrize("n,k0,a,ph", [(64, 5, 1.0, 0.0), (2048, 411, 3.5, 1.1), (4096, 1000, 0.25, -2.0)])
def test_tone_has_constant_envelope(n, k0, a, ph):
    t = np.arange(n)
    x = a * np.cos(2 * np.pi * ((k0 * t) % n) / n + ph)
    env = O.envelope(x)
    assert np.max(np.abs(env - a)) <= 1e-12 * a


def test_am_tone_envelope():
    n = 2048
    t = np.arange(n)
    kc, km, m, a = 500, 7, 0.6, 2.0
    x = a * (1 + m * np.cos(2 * np.pi * ((km * t) % n) / n)) * np.cos(2 * np.pi * ((kc * t) % n) / n)
    env = O.envelope(x)
    ref = a * (1 + m * np.cos(2 * np.pi * ((km * t) % n) / n))
    assert np.max(np.abs(env - ref)) <= 1e-12 * a


def test_matches_scipy_hilbert():
    sig = pytest.importorskip("scipy.signal")
    r = np.random.default_rng(3)
    x = r.standard_normal(1024)
    x -= x.mean()
    ref = np.abs(sig.hilbert(x))
    # scipy keeps the Nyquist bin in the analytic signal; remove it from the input
    X = np.fft.fft(x)
    X[512] = 0
    x = np.real(np.fft.ifft(X))
    ref = np.abs(sig.hilbert(x))
    assert np.max(np.abs(O.envelope(x) - ref)) <= 1e-12 * ref.max()


def test_peaks_first_index_and_shape():
    n = 256
    tr = np.zeros((2, 3, n))
    tt = np.arange(n)
    for i in range(2):
        for j in range(3):
            tr[i, j] = (1 + i + j) * np.cos(2 * np.pi * ((20 * tt) % n) / n) * np.exp(-0.5 * ((tt - 40 - 30 * j) / 6.0) ** 2)
    peak, arg = O.envelope_peaks(tr)
    assert peak.shape == (2, 3) and arg.shape == (2, 3)
    env = np.stack([[O.envelope(tr[i, j]) for j in range(3)] for i in range(2)])
    assert np.array_equal(peak, env.max(axis=-1))
    assert np.array_equal(arg, env.argmax(axis=-1))
    assert np.all(np.abs(arg - (40 + 30 * np.arange(3))[None, :]) <= 1)
