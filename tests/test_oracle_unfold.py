"""End-to-end pins for the oracle's unfolding (section 2: the E-field trace
is reconstructed per station from the two voltage channels with the
interpolated antenna pattern; section 1: 30-80 MHz band; section 4: FFTs).

Reductions with closed forms or library equivalents:
* identity pattern -> ideal 30-80 MHz band-pass (numpy.fft rfft/irfft);
* fold a known in-band E-field through the pattern, unfold, recover it;
* linearity in the voltages; zero in, zero out;
* N = 16: the full 2N x 2N real linear map, built column by column from
  unit impulses, equals one assembled from brute-force DFT sums and
  numpy.linalg.inv of the interpolated pattern;
* out-of-band tones vanish, in-band tones pass an identity pattern intact;
* horizon (exactly singular pattern) -> zero field and every bin counted.
"""
import numpy as np
import pytest

from oracle import oracle as O
from paper_1507_07733_amd import synth as S

G = S.GRID_COARSE
FS, LO, HI = S.FS_HZ, S.BAND_LO_HZ, S.BAND_HI_HZ


@pytest.fixture(scope="module")
def table():
    return S.pattern_table(G, cfg=0)


def band_mask(n):
    # independent of the oracle: frequencies of rfft bins compared in exact integers
    f_num = np.arange(n // 2 + 1, dtype=np.int64) * FS     # = f * n
    return ((f_num >= LO * n) & (f_num <= HI * n)).astype(float)


def test_identity_pattern_is_bandpass():
    t = S.identity_table(G)
    for n in (16, 2048, 4096):
        v = S.traces(3, n, cfg=0, event=n)
        e, sing, mi = O.unfold(G, t, v, [[40.0, 120.0], [77.0, 300.0]], FS, LO, HI)
        ref = np.fft.irfft(np.fft.rfft(v, axis=-1) * band_mask(n), n=n, axis=-1)
        for d in range(2):
            assert np.max(np.abs(e[d] - ref)) <= 1e-13 * np.max(np.abs(ref))
        assert np.all(sing == 0)
        assert mi < 1e-14


def fold(table, e_field, zen, az, n):
    """V = irfft(H(f_k) E(f_k)) over in-band bins (H from the oracle's interpolation)."""
    E = np.fft.rfft(e_field, axis=-1)                     # [S][2][n/2+1]
    V = np.zeros_like(E)
    for k in np.nonzero(band_mask(n))[0]:
        h = O.pattern_at_bin(G, table, int(k), n, FS, zen, az)
        V[:, :, k] = E[:, :, k] @ h.T
    return np.fft.irfft(V, n=n, axis=-1)


@pytest.mark.parametrize("zen,az", [(40.0, 120.0), (12.3, 357.9), (71.0, 3.3), (85.5, 200.0)])
def test_round_trip_recovers_field(table, zen, az):
    n = 2048
    r = np.random.default_rng(3)
    amp = r.uniform(5, 20, size=(4, 2))
    t0 = r.uniform(0, n, size=(4, 1))
    e_true = S.pulse(n, np.broadcast_to(t0, (4, 2)), amp)   # exactly in band
    v = fold(table, e_true, zen, az, n)
    e, sing, _ = O.unfold(G, table, v, [[zen, az]], FS, LO, HI)
    assert np.all(sing == 0)
    err = np.max(np.abs(e[0] - e_true), axis=-1) / np.max(np.abs(e_true), axis=-1)
    assert np.max(err) <= 1e-12


def test_linearity_and_zero(table):
    n = 4096
    v1 = S.traces(2, n, cfg=0, event=1)
    v2 = S.traces(2, n, cfg=0, event=2)
    dirs = [[22.0, 45.0]]
    e1, _, _ = O.unfold(G, table, v1, dirs, FS, LO, HI)
    e2, _, _ = O.unfold(G, table, v2, dirs, FS, LO, HI)
    e3, _, _ = O.unfold(G, table, 2.5 * v1 - 0.75 * v2, dirs, FS, LO, HI)
    ref = 2.5 * e1 - 0.75 * e2
    assert np.max(np.abs(e3 - ref)) <= 1e-12 * np.max(np.abs(ref))
    ez, _, _ = O.unfold(G, table, np.zeros((2, 2, n)), dirs, FS, LO, HI)
    assert np.all(ez == 0)


def test_dense_linear_map_n16(table):
    n = 16
    zen, az = 31.0, 211.0
    # map built column by column through the oracle
    m_orc = np.zeros((2 * n, 2 * n))
    for c in range(2):
        for j in range(n):
            v = np.zeros((1, 2, n))
            v[0, c, j] = 1.0
            e, _, _ = O.unfold(G, table, v, [[zen, az]], FS, LO, HI)
            m_orc[:, c * n + j] = e[0].reshape(-1)
    # brute force: E_p[t] = (2/N) Re sum_{k in band} Minv[k][p][c] exp(2 pi i k (t - j) / N)
    m_ref = np.zeros_like(m_orc)
    mask = band_mask(n)
    t = np.arange(n)
    for k in np.nonzero(mask)[0]:
        assert 0 < k < n // 2
        minv = np.linalg.inv(O.pattern_at_bin(G, table, int(k), n, FS, zen, az))
        ph = np.exp(2j * np.pi * k * ((t[:, None] - t[None, :]) % n) / n)
        for p in range(2):
            for c in range(2):
                m_ref[p * n:(p + 1) * n, c * n:(c + 1) * n] += (2.0 / n) * np.real(minv[p, c] * ph)
    assert np.max(np.abs(m_orc - m_ref)) <= 1e-13 * np.max(np.abs(m_ref))


def test_tones_in_and_out_of_band():
    t_id = S.identity_table(G)
    n = 2048
    tt = np.arange(n)
    v = np.zeros((1, 2, n))
    v[0, 0] = 3.0 * np.cos(2 * np.pi * ((500 * tt) % n) / n + 0.4)   # 48.8 MHz: in band
    v[0, 1] = 2.0 * np.cos(2 * np.pi * ((100 * tt) % n) / n - 1.0)   # 9.8 MHz: out of band
    e, _, _ = O.unfold(G, t_id, v, [[10.0, 10.0]], FS, LO, HI)
    assert np.max(np.abs(e[0, 0, 0] - v[0, 0])) <= 1e-13 * 3.0
    assert np.max(np.abs(e[0, 0, 1])) <= 1e-14 * 2.0


def test_horizon_is_singular(table):
    n = 2048
    v = S.traces(2, n, cfg=0, event=9)
    e, sing, _ = O.unfold(G, table, v, [[90.0, 120.0], [40.0, 120.0]], FS, LO, HI)
    nb = len(S.band_bins(n))
    assert np.all(sing[0] == nb) and np.all(e[0] == 0)
    assert np.all(sing[1] == 0) and np.max(np.abs(e[1])) > 0


def test_units_subset_matches_full(table):
    n = 2048
    v = S.traces(5, n, cfg=0, event=4)
    dirs = S.direction_grid(2, 3)
    e_full, _, _ = O.unfold(G, table, v, dirs, FS, LO, HI)
    units = np.array([[5, 4], [0, 0], [3, 2]])
    e_u, _, _ = O.unfold(G, table, v, dirs, FS, LO, HI, units=units)
    for i, (d, s) in enumerate(units):
        assert np.array_equal(e_u[i], e_full[d, s])
