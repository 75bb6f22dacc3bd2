"""Pins for the oracle's pattern interpolation (section 3: the vector
effective length is known on discrete frequency/zenith/azimuth nodes and is
linearly interpolated in between).

Pinned by: exact reproduction of node values; exact reproduction of a
function that is multilinear in (frequency, zenith, azimuth) node position,
with the expected value computed from exact rational node positions; the
closed-form lerp across the azimuth wrap; zenith clamping; azimuth
periodicity.
"""
from fractions import Fraction

import numpy as np
import pytest

from oracle import oracle as O
from paper_1507_07733_amd import synth as S

G = S.GRID_COARSE
FS = S.FS_HZ


@pytest.fixture(scope="module")
def table():
    return S.pattern_table(G, cfg=0)


def test_exact_at_nodes(table):
    # N = 2048 at 200 MHz: bins 512 and 768 are 50 and 75 MHz, exactly on the 1 MHz grid.
    for k, fi in ((512, 50), (768, 75)):
        for zen, az in ((40.0, 120.0), (0.0, 0.0), (85.0, 355.0), (90.0, 5.0)):
            h = O.pattern_at_bin(G, table, k, 2048, FS, zen, az)
            zi, ai = int(zen / 5), int(az / 5)
            ref = table[:, :, fi, zi, ai]
            assert np.array_equal(h, ref), (k, zen, az)


def _node_position(k, n, fs, f0, df):
    return Fraction(k * fs - f0 * n, n * df)


def test_multilinear_reproduced(table):
    a = np.array([[0.3 + 0.1j, -1.2 + 0.5j], [0.7 - 0.2j, 2.0 + 0.0j]])
    b = np.array([[0.01, -0.02j], [0.03 + 0.01j, 0.005]])
    gz = np.array([[1.0, 0.5], [-0.25, 2.0]])
    dz = np.array([[0.1, -0.05], [0.2, 0.07]])
    ea = np.array([[2.0, 1.0], [0.5, -1.0]])
    za = np.array([[0.03, 0.2], [-0.1, 0.04]])
    fi = np.arange(G.n_freq)[:, None, None]
    zi = np.arange(G.n_zen)[None, :, None]
    ai = np.arange(G.n_az)[None, None, :]
    t = np.empty(G.shape, complex)
    for c in range(2):
        for p in range(2):
            t[c, p] = (a[c, p] + b[c, p] * fi) * (gz[c, p] + dz[c, p] * zi) * (ea[c, p] + za[c, p] * ai)
    r = np.random.default_rng(5)
    for _ in range(40):
        n = int(r.choice([2048, 4096]))
        kb = S.band_bins(n)
        k = int(r.choice(kb))
        zen = float(r.uniform(0, 90))
        az = float(r.uniform(0, 354.99))       # stay off the wrap cell
        h = O.pattern_at_bin(G, t, k, n, FS, zen, az)
        fpos = float(_node_position(k, n, FS, G.f0_hz, G.df_hz))
        zpos = zen / G.dzen_deg
        apos = az / G.daz_deg
        for c in range(2):
            for p in range(2):
                ref = (a[c, p] + b[c, p] * fpos) * (gz[c, p] + dz[c, p] * zpos) * (ea[c, p] + za[c, p] * apos)
                assert abs(h[c, p] - ref) <= 1e-13 * max(1.0, abs(ref)), (k, n, zen, az, c, p)


def test_azimuth_wrap_cell(table):
    k, n = 512, 2048                 # on a frequency node
    zen = 40.0                       # on a zenith node
    for az in (355.0, 356.25, 358.0, 359.999):
        h = O.pattern_at_bin(G, table, k, n, FS, zen, az)
        tw = (az - 355.0) / 5.0
        ref = (1 - tw) * table[:, :, 50, 8, 71] + tw * table[:, :, 50, 8, 0]
        assert np.max(np.abs(h - ref)) <= 1e-15 * np.max(np.abs(ref)) * 4


def test_azimuth_periodic(table):
    for az in (12.5, 200.0, 355.5):
        h0 = O.pattern_at_bin(G, table, 600, 2048, FS, 33.3, az)
        for shift in (-360.0, 360.0, 720.0):
            h1 = O.pattern_at_bin(G, table, 600, 2048, FS, 33.3, az + shift)
            assert np.max(np.abs(h1 - h0)) <= 1e-13 * np.max(np.abs(h0))


def test_zenith_clamped(table):
    h90 = O.pattern_at_bin(G, table, 512, 2048, FS, 90.0, 120.0)
    assert np.array_equal(h90, table[:, :, 50, 18, 24])
    assert np.array_equal(O.pattern_at_bin(G, table, 512, 2048, FS, 97.0, 120.0), h90)
    assert np.array_equal(O.pattern_at_bin(G, table, 512, 2048, FS, -3.0, 120.0), table[:, :, 50, 0, 24])
    # horizon: theta components vanish exactly
    assert np.all(h90[:, 0] == 0)


def test_bin_outside_table_rejected(table):
    small = S.Grid(40, 19, 72, 0, 1_000_000, 0.0, 5.0, 0.0, 5.0)      # 0..39 MHz only
    with pytest.raises(ValueError):
        O.pattern_at_bin(small, np.zeros(small.shape, complex), 800, 2048, FS, 10.0, 10.0)


# ---- texture-filter weights (interpolation weights rounded to fixed point) ----

def test_quantized_fine_limit_and_nodes(table):
    """30 fractional bits reproduce the exact interpolation; nodes stay exact at any precision."""
    r = np.random.default_rng(3)
    for _ in range(20):
        k = int(r.integers(300, 900))
        z, a = r.uniform(0, 90), r.uniform(0, 360)
        h = O.pattern_at_bin(G, table, k, 2048, S.FS_HZ, z, a)
        hq = O.pattern_at_bin_quantized(G, table, k, 2048, S.FS_HZ, z, a, 30)
        assert np.max(np.abs(hq - h)) <= 1e-8 * np.max(np.abs(table))
    # bin 512 of 2048 at 200 MHz is 50 MHz, a frequency node; zenith and azimuth on nodes
    for b in (1, 4, 8):
        hq = O.pattern_at_bin_quantized(G, table, 512, 2048, S.FS_HZ, 35.0, 120.0, b)
        assert np.array_equal(hq, table[:, :, 50, 7, 24])


def test_quantized_one_bit_is_midpoint(table):
    """1 fractional bit: weight 0.3 becomes 0.5, weight 0.2 becomes 0; the value is a two-node mean."""
    # frequency and zenith on nodes (50 MHz, 35 deg); azimuth 120 + 0.3 * 5 deg lies between nodes 24 and 25
    hq = O.pattern_at_bin_quantized(G, table, 512, 2048, S.FS_HZ, 35.0, 121.5, 1)
    assert np.allclose(hq, 0.5 * (table[:, :, 50, 7, 24] + table[:, :, 50, 7, 25]), rtol=1e-15, atol=0)
    hq = O.pattern_at_bin_quantized(G, table, 512, 2048, S.FS_HZ, 35.0, 121.0, 1)
    assert np.array_equal(hq, table[:, :, 50, 7, 24])


def test_quantized_error_bound(table):
    """Moving one weight by d moves a trilinear value by at most d times the largest node difference
    along that axis in the cell; 8 bits give d <= 2^-9 per axis."""
    r = np.random.default_rng(4)
    n, fs = 2048, S.FS_HZ
    for _ in range(60):
        k = int(r.integers(300, 900))
        z, a = r.uniform(0, 89.9), r.uniform(0, 360)
        h = O.pattern_at_bin(G, table, k, n, fs, z, a)
        hq = O.pattern_at_bin_quantized(G, table, k, n, fs, z, a, 8)
        fpos = k * fs / n / G.df_hz
        i_f, i_z, i_a = int(fpos), int(z // G.dzen_deg), int(a // G.daz_deg)
        cell = table[:, :, i_f:i_f + 2, i_z:i_z + 2][..., [i_a, (i_a + 1) % G.n_az]]   # [2][2][2f][2z][2a]
        bound = 0.0
        for ax in (2, 3, 4):
            diff = np.abs(np.diff(cell, axis=ax))
            bound += 2.0 ** -9 * diff.max()
        assert np.max(np.abs(hq - h)) <= bound * (1 + 1e-9) + 1e-15
