"""Synthetic-input generator checks and the numbers the paper prints."""
import json
import os

import numpy as np

from paper_1507_07733_amd import synth as S

GOLD = os.path.join(os.path.dirname(__file__), "golden", "paper_facts.json")


def facts():
    with open(GOLD) as f:
        return json.load(f)


def test_paper_fp32_interpolation_bound_reading():
    # Reading: trilinear interpolation = 7 one-dimensional lerps, each of the
    # paper's six elementary operations adding at most one unit roundoff.
    f = facts()
    ops = f["fp32_linear_interp_ops"]["value"]
    bound = 7 * ops * 2.0 ** -24
    assert abs(bound - f["fp32_interp_max_rel_error"]["value"]) / bound < 0.01


def test_paper_pattern_footprint():
    f = facts()
    nf, nz, na = f["largest_pattern_nodes"]["value"]
    # two complex components (theta, phi) of 2 x 4 bytes each per node
    mb = nf * nz * na * 2 * 8 / 1e6
    assert abs(mb - f["largest_pattern_mbytes_fp32"]["value"]) < 0.05


def test_generator_is_deterministic():
    a = S.traces(4, 2048, cfg=1, event=3)
    b = S.traces(4, 2048, cfg=1, event=3)
    c = S.traces(4, 2048, cfg=1, event=4)
    assert np.array_equal(a, b) and not np.array_equal(a, c)
    assert np.array_equal(S.pattern_table(S.GRID_COARSE, 0), S.pattern_table(S.GRID_COARSE, 0))


def test_pulse_is_band_limited():
    f = facts()
    lo, hi = f["antenna_band_mhz"]["value"]
    for n in (2048, 4096):
        p = S.pulse(n, np.array([123.45]), np.array([10.0]))[0]
        spec = np.abs(np.fft.rfft(p))
        freq = np.arange(n // 2 + 1) * S.FS_HZ / n / 1e6
        out = (freq < lo) | (freq > hi)
        assert spec[out].max() <= 1e-11 * spec.max()


def test_table_horizon_and_dc():
    g = S.GRID_COARSE
    t = S.pattern_table(g, 0)
    assert np.all(t[:, 0, :, g.n_zen - 1, :] == 0)       # cos(90 deg) exactly zero
    assert np.all(t[:, :, 0] == 0)                       # resonance zero at DC
    assert np.all(np.isfinite(t))


def test_direction_grid_cell_centred():
    d = S.direction_grid(32, 64)
    assert d.shape == (2048, 2)
    assert d[0, 0] == 90.0 / 64 and d[-1, 0] == 90.0 - 90.0 / 64
    assert d[1, 1] == 360.0 / 64 and d.max(axis=0)[1] < 360.0


def test_event_mix_shapes():
    ev = S.event_mix(256, cfg=2)
    s = np.array([e.n_stations for e in ev])
    n = np.array([e.n_samples for e in ev])
    assert s.min() >= 3 and s.max() <= 124
    assert set(n.tolist()) <= {2048, 4096}
    assert 0.35 < np.mean(n == 2048) < 0.65


def test_counter_stream_properties():
    """The counter-based trace stream: deterministic, independent of which stations are asked for, noise of
    unit variance (Irwin-Hall sums), distinct events and channels, and the pulse where the stream puts it."""
    from paper_1507_07733_amd import synth as S
    a = S.stream_traces([3, 1000], 4, 1024)
    b = S.stream_traces([3, 1000], 4, 1024)
    assert a.dtype == np.float32 and a.shape == (2, 4, 2, 1024) and np.array_equal(a, b)
    sub = S.stream_traces([1000], 4, 1024, stations=[2, 0])[0]
    assert np.array_equal(sub[0], a[1, 2]) and np.array_equal(sub[1], a[1, 0])
    assert not np.array_equal(a[0], a[1]) and not np.array_equal(a[0, 0, 0], a[0, 0, 1])
    # 32-bit words of Philox are close to uniform: mean of 2^32-scaled words ~ 1/2
    r = S.philox4x32(np.arange(20000, dtype=np.uint64), 1, 2, 3, 7733, 0x7733)
    u = np.concatenate(r).astype(np.float64) / 2.0 ** 32
    assert abs(u.mean() - 0.5) < 0.005 and abs(u.var() - 1.0 / 12) < 0.002
    # noise alone (the pulse table zeroed) has mean 0 and variance 1
    d = S.dirichlet_table(1024)
    assert d[0] == np.float32(1.0) and abs(float(np.sum(d))) < 1e-3
    big = S.stream_traces(range(8), 8, 1024)
    resid = big.astype(np.float64)
    e_amp = []
    for e in range(8):
        for s in range(8):
            t0 = int(S.philox4x32(0, s, e, 1, 7733, 0x7733)[0]) & 1023
            for c in range(2):
                ua = np.float32(int(S.philox4x32(0, 2 * s + c, e, 2, 7733, 0x7733)[0]) >> 8) * np.float32(2.0 ** -24)
                amp = np.float32(np.float32(5.0) + np.float32(np.float32(15.0) * ua))
                e_amp.append(amp)
                resid[e, s, c] -= amp * np.roll(d, t0)
    assert min(e_amp) >= 5.0 and max(e_amp) < 20.0
    assert abs(resid.mean()) < 0.02 and abs(resid.var() - 1.0) < 0.03
