"""Pins for the oracle's reconstruction loop (section 2, Fig. 1): plane-wave
triangulation recovers a known direction from exact arrival times, and the
full loop (voltage timing -> triangulation -> unfold -> envelope timing)
converges near the true direction of a synthetic plane-wave event."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_1507_07733_amd import synth as S


@pytest.mark.parametrize("zen,az", [(10.0, 30.0), (45.0, 200.0), (65.0, 300.0), (30.0, 359.0)])
def test_plane_fit_recovers_direction(zen, az):
    pos = S.station_positions()
    fs = 10 ** 15            # femtosecond samples: rounding the times is negligible
    t = np.round(5e14 + S.plane_wave_delays(pos, zen, az, fs_hz=fs)).astype(np.int64)
    d = O.plane_fit(pos, t, fs)
    assert abs(d[0] - zen) < 1e-6
    assert min(abs(d[1] - az), 360 - abs(d[1] - az)) < 1e-5


def test_plane_fit_rejects_collinear_stations():
    pos = np.array([[0.0, 0.0], [100.0, 0.0], [200.0, 0.0], [300.0, 0.0]])
    with pytest.raises(ValueError):
        O.plane_fit(pos, [0, 1, 2, 3], S.FS_HZ)


@pytest.mark.parametrize("zen,az", [(35.0, 120.0), (55.0, 250.0)])
def test_reconstruction_converges_near_truth(zen, az):
    g = S.GRID_COARSE
    t = S.pattern_table(g, cfg=0)
    pos = S.station_positions(40, area_km2=2.0)
    v, t_true = S.plane_wave_traces(pos, 2048, zen, az, cfg=6, event=int(zen))
    dirs, times, conv = O.reconstruct(g, t, v, pos, S.FS_HZ, S.BAND_LO_HZ, S.BAND_HI_HZ, max_iter=6)
    assert conv
    assert len(times) == len(dirs) + 1
    assert np.array_equal(times[-1], times[-2])          # converged: the last pass repeated its times
    pw = (v.astype(np.float64) ** 2).sum(axis=1)
    assert np.array_equal(times[0], pw.argmax(axis=1))    # first times: voltage maxima
    # every direction is the plane fit of the times before it
    for i, d in enumerate(dirs):
        assert np.allclose(O.plane_fit(pos, times[i], S.FS_HZ), d, rtol=0, atol=1e-12)
    # the final times are the total-field envelope maxima of the unfold at the final direction
    e, _, _ = O.unfold(g, t, v, dirs[-1:], S.FS_HZ, S.BAND_LO_HZ, S.BAND_HI_HZ)
    for s in range(len(pos)):
        tot = np.sqrt(O.envelope(e[0, s, 0]) ** 2 + O.envelope(e[0, s, 1]) ** 2)
        assert tot.argmax() == times[-1][s]
    times = times[-1]
    zf, af = dirs[-1]
    assert abs(zf - zen) < 1.0
    assert min(abs(af - az), 360 - abs(af - az)) < 2.0
    # the timings are a plane wave up to a common offset (group delay of the unfolding)
    off = np.median(times - t_true)
    assert np.percentile(np.abs(times - t_true - off), 90) < 6
