"""Pins for the oracle's direction-fit score and refinement (reading: the
timing inconsistency of the unfolded stations with a plane wave from the
candidate direction, minimised over candidates, then refined locally)."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_1507_07733_amd import synth as S


def test_objective_is_least_squares_residual():
    """chi2 = residual sum of squares of the one-parameter least-squares fit of t0 (numpy lstsq),
    with the plane-wave delays taken from the input generator."""
    r = np.random.default_rng(1)
    pos = S.station_positions(25, area_km2=1.0)
    dirs = np.array([[10.0, 30.0], [45.0, 200.0], [70.0, 359.5], [0.0, 0.0]])
    times = r.integers(0, 2048, size=(len(dirs), len(pos)))
    chi2, _ = O.direction_objective(pos, dirs, times, S.FS_HZ)
    dt = 1e9 / S.FS_HZ
    for i, (z, a) in enumerate(dirs):
        b = (times[i] - S.plane_wave_delays(pos, z, a, S.FS_HZ)) * dt
        _, res, _, _ = np.linalg.lstsq(np.ones((len(pos), 1)), b, rcond=None)
        assert chi2[i] == pytest.approx(res[0], rel=1e-10)


def test_objective_vanishes_for_the_true_direction():
    pos = S.station_positions(40, area_km2=2.0)
    fs = 10 ** 15
    t = np.round(3e14 + S.plane_wave_delays(pos, 35.0, 120.0, fs)).astype(np.int64)
    dirs = np.array([[35.0, 120.0], [36.0, 120.0], [35.0, 121.0], [30.0, 300.0]])
    chi2, _ = O.direction_objective(pos, dirs, np.tile(t, (len(dirs), 1)), fs)
    assert chi2[0] < 1e-6                      # ns^2: only the femtosecond rounding remains
    assert np.all(chi2[1:] > 1e2)
    # a common shift of every time does not change the score
    chi2s, _ = O.direction_objective(pos, dirs, np.tile(t + 12345, (len(dirs), 1)), fs)
    assert np.allclose(chi2s, chi2, rtol=1e-9, atol=1e-6)


def test_power_is_sum_of_squared_peaks():
    pos = S.station_positions(5)
    pk = np.arange(10.0).reshape(2, 5)
    _, pw = O.direction_objective(pos, [[1.0, 2.0], [3.0, 4.0]], np.zeros((2, 5)), S.FS_HZ, peaks=pk)
    assert np.array_equal(pw, [0 + 1 + 4 + 9 + 16, 25 + 36 + 49 + 64 + 81])


def test_local_grid_values():
    g = O.local_grid(45.0, 10.0, 1.0, 2.0, 3)
    assert np.array_equal(g, [[44, 8], [44, 10], [44, 12], [45, 8], [45, 10], [45, 12], [46, 8], [46, 10], [46, 12]])
    g = O.local_grid(0.5, 1.0, 1.0, 2.0, 3)       # zenith clamp at 0, azimuth wrap below 0
    assert np.array_equal(g[:, 0], [0, 0, 0, 0.5, 0.5, 0.5, 1.5, 1.5, 1.5])
    assert np.array_equal(g[:3, 1], [359, 1, 3])
    g = O.local_grid(89.5, 359.0, 1.0, 1.0, 3)    # zenith clamp at 90, azimuth wrap at 360
    assert np.array_equal(g[6:, 0], [90, 90, 90])
    assert np.array_equal(g[:3, 1], [358, 359, 0])
    assert np.array_equal(O.local_grid(12.0, 34.0, 1.0, 1.0, 1), [[12.0, 34.0]])


@pytest.mark.parametrize("zen,az", [(25.0, 40.0), (38.0, 290.0)])
def test_fit_converges_near_truth(zen, az):
    g = S.GRID_COARSE
    t = S.pattern_table(g, cfg=0)
    pos = S.station_positions(30, area_km2=0.5)
    v, _ = S.plane_wave_traces(pos, 1024, zen, az, cfg=7, event=int(az))
    coarse = S.direction_grid(6, 12)            # 7.5 deg x 30 deg cells
    fit = O.direction_fit(g, t, v, pos, coarse, S.FS_HZ, S.BAND_LO_HZ, S.BAND_HI_HZ, levels=3, k=5,
                          step=(15.0, 30.0))
    z, a = fit["result"]
    assert abs(z - zen) < 1.0 and min(abs(a - az), 360 - abs(a - az)) < 2.0
    # each level's best is at least as good as the previous level's best (the centre is in the grid)
    off = [0] + [len(coarse) + 25 * i for i in range(3)]
    bests = [fit["chi2"][off[i] + fit["best"][i]] for i in range(4)]
    assert all(bests[i + 1] <= bests[i] + 1e-9 for i in range(3))
    assert fit["best"][0] == np.argmin(fit["chi2"][:len(coarse)])
