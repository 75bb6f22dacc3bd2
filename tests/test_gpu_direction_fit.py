"""GPU parity of the device direction fit (au_direction_fit) against the
oracle, level by level:
  - the station times behind each level's scores are the envelope-scan
    maxima of that level's candidates, each checked to be a valid maximum of
    the oracle's total-field envelope at every level (all candidates, or a
    sample of the coarse level at full size);
  - each score equals the oracle's score of the same times (1e-10 relative);
  - each best index is the first minimum of the GPU's scores;
  - each refinement grid equals the oracle's grid around the GPU's previous
    best exactly (both evaluate it in plain double);
and, unconditionally for FP64, against the oracle's own fit: level by level
the grids are equal and the scores agree while both picked the same
candidate; where the picks differ, the oracle's score at the GPU's pick
equals the oracle's minimum within rounding (a tie), and when every level
picked the same candidate the results are equal."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_1507_07733_amd import synth as S

from helpers import TOL_FP32, TOL_FP64, oracle_unfold

pytestmark = pytest.mark.gpu


def say(*a):
    print("[case]", *a, flush=True)


@pytest.fixture(scope="module")
def api():
    import torch
    from paper_1507_07733_amd import api as A
    A.lib()
    torch.cuda.init()
    return A


def check_times_valid(g, t, v, pos, dirs, tt, tol, sel):
    """tt [D][S]: each GPU time is a maximum of the oracle's total-field envelope (directions sel)."""
    units = np.array([[d, s] for d in sel for s in range(len(pos))])
    e, _, _ = oracle_unfold(g, t, v, dirs, units=units)
    for u, (d, s) in enumerate(units):
        env = np.sqrt(O.envelope(e[u, 0]) ** 2 + O.envelope(e[u, 1]) ** 2)
        assert env[tt[d, s]] >= env.max() * (1 - 2 * tol), (d, s)


def check_fit(api, tab, g, t, ev, v, dv, pos, coarse, fit, levels, k, step, tol, coarse_sample=None):
    level_dirs = [np.asarray(coarse, dtype=np.float64)] + [fit["level_dirs"][i] for i in range(levels)]
    off = 0
    prev = None
    for lv, dirs in enumerate(level_dirs):
        if lv > 0:
            sc = 2.0 ** -lv
            assert np.array_equal(dirs, O.local_grid(prev[0], prev[1], step[0] * sc, step[1] * sc, k)), lv
        peak, arg, _ = api.unfold_envelope_scan(tab, ev, dv, dirs)
        pk = peak[..., 2].double().cpu().numpy()
        tt = arg[..., 2].cpu().numpy()
        sel = range(len(dirs))
        if lv == 0 and coarse_sample is not None:
            sel = np.random.default_rng(5).choice(len(dirs), coarse_sample, replace=False)
        check_times_valid(g, t, v, pos, dirs, tt, tol, sel)
        chi2_ref, pw_ref = O.direction_objective(pos, dirs, tt, S.FS_HZ, peaks=pk)
        n = len(dirs)
        got = fit["chi2"][off:off + n]
        assert np.allclose(got, chi2_ref, rtol=1e-10, atol=1e-9), lv
        assert np.allclose(fit["power"][off:off + n], pw_ref, rtol=1e-12, atol=0), lv
        assert fit["best"][lv] == int(np.argmin(got)), lv
        prev = dirs[fit["best"][lv]]
        off += n
    assert np.array_equal(fit["result"], prev)


def compare_with_oracle_fit(ref, fit, coarse, levels, k):
    """Level by level against the oracle's own fit (see the module docstring); returns levels compared."""
    off = 0
    for lv in range(levels + 1):
        n = len(coarse) if lv == 0 else k * k
        if lv > 0:
            assert np.array_equal(ref["level_dirs"][lv - 1], fit["level_dirs"][lv - 1]), lv
        rc = ref["chi2"][off:off + n]
        assert np.allclose(fit["chi2"][off:off + n], rc, rtol=1e-10, atol=1e-9), lv
        if ref["best"][lv] != fit["best"][lv]:
            gb = int(fit["best"][lv])
            assert rc[gb] <= rc.min() * (1 + 1e-9) + 1e-9, (lv, rc[gb], rc.min())
            return lv
        off += n
    assert np.array_equal(ref["result"], fit["result"])
    return levels + 1


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_direction_fit_matches_oracle(api, prec):
    import torch
    g = S.GRID_COARSE
    t = S.pattern_table(g, cfg=0)
    dt = np.float64
    if prec == "fp32":
        t = t.astype(np.complex64)
        dt = np.float32
    tab = api.Table(g, t)
    pos = S.station_positions(30, area_km2=0.5)
    zen, az = 38.0, 290.0
    v, _ = S.plane_wave_traces(pos, 1024, zen, az, cfg=7, event=290, dtype=dt)
    dv = torch.from_numpy(v).cuda()
    coarse = S.direction_grid(6, 12)
    levels, k, step = 3, 5, (15.0, 30.0)
    ev = api.make_event(len(pos), 1024, prec=api.AU_PREC_FP64 if prec == "fp64" else api.AU_PREC_FP32,
                        trace_dtype=api.AU_F64 if prec == "fp64" else api.AU_F32)
    say("direction fit", prec, "S 30 N 1024 coarse 72 levels 3 k 5")
    fit = api.direction_fit(tab, ev, dv, pos, coarse, levels=levels, k=k, step=step)
    check_fit(api, tab, g, t, ev, v, dv, pos, coarse, fit, levels, k, step,
              TOL_FP64 if prec == "fp64" else TOL_FP32)
    z, a = fit["result"]
    assert abs(z - zen) < 1.0 and min(abs(a - az), 360 - abs(a - az)) < 2.0
    if prec == "fp64":
        ref = O.direction_fit(g, t, v, pos, coarse, S.FS_HZ, S.BAND_LO_HZ, S.BAND_HI_HZ, levels=levels, k=k,
                              step=step)
        n_same = compare_with_oracle_fit(ref, fit, coarse, levels, k)
        print("levels matching the oracle's fit pick for pick: %d of %d" % (n_same, levels + 1))


def test_direction_fit_full_station_count_and_errors(api):
    import torch
    g = S.GRID_COARSE
    t = S.pattern_table(g, cfg=0)
    tab = api.Table(g, t)
    pos = S.station_positions(124)
    v, _ = S.plane_wave_traces(pos, 4096, 52.0, 140.0, cfg=7, event=1)
    dv = torch.from_numpy(v).cuda()
    coarse = S.direction_grid(16, 32)
    ev = api.make_event(124, 4096)
    say("direction fit S 124 N 4096 coarse 512 levels 4 k 5; workspace and errors")
    nb = api.direction_fit_workspace_bytes(tab, ev, len(coarse), 4, 5)
    work = torch.empty(nb, dtype=torch.uint8, device="cuda")
    fit = api.direction_fit(tab, ev, dv, pos, coarse, levels=4, k=5, step=(90 / 16, 360 / 32), work=work)
    check_fit(api, tab, g, t, ev, v, dv, pos, coarse, fit, 4, 5, (90 / 16, 360 / 32), TOL_FP64, coarse_sample=12)
    z, a = fit["result"]
    assert abs(z - 52.0) < 1.0 and min(abs(a - 140.0), 360 - abs(a - 140.0)) < 2.0
    fit0 = api.direction_fit(tab, ev, dv, pos, coarse, levels=0, k=5)
    assert fit0["best"][0] == fit["best"][0] and np.array_equal(fit0["chi2"], fit["chi2"][:len(coarse)])
    with pytest.raises(api.AuError):
        api.direction_fit(tab, ev, dv, pos, coarse, levels=4, k=5, step=(90 / 16, 360 / 32), work=work[:-1])
    with pytest.raises(api.AuError):
        api.direction_fit(tab, ev, dv, pos, coarse, levels=2, k=5, step=(0.0, 1.0))
    with pytest.raises(api.AuError):
        api.direction_fit(tab, ev, dv, pos, coarse, levels=17, k=5)
    with pytest.raises(api.AuError):
        api.direction_fit(tab, ev, dv, pos, coarse, levels=1, k=16)
