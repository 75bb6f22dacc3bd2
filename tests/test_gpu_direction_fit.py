"""GPU parity of the device direction fit (au_direction_fit) against the
oracle, level by level:
  - the station times behind each level's scores are the envelope-scan
    maxima of that level's candidates (checked valid against the oracle's
    envelopes on the coarse level);
  - each score equals the oracle's score of the same times (1e-10 relative);
  - each best index is the first minimum of the GPU's scores;
  - each refinement grid equals the oracle's grid around the GPU's previous
    best exactly (both evaluate it in plain double);
and where every level chose the same candidate as the oracle's fit, the
result equals the oracle's exactly."""
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


def check_fit(api, tab, g, t, ev, v, dv, pos, coarse, fit, levels, k, step, tol, check_times=True):
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
        if check_times and lv == 0:
            e, _, _ = oracle_unfold(g, t, v, dirs)
            for d in range(len(dirs)):
                for s in range(len(pos)):
                    env = np.sqrt(O.envelope(e[d, s, 0]) ** 2 + O.envelope(e[d, s, 1]) ** 2)
                    assert env[tt[d, s]] >= env.max() * (1 - 2 * tol), (d, s)
        chi2_ref, pw_ref = O.direction_objective(pos, dirs, tt, S.FS_HZ, peaks=pk)
        n = len(dirs)
        got = fit["chi2"][off:off + n]
        assert np.allclose(got, chi2_ref, rtol=1e-10, atol=1e-9), lv
        assert np.allclose(fit["power"][off:off + n], pw_ref, rtol=1e-12, atol=0), lv
        assert fit["best"][lv] == int(np.argmin(got)), lv
        prev = dirs[fit["best"][lv]]
        off += n
    assert np.array_equal(fit["result"], prev)


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
        if np.array_equal(ref["best"], fit["best"]):
            assert np.array_equal(ref["result"], fit["result"])
            assert np.allclose(ref["chi2"], fit["chi2"], rtol=1e-10, atol=1e-9)


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
    check_fit(api, tab, g, t, ev, v, dv, pos, coarse, fit, 4, 5, (90 / 16, 360 / 32), TOL_FP64, check_times=False)
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
