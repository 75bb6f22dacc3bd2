"""GPU parity of the device reconstruction loop (au_reconstruct, section 2,
Fig. 1) against the oracle's loop.

Every step is checked on what it must produce, pass by pass:
  - row 0 (voltage maxima, decided in double on both sides) is bit-exact;
  - each direction is the oracle's plane fit of the GPU's times before it;
  - each later row is a valid argmax of the oracle's total-field envelope of
    the oracle's unfold at the GPU's direction (equal unless a near-tie);
and where the GPU's times equal the oracle's at every pass, the directions,
pass count and convergence flag equal the oracle's."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_1507_07733_amd import synth as S

from helpers import TOL_FP32, TOL_FP64, assert_traces_close, oracle_unfold

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


def total_env(e2):
    return np.sqrt(O.envelope(e2[0]) ** 2 + O.envelope(e2[1]) ** 2)


def check_passes(g, t, v, pos, rec, tol):
    """Step-by-step validity of a GPU reconstruction; returns the number of rows equal to the oracle's."""
    vv = np.asarray(v, dtype=np.float64)
    assert np.array_equal(rec.times[0], (vv ** 2).sum(axis=1).argmax(axis=1))
    assert len(rec.times) == len(rec.dirs) + 1
    for i, d in enumerate(rec.dirs):
        ref_d = O.plane_fit(pos, rec.times[i], S.FS_HZ)
        assert abs(d[0] - ref_d[0]) < 1e-9, (i, d, ref_d)
        daz = abs(d[1] - ref_d[1])
        assert min(daz, 360 - daz) < 1e-9, (i, d, ref_d)
        e, _, _ = oracle_unfold(g, t, v, d[None, :])
        for s in range(len(pos)):
            env = total_env(e[0, s])
            assert env[rec.times[i + 1][s]] >= env.max() * (1 - 2 * tol), (i, s)


@pytest.mark.parametrize("max_iter", [5, 10])
def test_reconstruct_every_pass_when_not_converging(api, max_iter):
    """Noise traces whose loop never settles (the oracle runs every pass without converging): the
    device loop's launches then go out in several chunks, each ending with a read of the results,
    and every pass must still be the oracle's."""
    import torch
    g = S.GRID_COARSE
    t = S.pattern_table(g, cfg=0)
    tab = api.Table(g, t)
    n_st, n = 12, 1024
    pos = S.station_positions(n_st, area_km2=6.0 * n_st / 124)
    v = S.traces(n_st, n, cfg=0, event=905)
    o_dirs, o_times, o_conv = O.reconstruct(g, t, v, pos, S.FS_HZ, S.BAND_LO_HZ, S.BAND_HI_HZ, max_iter=max_iter)
    assert len(o_dirs) == max_iter and not o_conv  # the case this test is for
    ev = api.make_event(n_st, n)
    say("reconstruct fp64 noise S", n_st, "N", n, "max_iter", max_iter)
    rec = api.reconstruct(tab, ev, torch.from_numpy(v).cuda(), pos, max_iter=max_iter)
    check_passes(g, t, v, pos, rec, TOL_FP64)
    assert rec.times.shape == o_times.shape and np.array_equal(rec.times, o_times)
    assert rec.converged == o_conv
    assert np.max(np.abs(rec.dirs - o_dirs)) < 1e-9


@pytest.mark.parametrize("n_st,n,zen,az", [(40, 2048, 35.0, 120.0), (124, 4096, 55.0, 250.0),
                                           (124, 2048, 20.0, 10.0)])
def test_reconstruct_fp64_matches_oracle(api, n_st, n, zen, az):
    import torch
    g = S.GRID_COARSE
    t = S.pattern_table(g, cfg=0)
    tab = api.Table(g, t)
    pos = S.station_positions(n_st, area_km2=6.0 * n_st / 124)
    v, _ = S.plane_wave_traces(pos, n, zen, az, cfg=6, event=n_st + n)
    ev = api.make_event(n_st, n)
    say("reconstruct fp64 S", n_st, "N", n, "dir", zen, az)
    rec = api.reconstruct(tab, ev, torch.from_numpy(v).cuda(), pos, max_iter=8, efield=True)
    check_passes(g, t, v, pos, rec, TOL_FP64)
    o_dirs, o_times, o_conv = O.reconstruct(g, t, v, pos, S.FS_HZ, S.BAND_LO_HZ, S.BAND_HI_HZ, max_iter=8)
    assert rec.times.shape == o_times.shape and np.array_equal(rec.times, o_times)
    assert rec.converged == o_conv
    assert np.max(np.abs(rec.dirs - o_dirs)) < 1e-9
    # the final traces and envelope maxima are those of the final direction
    ref, _, _ = oracle_unfold(g, t, v, rec.direction[None, :])
    assert_traces_close(rec.efield.cpu().numpy(), ref[0], TOL_FP64, "final traces")
    peak, arg, _ = api.unfold_envelope_scan(tab, ev, torch.from_numpy(v).cuda(), rec.direction[None, :])
    assert torch.equal(rec.peak.cpu(), peak[0].cpu())
    assert np.array_equal(arg[0, :, 2].cpu().numpy(), rec.times[-1])
    zf, af = rec.direction
    assert abs(zf - zen) < 1.0 and min(abs(af - az), 360 - abs(af - az)) < 2.0


def test_reconstruct_fp32(api):
    import torch
    g = S.GRID_FINE
    t32 = S.pattern_table(g, cfg=2).astype(np.complex64)
    tab = api.Table(g, t32)
    pos = S.station_positions(124)
    n = 4096
    v, _ = S.plane_wave_traces(pos, n, 48.0, 300.0, cfg=6, event=9, dtype=np.float32)
    ev = api.make_event(len(pos), n, prec=api.AU_PREC_FP32, trace_dtype=api.AU_F32)
    say("reconstruct fp32 S 124 N 4096")
    rec = api.reconstruct(tab, ev, torch.from_numpy(v).cuda(), pos, max_iter=6)
    check_passes(g, t32, v, pos, rec, TOL_FP32)
    zf, af = rec.direction
    assert abs(zf - 48.0) < 1.0 and min(abs(af - 300.0), 360 - abs(af - 300.0)) < 2.0


def test_reconstruct_small_and_single_pass(api):
    import torch
    g = S.GRID_COARSE
    t = S.pattern_table(g, cfg=0)
    tab = api.Table(g, t)
    pos = S.station_positions(3, area_km2=0.01)
    v, _ = S.plane_wave_traces(pos, 256, 30.0, 45.0, cfg=6, event=3)
    ev = api.make_event(3, 256)
    say("reconstruct S 3 N 256 max_iter 1")
    rec = api.reconstruct(tab, ev, torch.from_numpy(v).cuda(), pos, max_iter=1)
    o_dirs, o_times, o_conv = O.reconstruct(g, t, v, pos, S.FS_HZ, S.BAND_LO_HZ, S.BAND_HI_HZ, max_iter=1)
    assert len(rec.dirs) == 1 and rec.times.shape == (2, 3)
    check_passes(g, t, v, pos, rec, TOL_FP64)
    assert rec.converged == o_conv
    if np.array_equal(rec.times, o_times):
        assert np.max(np.abs(rec.dirs - o_dirs)) < 1e-9
    # a workspace of the stated size gives the same result; one byte less is refused
    nb = api.reconstruct_workspace_bytes(tab, ev, 1)
    work = torch.empty(nb, dtype=torch.uint8, device="cuda")
    rec2 = api.reconstruct(tab, ev, torch.from_numpy(v).cuda(), pos, max_iter=1, work=work)
    assert np.array_equal(rec2.times, rec.times) and np.array_equal(rec2.dirs, rec.dirs)
    with pytest.raises(api.AuError):
        api.reconstruct(tab, ev, torch.from_numpy(v).cuda(), pos, max_iter=1, work=work[:-1])


def test_reconstruct_rejects_degenerate_geometry(api):
    import torch
    g = S.GRID_COARSE
    tab = api.Table(g, S.pattern_table(g, cfg=0))
    pos = np.array([[0.0, 0.0], [100.0, 50.0], [200.0, 100.0], [300.0, 150.0]])   # collinear
    v = S.traces(4, 512, cfg=4, event=1)
    ev = api.make_event(4, 512)
    say("reconstruct collinear stations")
    with pytest.raises(api.AuError) as ex:
        api.reconstruct(tab, ev, torch.from_numpy(v).cuda(), pos, max_iter=4)
    assert ex.value.status == api.AU_EINVAL
    with pytest.raises(ValueError):
        O.plane_fit(pos, [0, 1, 2, 3], S.FS_HZ)
    bad = pos.copy()
    bad[1, 0] = np.nan
    with pytest.raises(api.AuError):
        api.reconstruct(tab, ev, torch.from_numpy(v).cuda(), bad, max_iter=4)
    with pytest.raises(api.AuError):
        api.reconstruct(tab, ev, torch.from_numpy(v).cuda(), pos, max_iter=0)


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_reconstruct_batch_equals_single(api, prec):
    """Many events in one call (uneven station counts, a shared input, a degenerate layout): every
    event's directions, times, pass count and stop reason equal the one-event loop's, bitwise."""
    import torch
    f32 = prec == "fp32"
    g = S.GRID_COARSE
    t = S.pattern_table(g, cfg=0)
    if f32:
        t = t.astype(np.complex64)
    tab = api.Table(g, t)
    n = 2048
    dt = np.float32 if f32 else np.float64
    cases = [(40, 1.9, 35.0, 120.0), (124, 6.0, 20.0, 10.0), (3, 0.01, 30.0, 45.0), (17, 0.8, 50.0, 300.0),
             (60, 2.9, 10.0, 200.0)]
    pos_l, vol_l = [], []
    for i, (ns, area, z, a) in enumerate(cases):
        p = S.station_positions(ns, area_km2=area)
        v, _ = S.plane_wave_traces(p, n, z, a, cfg=8, event=i, dtype=dt)
        pos_l.append(p)
        vol_l.append(v)
    # event 5 reuses event 1's traces; event 6 has collinear stations
    pos_l.append(pos_l[1])
    col = np.stack([np.linspace(0, 400, 5), np.linspace(0, 200, 5)], 1)
    pos_l.append(col)
    vol_l.append(S.traces(5, n, cfg=8, event=9, dtype=dt))
    ns = [len(p) for p in pos_l]
    offs, flat, o = [], [], 0
    for i in range(len(ns)):
        if i == 5:
            offs.append(offs[1])
            continue
        v = vol_l[i if i < 5 else 5]
        offs.append(o)
        flat.append(v.ravel())
        o += v.size
    volt = torch.from_numpy(np.concatenate(flat)).cuda()
    ev = api.make_event(3, n, prec=api.AU_PREC_FP32 if f32 else api.AU_PREC_FP64,
                        trace_dtype=api.AU_F32 if f32 else api.AU_F64)
    say("reconstruct batch", prec, "events", len(ns))
    res = api.reconstruct_batch(tab, ev, volt, ns, offs, np.concatenate(pos_l), max_iter=6)
    for i, r in enumerate(res):
        evi = api.make_event(ns[i], n, prec=ev.prec, trace_dtype=ev.trace_dtype)
        vi = volt[offs[i]:offs[i] + ns[i] * 2 * n].view(ns[i], 2, n)
        if i == 6:
            assert r.converged == -1
            with pytest.raises(api.AuError):
                api.reconstruct(tab, evi, vi, pos_l[i], max_iter=6)
            continue
        one = api.reconstruct(tab, evi, vi, pos_l[i], max_iter=6)
        assert np.array_equal(r.dirs, one.dirs), i
        assert np.array_equal(r.times, one.times), i
        assert r.converged == int(one.converged), i
    assert np.array_equal(res[5].dirs, res[1].dirs) and np.array_equal(res[5].times, res[1].times)
