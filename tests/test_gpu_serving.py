"""GPU tests of the continuous-batching server (au_server_*): results equal
alone and in a mix, FIFO admission under a memory budget, lifecycle and
error codes.  Each test prints its case before touching the GPU."""
import time

import numpy as np
import pytest

from paper_1507_07733_amd import synth as S

from helpers import TOL_FP32, TOL_FP64, assert_fp32_close, assert_traces_close, oracle_unfold

pytestmark = pytest.mark.gpu

GF = S.GRID_FINE


def say(*a):
    print("[case]", *a, flush=True)


@pytest.fixture(scope="module")
def api():
    import torch
    from paper_1507_07733_amd import api as A
    A.lib()
    torch.cuda.init()
    return A


@pytest.fixture(scope="module")
def fine32(api):
    t = S.pattern_table(GF, cfg=2).astype(np.complex64)
    return t, api.Table(GF, t)


def event_bytes(s, n, d, el=4):
    return d * s * 2 * n * el + s * 2 * n * el + (s + d) * n * 16


def test_result_same_alone_and_in_mix(api, fine32):
    """Continuous batching: a burst is grouped into shared launches (the target shares its batch with
    other events), and the target's result is bitwise the same alone and in the mix."""
    t, tab = fine32
    dirs = S.direction_grid(4, 4)
    target = S.traces(37, 2048, cfg=3, event=7, dtype=np.float32)
    r = np.random.default_rng(5)
    others = []
    for i in range(24):
        s = int(r.integers(3, 125))
        n = int(r.choice([2048, 4096]))
        others.append(S.traces(s, n, cfg=3, event=100 + i, dtype=np.float32))
    say("server alone")
    sv = api.Server(tab, hbm_budget_bytes=8 << 30, staging_bytes=512 << 20, n_streams=4,
                    max_batch_events=8, tick_s=0.05)
    try:
        tk = sv.submit(target, dirs)
        res = sv.wait(tk)
        assert res.batch_events == 1
        alone = sv.result(tk)
        sv.release(tk)
        say("server mix: burst of 25 events, batches of up to 8")
        tickets = []
        for i, v in enumerate(others):
            if i == 11:
                tickets.append(("target", sv.submit(target, dirs)))
            tickets.append(("other", sv.submit(v, S.direction_grid(2, 4))))
        mixed = None
        by_batch = {}
        target_res = None
        for kind, tkn in tickets:
            res = sv.wait(tkn)
            assert res.t_arrival <= res.t_admit <= res.t_launch <= res.t_complete
            by_batch.setdefault(res.batch_id, []).append(kind)
            assert res.batch_events >= 1
            if kind == "target":
                mixed = sv.result(tkn)
                target_res = (res.batch_id, res.batch_events)
            sv.release(tkn)
        st = sv.stats()
        sizes = sorted(len(v) for v in by_batch.values())
        print("batch sizes", sizes, "stats", st)
        assert st["completed"] == 26 and st["in_flight"] == 0 and st["arena_in_use"] == 0
        assert max(sizes) > 1
        bid, bev = target_res
        assert bev > 1 and len(by_batch[bid]) == bev and by_batch[bid].count("other") == bev - 1
        # same kernels and per-unit arithmetic whatever the batch: identical
        assert np.array_equal(alone, mixed)
        units = np.array([[0, 0], [5, 36], [15, 20], [9, 3]])
        ref, _, _ = oracle_unfold(GF, t, target, dirs, units=units)
        got = np.stack([alone[d, s] for d, s in units])
        assert_fp32_close(got, ref, TOL_FP32, "served")
    finally:
        sv.close()


def test_arena_filled_exactly_still_launches(api, fine32):
    """Admitted events that fill the arena to the byte still launch (batch descriptors never need arena
    space), and the queued fourth event is admitted once one is released."""
    t, tab = fine32
    dirs = S.direction_grid(2, 3)
    s, n = 20, 2048
    probe = api.Server(tab, hbm_budget_bytes=64 << 20, staging_bytes=16 << 20)
    try:
        one = probe.request_bytes(s, n, len(dirs))
    finally:
        probe.close()
    say("server arena of exactly 3 events", 3 * one)
    sv = api.Server(tab, hbm_budget_bytes=3 * one, staging_bytes=64 << 20, n_streams=2, max_batch_events=4,
                    tick_s=0.05)
    try:
        vs = [S.traces(s, n, cfg=3, event=400 + i, dtype=np.float32) for i in range(4)]
        tks = [sv.submit(v, dirs) for v in vs]
        res = [sv.wait(tk, timeout_s=30) for tk in tks[:3]]
        assert all(r.batch_events == 3 and r.batch_id == res[0].batch_id for r in res)
        st = sv.stats()
        assert st["arena_peak"] == 3 * one and st["queued"] == 1
        outs = [sv.result(tk) for tk in tks[:3]]
        sv.release(tks[0])
        r4 = sv.wait(tks[3], timeout_s=30)
        assert r4.t_admit >= res[0].t_complete
        outs.append(sv.result(tks[3]))
        for tk in tks[1:]:
            sv.release(tk)
        ev = api.make_event(s, n, prec=api.AU_PREC_FP32, trace_dtype=api.AU_F32)
        import torch
        for v, o in zip(vs, outs):
            plain = api.unfold_direction_scan(tab, ev, torch.from_numpy(v).cuda(), dirs).cpu().numpy()
            assert np.array_equal(o, plain)
    finally:
        sv.close()


def test_fifo_admission_under_a_small_budget(api, fine32):
    t, tab = fine32
    dirs = S.direction_grid(2, 2)
    s, n = 40, 4096
    one = event_bytes(s, n, len(dirs))
    budget = int(one * 1.6) + (4 << 20)       # room for one event at a time
    say("server budget", budget)
    sv = api.Server(tab, hbm_budget_bytes=budget, staging_bytes=256 << 20, n_streams=2, max_batch_events=4)
    try:
        vs = [S.traces(s, n, cfg=3, event=200 + i, dtype=np.float32) for i in range(4)]
        tks = [sv.submit(v, dirs) for v in vs]
        res = []
        for tk in tks:                                   # release in order so the next can be admitted
            res.append(sv.wait(tk, timeout_s=30))
            sv.release(tk)
        for a, b in zip(res, res[1:]):
            assert b.t_admit >= a.t_complete - 1e-3      # never two admitted at once
        st = sv.stats()
        assert st["arena_peak"] <= budget and st["completed"] == 4
    finally:
        sv.close()


def test_fp64_server_matches_plain_path(api):
    import torch
    g = S.GRID_COARSE
    t = S.pattern_table(g, cfg=1)
    tab = api.Table(g, t)
    dirs = S.direction_grid(3, 3)
    v = S.traces(11, 2048, cfg=3, event=300)
    say("server fp64")
    sv = api.Server(tab, hbm_budget_bytes=1 << 30, staging_bytes=64 << 20, prec=api.AU_PREC_FP64,
                    trace_dtype=api.AU_F64)
    try:
        tk = sv.submit(v, dirs)
        sv.wait(tk)
        got = sv.result(tk)
        ev = api.make_event(11, 2048)
        plain = api.unfold_direction_scan(tab, ev, torch.from_numpy(v).cuda(), dirs).cpu().numpy()
        assert np.array_equal(got, plain)
        ref, _, _ = oracle_unfold(g, t, v, dirs)
        assert_traces_close(got, ref, TOL_FP64, "served fp64")
        sv.release(tk)
    finally:
        sv.close()


def test_server_errors_and_lifecycle(api, fine32):
    t, tab = fine32
    say("server errors")
    sv = api.Server(tab, hbm_budget_bytes=64 << 20, staging_bytes=32 << 20)
    try:
        with pytest.raises(api.AuError) as e:
            sv.submit(np.zeros((3, 2, 3000), np.float32), [[10.0, 10.0]])
        assert e.value.status == api.AU_EINVAL
        with pytest.raises(api.AuError) as e:                       # larger than the whole arena
            sv.submit(np.zeros((124, 2, 4096), np.float32), S.direction_grid(8, 8))
        assert e.value.status == api.AU_ENOMEM
        with pytest.raises(api.AuError) as e:
            sv.poll(987654)
        assert e.value.status == api.AU_ENOTFOUND
        tk = sv.submit(np.zeros((3, 2, 2048), np.float32), [[10.0, 10.0]])
        sv.release(tk)                                              # before or after completion: fine
        with pytest.raises(api.AuError) as e:
            sv.release(tk)
        assert e.value.status == api.AU_ENOTFOUND
        time.sleep(0.05)
        tk2 = sv.submit(np.ones((3, 2, 2048), np.float32), [[10.0, 10.0]])
        sv.wait(tk2)
        sv.release(tk2)
        st = sv.stats()
        assert st["arena_in_use"] == 0 and st["in_flight"] == 0
    finally:
        sv.close()
