"""au_unfold_direction_scan_noalloc (the direction scan whose work space is a
fixed device array of the library) against au_unfold_direction_scan (work
space from the caller): the same kernels, so the outputs and counters must be
bitwise equal.  Two calls in a row, the second with a smaller event (fewer
stations, shorter traces, fewer directions), so the second reads only what it
wrote over the first's leftovers; then a direction count whose coefficients
exceed the array (processed in chunks), FP64, and the size limit."""
import numpy as np
import pytest

from paper_1507_07733_amd import synth as S

from helpers import TOL_FP32, TOL_FP64, assert_close, oracle_unfold

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


def run_both(api, tab, ev, v, dirs):
    import torch
    dv = torch.from_numpy(v).cuda()
    dd = torch.from_numpy(np.ascontiguousarray(dirs, dtype=np.float64)).cuda()
    out = torch.full((len(dirs), ev.n_stations, 2, ev.n_samples), float("nan"),
                     dtype=api.out_dtype(ev.prec), device="cuda")
    c_na = torch.zeros(2, dtype=torch.int64, device="cuda")
    api.unfold_direction_scan_noalloc(tab, ev, dv, dd, out, counts=c_na)
    c_ws = torch.zeros(2, dtype=torch.int64, device="cuda")
    ref = api.unfold_direction_scan(tab, ev, dv, dirs, counts=c_ws)
    torch.cuda.synchronize()
    return out.cpu().numpy(), ref.cpu().numpy(), c_na.cpu().tolist(), c_ws.cpu().tolist()


def test_noalloc_matches_workspace_path_twice(api):
    g = S.GRID_FINE
    t32 = S.pattern_table(g, cfg=2).astype(np.complex64)
    tab = api.Table(g, t32)
    for s, n, dirs in ((40, 4096, S.direction_grid(4, 6)), (7, 2048, S.direction_grid(2, 3))):
        ev = api.make_event(s, n, prec=api.AU_PREC_FP32, trace_dtype=api.AU_F32)
        v = S.traces(s, n, cfg=2, event=s, dtype=np.float32)
        say("noalloc fp32 S", s, "N", n, "D", len(dirs))
        got, ref, c_na, c_ws = run_both(api, tab, ev, v, dirs)
        assert np.array_equal(got, ref)
        assert c_na == c_ws
        units = np.array([[0, 0], [len(dirs) - 1, s - 1], [1, s // 2]])
        o = oracle_unfold(g, t32, v, dirs, units=units)[0]
        assert_close(np.stack([got[d, st] for d, st in units]), o, True, "noalloc fp32")


def test_noalloc_direction_chunks_and_fp64(api):
    # 1 000 stations x 4096 FP64: spectra 31.25 MiB, 64 KiB of coefficients per direction, so 30
    # directions take three chunks (12, 12, 6) of the 32 MiB array
    g = S.GRID_COARSE
    t = S.pattern_table(g, cfg=1)
    tab = api.Table(g, t)
    s, n = 1000, 4096
    dirs = S.direction_grid(5, 6)
    ev = api.make_event(s, n)
    v = S.traces(s, n, cfg=1, event=9)
    say("noalloc fp64 S 1000 N 4096 D 30 (three chunks)")
    got, ref, c_na, c_ws = run_both(api, tab, ev, v, dirs)
    assert np.array_equal(got, ref)
    assert c_na == c_ws
    units = np.array([[0, 0], [11, 777], [12, 3], [29, 999]])
    o = oracle_unfold(g, t, v, dirs, units=units)[0]
    assert_close(np.stack([got[d, st] for d, st in units]), o, False, "noalloc fp64 chunks")
    del got, ref
    # a second, smaller call after the large one
    s2, n2, d2 = 5, 1024, S.direction_grid(3, 3)
    ev2 = api.make_event(s2, n2)
    v2 = S.traces(s2, n2, cfg=1, event=10)
    say("noalloc fp64 after the large call: S 5 N 1024 D 9")
    got2, ref2, _, _ = run_both(api, tab, ev2, v2, d2)
    assert np.array_equal(got2, ref2)


def test_noalloc_rejects_oversized_events(api):
    import torch
    g = S.GRID_COARSE
    tab = api.Table(g, S.pattern_table(g, cfg=1))
    s, n = 1100, 4096                      # 1 100 x 1 024 x 32 B of FP64 spectra > 32 MiB
    ev = api.make_event(s, n)
    v = torch.zeros((s, 2, n), dtype=torch.float64, device="cuda")
    dd = torch.zeros((1, 2), dtype=torch.float64, device="cuda")
    out = torch.zeros((1, s, 2, n), dtype=torch.float64, device="cuda")
    say("noalloc oversized event rejected")
    with pytest.raises(api.AuError) as e:
        api.unfold_direction_scan_noalloc(tab, ev, v, dd, out)
    assert e.value.status == api.AU_EINVAL and "32 MiB" in str(e.value)
    assert not torch.any(out)
