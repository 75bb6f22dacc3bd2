"""GPU parity of the HIP path against the CPU oracle, through the C ABI.

Each test prints the case it is about to run before touching the GPU.
"""
import numpy as np
import pytest

from oracle import oracle as O
from paper_1507_07733_amd import synth as S

from helpers import TOL_FP32, TOL_FP64, assert_close, assert_fp32_close, assert_traces_close, oracle_unfold, trace_errors

pytestmark = pytest.mark.gpu

G = S.GRID_COARSE
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
def coarse(api):
    t = S.pattern_table(G, cfg=0)
    return t, api.Table(G, t)


@pytest.fixture(scope="module")
def coarse_c64(api):
    t = S.pattern_table(G, cfg=0).astype(np.complex64)
    return t, api.Table(G, t)


@pytest.fixture(scope="module")
def identity(api):
    t = S.identity_table(G)
    return t, api.Table(G, t)


def to_dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


@pytest.mark.parametrize("n", [16, 32, 64, 128, 256, 512, 1024, 2048, 4096])
@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_identity_pattern_bandpass_every_size(api, identity, n, prec):
    t, tab = identity
    s = 3 if n < 1024 else 5
    p = api.AU_PREC_FP64 if prec == "fp64" else api.AU_PREC_FP32
    dt = np.float64 if prec == "fp64" else np.float32
    v = S.traces(s, n, cfg=0, event=1000 + n, dtype=dt)
    ev = api.make_event(s, n, prec=p, trace_dtype=api.AU_F64 if dt == np.float64 else api.AU_F32)
    say("identity", prec, "S", s, "N", n)
    out = api.unfold_event(tab, ev, to_dev(v), 33.0, 71.0)
    import torch
    torch.cuda.synchronize()
    ref, _, _ = oracle_unfold(G, t, v, [[33.0, 71.0]])
    assert_close(out.cpu().numpy(), ref[0], prec == "fp32", "identity")


def test_single_event_fp64_config0(api, coarse):
    # 10 stations x 2 channels x 2048 float64 samples, one direction (40, 120) deg
    t, tab = coarse
    v = S.traces(10, 2048, cfg=0, event=0)
    ev = api.make_event(10, 2048)
    say("cfg0 fp64 unfold_event")
    out = api.unfold_event(tab, ev, to_dev(v), 40.0, 120.0).cpu().numpy()
    ref, sing, _ = oracle_unfold(G, t, v, [[40.0, 120.0]])
    r = assert_traces_close(out, ref[0], TOL_FP64, "cfg0")
    assert np.all(sing == 0)
    print("max r", r.max())


@pytest.mark.parametrize("n,s", [(4096, 7), (2048, 13), (1024, 3)])
def test_direction_scan_fp64(api, coarse, n, s):
    t, tab = coarse
    v = S.traces(s, n, cfg=1, event=n + s)
    dirs = np.concatenate([S.direction_grid(4, 6), [[0.0, 0.0], [89.0, 359.999], [12.5, -30.0]]])
    ev = api.make_event(s, n)
    import torch
    counts = torch.zeros(2, dtype=torch.int64, device="cuda")
    say("scan fp64 N", n, "S", s, "D", len(dirs))
    out = api.unfold_direction_scan(tab, ev, to_dev(v), dirs, counts=counts).cpu().numpy()
    ref, sing, _ = oracle_unfold(G, t, v, dirs)
    assert_traces_close(out, ref, TOL_FP64, "scan")
    assert counts.cpu().tolist() == [0, 0]


def test_horizon_singular_counts(api, coarse):
    t, tab = coarse
    n, s = 2048, 4
    v = S.traces(s, n, cfg=1, event=5)
    dirs = np.array([[90.0, 10.0], [90.0, 200.0], [45.0, 10.0]])
    import torch
    for prec in (api.AU_PREC_FP64, api.AU_PREC_FP32):
        ev = api.make_event(s, n, prec=prec)
        counts = torch.zeros(2, dtype=torch.int64, device="cuda")
        say("horizon prec", prec)
        out = api.unfold_direction_scan(tab, ev, to_dev(v), dirs, counts=counts).cpu().numpy()
        nb = api.band_bins(ev)[1]
        c = counts.cpu().tolist()
        assert c[1] == 2 * nb
        if prec == api.AU_PREC_FP32:
            assert c[0] >= 2 * nb
        assert np.all(out[:2] == 0)
        assert np.max(np.abs(out[2])) > 0


@pytest.mark.parametrize("n", [2048, 4096])
def test_fp32_path_against_fp64_oracle(api, n):
    # fine grid, complex64 table, float32 traces: the oracle runs on the same
    # float32 values promoted to float64
    t64 = S.pattern_table(GF, cfg=2)
    t32 = t64.astype(np.complex64)
    tab = api.Table(GF, t32)
    s = 6
    v = S.traces(s, n, cfg=2, event=n, dtype=np.float32)
    dirs = np.concatenate([S.direction_grid(4, 4), [[0.5, 359.5], [87.0, 0.0]]])
    ev = api.make_event(s, n, prec=api.AU_PREC_FP32, trace_dtype=api.AU_F32)
    say("fp32 fine N", n)
    out = api.unfold_direction_scan(tab, ev, to_dev(v), dirs).cpu().numpy()
    ref, _, _ = oracle_unfold(GF, t32, v, dirs)
    rs, r = assert_fp32_close(out, ref, TOL_FP32, "fp32")
    print("fp32 max r per station %.3e per component %.3e median %.3e" % (rs.max(), r.max(), np.median(r)))


def corner_max(grid, table, k, n, zen, az):
    """max |table| over the 8 interpolation corners of bin k (test-local cell math)."""
    num = k * S.FS_HZ - grid.f0_hz * n
    den = n * grid.df_hz
    fi = min(num // den, grid.n_freq - 2)
    v = min(max((zen - grid.zen0_deg) / grid.dzen_deg, 0.0), grid.n_zen - 1)
    zi = min(int(np.floor(v)), grid.n_zen - 2)
    w = ((az - grid.az0_deg) % 360.0) / grid.daz_deg
    ai = int(np.floor(w)) % grid.n_az
    aj = (ai + 1) % grid.n_az
    sub = table[:, :, fi:fi + 2, zi:zi + 2][..., [ai, aj]]
    return np.max(np.abs(sub))


def test_pattern_response_fp64_and_fp32_bound(api, coarse, coarse_c64):
    dirs = np.array([[40.0, 120.0], [17.3, 358.2], [88.8, 3.1], [0.0, 0.0], [63.0, 181.0]])
    n = 2048
    for prec, (t, tab) in ((api.AU_PREC_FP64, coarse), (api.AU_PREC_FP32, coarse_c64)):
        ev = api.make_event(4, n, prec=prec)
        say("pattern_response prec", prec)
        h = api.pattern_response(tab, ev, dirs).cpu().numpy()
        k_lo, nb = api.band_bins(ev)
        worst = 0.0
        for di, (z, a) in enumerate(dirs):
            for j in range(0, nb, 7):
                k = k_lo + j
                ref = O.pattern_at_bin(G, t.astype(np.complex128), k, n, S.FS_HZ, z, a)
                err = np.max(np.abs(h[di, j] - ref))
                if prec == api.AU_PREC_FP64:
                    assert err <= 1e-15 * max(np.max(np.abs(ref)), 1e-300) * 8
                else:
                    # the paper's single-precision bound: 7 lerps x 6 operations x 2^-24
                    bound = 42 * 2.0 ** -24 * corner_max(G, t, k, n, z, a)
                    worst = max(worst, err / bound)
                    assert err <= bound, (di, j, err, bound)
        print("fp32 interp: worst err / bound = %.3f" % worst)


def test_pattern_response_texture_weights(api, coarse, coarse_c64):
    """Interpolation with weights rounded to 8 fractional bits (a texture filter's fixed point): GPU
    equals the oracle's quantized interpolation (FP64 to rounding, FP32 within the FP32 bound), and
    the precision cost against exact weights is reported."""
    r = np.random.default_rng(11)
    dirs = np.stack([r.uniform(0, 89.9, 24), r.uniform(0, 360, 24)], 1)
    n = 2048
    rel_cost = []
    for prec, (t, tab) in ((api.AU_PREC_FP64, coarse), (api.AU_PREC_FP32, coarse_c64)):
        ev = api.make_event(4, n, prec=prec)
        say("pattern_response_quantized prec", prec)
        hq = api.pattern_response(tab, ev, dirs, weight_bits=8).cpu().numpy()
        k_lo, nb = api.band_bins(ev)
        t128 = t.astype(np.complex128)
        for di, (z, a) in enumerate(dirs):
            for j in range(0, nb, 5):
                k = k_lo + j
                ref = O.pattern_at_bin_quantized(G, t128, k, n, S.FS_HZ, z, a, 8)
                err = np.max(np.abs(hq[di, j] - ref))
                cm = corner_max(G, t, k, n, z, a)
                if prec == api.AU_PREC_FP64:
                    assert err <= 8e-16 * cm
                    exact = O.pattern_at_bin(G, t128, k, n, S.FS_HZ, z, a)
                    big = np.abs(exact) > 0.1 * cm
                    rel_cost.extend((np.abs(ref - exact)[big] / np.abs(exact)[big]).tolist())
                else:
                    assert err <= 42 * 2.0 ** -24 * cm, (di, j, err)
    rel_cost = np.array(rel_cost)
    print("8-bit weights vs exact: median %.2e, p99 %.2e, max %.2e relative (entries above 10%% of the corner max)"
          % (np.median(rel_cost), np.percentile(rel_cost, 99), rel_cost.max()))
    assert rel_cost.max() < 0.05


@pytest.mark.parametrize("flags", [0, 1, 2, 3, 4, 6, 7])
def test_batch_plan_uneven_events(api, coarse, flags):
    import torch
    t, tab = coarse
    specs = [(3, 2048, S.direction_grid(2, 3)), (17, 4096, S.direction_grid(1, 4)),
             (9, 1024, S.direction_grid(3, 1)), (1, 2048, [[45.0, 45.0]]), (12, 4096, [[10.0, 300.0], [80.0, 0.0]])]
    say("batch fp64 flags", flags)
    plan = api.Plan(tab, specs, prec=api.AU_PREC_FP64, trace_dtype=api.AU_F64, flags=flags)
    volt = np.zeros(plan.volt_elems)
    vs = []
    for e, (s, n, _) in enumerate(specs):
        v = S.traces(s, n, cfg=2, event=50 + e)
        vs.append(v)
        o = plan.volt_offsets[e]
        volt[o:o + v.size] = v.ravel()
    dv = to_dev(volt)
    out = torch.full((plan.efield_elems,), float("nan"), dtype=torch.float64, device="cuda")
    counts = torch.zeros(2, dtype=torch.int64, device="cuda")
    plan.run(dv, out, counts)
    plan.run(dv, out, counts)            # a second run (graph replay when captured)
    torch.cuda.synchronize()
    for e, (s, n, d) in enumerate(specs):
        got = plan.event_output(out, e).cpu().numpy()
        ref, _, _ = oracle_unfold(G, t, vs[e], d)
        assert_traces_close(got, ref, TOL_FP64, "batch event %d" % e)
    assert plan.station_unfolds == sum(s * len(d) for s, _, d in specs)


# the default band (spectra by the streaming kernel) and one wider than N/4 bins (by the
# one-station-per-workgroup kernel): plan and plain scan take the same kernel either way
@pytest.mark.parametrize("band", [(30_000_000, 80_000_000), (1_000_000, 99_000_000)], ids=["30-80", "1-99"])
def test_batch_plan_fp32_matches_plain_fp32(api, band):
    import torch
    lo, hi = band
    t32 = S.pattern_table(GF, cfg=2).astype(np.complex64)
    tab = api.Table(GF, t32)
    specs = [(5, 2048, S.direction_grid(2, 2)), (11, 4096, S.direction_grid(2, 1)), (4, 2048, [[30.0, 30.0]])]
    say("batch fp32 graph+persistent vs plain, band", lo, hi)
    plan = api.Plan(tab, specs, prec=api.AU_PREC_FP32, trace_dtype=api.AU_F32, flags=3, band_lo_hz=lo, band_hi_hz=hi)
    volt = np.zeros(plan.volt_elems, dtype=np.float32)
    vs = []
    for e, (s, n, _) in enumerate(specs):
        v = S.traces(s, n, cfg=2, event=80 + e, dtype=np.float32)
        vs.append(v)
        volt[plan.volt_offsets[e]:plan.volt_offsets[e] + v.size] = v.ravel()
    out = torch.zeros(plan.efield_elems, dtype=torch.float32, device="cuda")
    plan.run(to_dev(volt), out)
    torch.cuda.synchronize()
    for e, (s, n, d) in enumerate(specs):
        got = plan.event_output(out, e).cpu().numpy()
        ev = api.make_event(s, n, prec=api.AU_PREC_FP32, trace_dtype=api.AU_F32, band_lo_hz=lo, band_hi_hz=hi)
        plain = api.unfold_direction_scan(tab, ev, to_dev(vs[e]), d).cpu().numpy()
        # same kernels, same per-unit arithmetic: bitwise equal whatever the batch mix
        assert np.array_equal(got, plain)
        ref = O.unfold(GF, t32.astype(np.complex128), vs[e].astype(np.float64), np.asarray(d, dtype=np.float64),
                       S.FS_HZ, lo, hi)[0]
        assert_fp32_close(got, ref, TOL_FP32, "batch fp32 event %d" % e)


def test_workspace_argument_and_errors(api, coarse):
    import torch
    t, tab = coarse
    ev = api.make_event(4, 2048)
    v = to_dev(S.traces(4, 2048, cfg=0, event=3))
    need = api.workspace_bytes(tab, ev, 3)
    work = torch.empty(need, dtype=torch.uint8, device="cuda")
    dirs = [[10.0, 10.0], [20.0, 20.0], [30.0, 30.0]]
    say("workspace given")
    a = api.unfold_direction_scan(tab, ev, v, dirs, work=work)
    b = api.unfold_direction_scan(tab, ev, v, dirs)
    assert torch.equal(a, b)
    small = torch.empty(need - 256, dtype=torch.uint8, device="cuda")
    with pytest.raises(api.AuError) as ei:
        api.unfold_direction_scan(tab, ev, v, dirs, work=small)
    assert ei.value.status == api.AU_ENOMEM
    bad = api.make_event(4, 3000)
    with pytest.raises(api.AuError) as ei:
        api.workspace_bytes(tab, bad, 1)
    assert ei.value.status == api.AU_EINVAL
    nyq = api.make_event(4, 2048, band_lo_hz=60_000_000, band_hi_hz=S.FS_HZ // 2)
    with pytest.raises(api.AuError) as ei:
        api.workspace_bytes(tab, nyq, 1)         # the Nyquist bin never enters a band
    assert ei.value.status == api.AU_EINVAL
    ev32 = api.make_event(4, 2048, prec=api.AU_PREC_FP64)
    t32 = api.Table(G, t.astype(np.complex64))
    with pytest.raises(api.AuError):
        api.workspace_bytes(t32, ev32, 1)        # FP64 needs a complex128 table


@pytest.mark.parametrize("n", [1024, 2048, 4096])
@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_every_unfold_variant(api, coarse, n, prec):
    t, tab = coarse
    p = api.AU_PREC_FP64 if prec == "fp64" else api.AU_PREC_FP32
    s = 5
    v = S.traces(s, n, cfg=3, event=n)
    dirs = np.array([[40.0, 120.0], [72.5, 359.0], [5.0, 3.0]])
    ev = api.make_event(s, n, prec=p)
    ref, _, _ = oracle_unfold(G, t, v, dirs)
    keep = api.get_unfold_variant(p, n)
    built = 0
    try:
        for vi, (e, rmax, twmode, wave, pair, pp) in enumerate(api.unfold_variants()):
            try:
                api.set_unfold_variant(p, n, vi)
            except api.AuError:
                continue                      # not built for this size / precision
            built += 1
            say("variant", vi, "E", e, "rmax", rmax, "twmode", twmode, "wave", wave, "pair", pair, "pp", pp, prec, "N", n)
            out = api.unfold_direction_scan(tab, ev, to_dev(v), dirs).cpu().numpy()
            assert_close(out, ref, prec == "fp32", "variant %d" % vi)
    finally:
        api.set_unfold_variant(p, n, keep)
    assert built >= 4


# (name, lo_hz, hi_hz, table): a band from DC with the identity table and offset traces (the DC bin
# carries signal), one wider than two bins per thread at 4 096 samples, one bin, and a band narrower
# than the threads of a transform (most threads hold no bin)
VARIANT_BANDS = [("dc", 0, 40_000_000, "identity"), ("wide", 1_000_000, 99_000_000, "pattern"),
                 ("one_bin", 50_000_000, 50_000_000, "pattern"), ("narrow", 61_000_000, 64_000_000, "pattern")]


@pytest.mark.parametrize("band", VARIANT_BANDS, ids=[b[0] for b in VARIANT_BANDS])
@pytest.mark.parametrize("n", [2048, 4096])
@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_every_unfold_variant_band_edges(api, coarse, identity, band, n, prec):
    """Every built shape on bands where the bins a thread solves change: the paired-lane shapes
    place bin k in register k / TT of thread k mod TT and its mirror in the partner lane."""
    name, lo, hi, table = band
    t, tab = identity if table == "identity" else coarse
    p = api.AU_PREC_FP64 if prec == "fp64" else api.AU_PREC_FP32
    dt = np.float64 if prec == "fp64" else np.float32
    s = 3
    v = S.traces(s, n, cfg=3, event=n + 1, dtype=dt)
    if name == "dc":
        v = (v + dt(2.5)).astype(dt)
    dirs = np.array([[40.0, 120.0], [5.0, 3.0]])
    ev = api.make_event(s, n, prec=p, trace_dtype=api.AU_F64 if prec == "fp64" else api.AU_F32, band_lo_hz=lo,
                        band_hi_hz=hi)
    ref, _, _ = O.unfold(G, np.asarray(t).astype(np.complex128), v.astype(np.float64), dirs, S.FS_HZ, lo, hi)
    if name == "dc":
        assert np.abs(ref.mean(axis=-1)).min() > 1.0
    keep = api.get_unfold_variant(p, n)
    built = 0
    try:
        for vi, (e, rmax, twmode, wave, pair, pp) in enumerate(api.unfold_variants()):
            try:
                api.set_unfold_variant(p, n, vi)
            except api.AuError:
                continue
            built += 1
            say("variant", vi, "pair", pair, "pp", pp, "band", name, prec, "N", n)
            out = api.unfold_direction_scan(tab, ev, to_dev(v), dirs).cpu().numpy()
            assert_close(out, ref, prec == "fp32", "variant %d band %s" % (vi, name))
    finally:
        api.set_unfold_variant(p, n, keep)
    assert built >= 4


def test_autotune_selects_a_built_variant(api, coarse):
    t, tab = coarse
    ev = api.make_event(16, 2048, prec=api.AU_PREC_FP64)
    say("autotune fp64 2048")
    best, ms = api.autotune(tab, ev, n_dir=4, reps=1)
    assert ms[best] > 0 and ms[best] == min(m for m in ms if m > 0)
    assert api.get_unfold_variant(api.AU_PREC_FP64, 2048) == best


@pytest.mark.parametrize("flags", [3, 6])
def test_plan_autotune_keeps_results(api, flags):
    """In-plan tuning picks a built variant per class, leaves the global choice alone, and the
    tuned plan (graph re-captured when flags has AU_PLAN_GRAPH) still meets the FP32 bar."""
    import torch
    t32 = S.pattern_table(GF, cfg=2).astype(np.complex64)
    tab = api.Table(GF, t32)
    specs = [(13, 4096, S.direction_grid(2, 2)), (7, 2048, S.direction_grid(3, 1)), (3, 1024, [[30.0, 30.0]])]
    say("plan autotune flags", flags)
    plan = api.Plan(tab, specs, prec=api.AU_PREC_FP32, trace_dtype=api.AU_F32, flags=flags)
    volt = np.zeros(plan.volt_elems, dtype=np.float32)
    vs = []
    for e, (s, n, _) in enumerate(specs):
        v = S.traces(s, n, cfg=2, event=90 + e, dtype=np.float32)
        vs.append(v)
        volt[plan.volt_offsets[e]:plan.volt_offsets[e] + v.size] = v.ravel()
    dv = to_dev(volt)
    out = torch.zeros(plan.efield_elems, dtype=torch.float32, device="cuda")
    plan.run(dv, out)                                   # captures the graph with the default variants
    before = {n: api.get_unfold_variant(api.AU_PREC_FP32, n) for n in (1024, 2048, 4096)}
    res = plan.autotune(dv, out, reps=1)
    assert [r[0] for r in res] == [4096, 2048, 1024]
    for (n, best, ms), (n2, _, var) in zip(res, plan.classes()):
        assert n == n2 and var == best
        assert ms[best] > 0 and ms[best] == min(m for m in ms if m > 0)
    assert before == {n: api.get_unfold_variant(api.AU_PREC_FP32, n) for n in (1024, 2048, 4096)}
    out.fill_(float("nan"))
    plan.run(dv, out)
    plan.run(dv, out)
    torch.cuda.synchronize()
    for e, (s, n, d) in enumerate(specs):
        ref, _, _ = oracle_unfold(GF, t32, vs[e], d)
        assert_fp32_close(plan.event_output(out, e).cpu().numpy(), ref, TOL_FP32, "tuned plan event %d" % e)
