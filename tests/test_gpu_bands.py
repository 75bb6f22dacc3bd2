"""GPU parity of the unfolding for bands other than 30-80 MHz, against the oracle run with the
same band, for every built unfold variant: a band that includes DC (only the real part of the
DC bin is kept, both sides), a band wider than the bins each thread prefetches (so the staging
also takes its fallback loop), a one-bin band and an empty band (zero output).  The envelope
peaks get the DC and wide bands too."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_1507_07733_amd import synth as S

from helpers import TOL_FP32, TOL_FP64, assert_close

pytestmark = pytest.mark.gpu

G = S.GRID_COARSE

# (name, lo_hz, hi_hz): hi < fs/2 = 100 MHz; the coarse table covers 0-100 MHz
BANDS = [
    ("dc", 0, 30_000_000),
    ("wide", 1_000_000, 99_000_000),
    ("one_bin", 50_000_000, 50_000_000),
    ("empty", 50_000_001, 50_000_002),
]


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
    return t, api.Table(G, t), api.Table(G, t.astype(np.complex64))


@pytest.fixture(scope="module")
def identity(api):
    # the synthetic pattern vanishes at 0 Hz (its DC bin is singular); the identity
    # pattern keeps the DC bin, so the real-part rule is exercised
    t = S.identity_table(G)
    return t, api.Table(G, t), api.Table(G, t.astype(np.complex64))


def oracle_band(t, v, dirs, lo, hi):
    return O.unfold(G, t.astype(np.complex128), np.asarray(v, dtype=np.float64), dirs, S.FS_HZ, lo, hi)[0]


CASES = [b + ("pattern",) for b in BANDS] + [("dc", 0, 30_000_000, "identity")]


@pytest.mark.parametrize("n", [2048, 4096])
@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("case", CASES, ids=["%s-%s" % (c[0], c[3]) for c in CASES])
def test_band_every_variant(api, coarse, identity, case, prec, n):
    import torch
    name, lo, hi, table = case
    t, tab64, tab32 = coarse if table == "pattern" else identity
    p = api.AU_PREC_FP64 if prec == "fp64" else api.AU_PREC_FP32
    tab = tab64 if prec == "fp64" else tab32
    tref = t if prec == "fp64" else t.astype(np.complex64)
    s = 4
    dt = np.float64 if prec == "fp64" else np.float32
    v = S.traces(s, n, cfg=3, event=n + len(name), dtype=dt)
    dirs = np.array([[40.0, 120.0], [72.5, 359.0], [5.0, 3.0]])
    ev = api.make_event(s, n, prec=p, trace_dtype=api.AU_F64 if prec == "fp64" else api.AU_F32,
                        band_lo_hz=lo, band_hi_hz=hi)
    k_lo, nb = api.band_bins(ev)
    if name == "dc":
        assert k_lo == 0 and nb > 1
    elif name == "wide":
        assert nb > n // 4              # more bins than a thread group prefetches
    elif name == "one_bin":
        assert nb == 1
    else:
        assert nb == 0
    ref = oracle_band(tref, v, dirs, lo, hi)
    if nb == 0:
        assert not np.any(ref)
    if table == "identity":
        assert np.any(np.abs(ref.mean(axis=-1)) > 1e-3)   # the DC bin carries signal
    keep = api.get_unfold_variant(p, n)
    built = 0
    try:
        for vi, shape in enumerate(api.unfold_variants()):
            try:
                api.set_unfold_variant(p, n, vi)
            except api.AuError:
                continue
            built += 1
            say("band", name, table, prec, "N", n, "variant", vi, shape)
            out = api.unfold_direction_scan(tab, ev, torch.from_numpy(v).cuda(), dirs).cpu().numpy()
            if nb == 0:
                assert not np.any(out), "empty band must give zero traces"
            else:
                assert_close(out, ref, prec == "fp32", "band %s variant %d" % (name, vi))
    finally:
        api.set_unfold_variant(p, n, keep)
    assert built >= 4


ENV_CASES = [BANDS[0] + ("pattern",), BANDS[1] + ("pattern",), ("dc", 0, 30_000_000, "identity")]


@pytest.mark.parametrize("case", ENV_CASES, ids=["%s-%s" % (c[0], c[3]) for c in ENV_CASES])
@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_band_envelope_peaks(api, coarse, identity, case, prec):
    import torch
    from test_gpu_envelope import check_peaks
    name, lo, hi, table = case
    t, tab64, tab32 = coarse if table == "pattern" else identity
    n, s = 4096, 5
    p = api.AU_PREC_FP64 if prec == "fp64" else api.AU_PREC_FP32
    tab = tab64 if prec == "fp64" else tab32
    tref = t if prec == "fp64" else t.astype(np.complex64)
    dt = np.float64 if prec == "fp64" else np.float32
    v = S.traces(s, n, cfg=4, event=31, dtype=dt)
    dirs = np.array([[40.0, 120.0], [70.0, 355.0], [12.0, 200.0]])
    ev = api.make_event(s, n, prec=p, trace_dtype=api.AU_F64 if prec == "fp64" else api.AU_F32,
                        band_lo_hz=lo, band_hi_hz=hi)
    say("band envelope", name, table, prec)
    peak, arg, _ = api.unfold_envelope_scan(tab, ev, torch.from_numpy(v).cuda(), dirs)
    ref = oracle_band(tref, v, dirs, lo, hi)
    frac = check_peaks(peak.cpu().numpy(), arg.cpu().numpy(), ref, TOL_FP64 if prec == "fp64" else TOL_FP32)
    assert frac > 0.9


# 0-100 MHz in 0.1 MHz steps: the 30-80 MHz band spans about 500 frequency nodes and the
# 1-99 MHz band about 980, more than the coefficient kernel's angular slice holds in LDS at
# once (256 nodes), so it takes the band in windows of nodes; every window boundary is crossed.
GRID_DENSE_F = S.Grid(1001, 10, 36, 0, 100_000, 0.0, 10.0, 0.0, 10.0)


@pytest.mark.parametrize("band", [(30_000_000, 80_000_000), (1_000_000, 99_000_000)], ids=["30-80", "1-99"])
@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_dense_frequency_grid_windows(api, prec, band):
    import torch
    lo, hi = band
    g = GRID_DENSE_F
    t = S.pattern_table(g, cfg=1)
    p = api.AU_PREC_FP64 if prec == "fp64" else api.AU_PREC_FP32
    tref = t if prec == "fp64" else t.astype(np.complex64)
    tab = api.Table(g, tref)
    n, s = 2048, 3
    dt = np.float64 if prec == "fp64" else np.float32
    v = S.traces(s, n, cfg=3, event=77, dtype=dt)
    dirs = np.array([[40.0, 120.0], [72.5, 355.0], [3.0, 8.0]])
    ev = api.make_event(s, n, prec=p, trace_dtype=api.AU_F64 if prec == "fp64" else api.AU_F32,
                        band_lo_hz=lo, band_hi_hz=hi)
    k_lo, nb = api.band_bins(ev)
    nodes = (k_lo + nb - 1) * S.FS_HZ // (n * g.df_hz) - k_lo * S.FS_HZ // (n * g.df_hz) + 2
    assert nodes > 256
    say("dense frequency grid", prec, "band", lo, hi, "nodes", nodes)
    out = api.unfold_direction_scan(tab, ev, torch.from_numpy(v).cuda(), dirs).cpu().numpy()
    ref = O.unfold(g, tref.astype(np.complex128), np.asarray(v, dtype=np.float64), dirs, S.FS_HZ, lo, hi)[0]
    assert_close(out, ref, prec == "fp32", "dense grid %s" % prec)
    # the interpolated pattern itself, at every bin (pattern-response mode of the same kernel)
    from test_gpu_parity import corner_max
    h = api.pattern_response(tab, ev, dirs).cpu().numpy()
    t128 = tref.astype(np.complex128)
    for di, (z, a) in enumerate(dirs):
        for j in range(nb):
            ref_h = O.pattern_at_bin(g, t128, k_lo + j, n, S.FS_HZ, z, a)
            err = np.max(np.abs(h[di, j] - ref_h))
            if prec == "fp64":
                assert err <= 8e-15 * max(np.max(np.abs(ref_h)), 1e-300), (di, j, err)
            else:
                # 7 lerps x 6 operations x 2^-24 of the largest corner, as for the coarse grid
                assert err <= 42 * 2.0 ** -24 * corner_max(g, t128, k_lo + j, n, z, a), (di, j, err)
