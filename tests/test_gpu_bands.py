"""GPU parity of the unfolding for bands other than 30-80 MHz, against the oracle run with the
same band, for every built unfold variant: a band that includes DC (only the real part of the
DC bin is kept, both sides), a band wider than the bins each thread prefetches (so the staging
also takes its fallback loop), a one-bin band and an empty band (zero output).  The envelope
peaks get the DC and wide bands too."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_1507_07733_amd import synth as S

from helpers import TOL_FP32, TOL_FP64, assert_traces_close

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
                assert_traces_close(out, ref, TOL_FP64 if prec == "fp64" else TOL_FP32,
                                    "band %s variant %d" % (name, vi))
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
