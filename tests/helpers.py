"""Shared test helpers: the per-trace comparison rule and oracle calls.

Comparison rule: for every output trace (direction, station, component),
r = max_n |E_gpu - E_oracle| / max_n |E_oracle|; an all-zero oracle trace
requires an all-zero GPU trace.  Bars: r <= 1e-12 for the FP64 path,
r <= 1e-5 for the FP32 path.  The FP32 bar is stated relative to the peak
amplitude of the station's E-field trace (both polarisation components,
station_errors); the per-component form used by most tests is stricter and
holds there, but a component carrying a small fraction of the field picks
up the rounding of the strong one through the inverse.
"""
import numpy as np

from oracle import oracle as O
from paper_1507_07733_amd import synth as S

TOL_FP64 = 1e-12
TOL_FP32 = 1e-5


def trace_errors(got, ref):
    """Per-trace relative error r over the last axis; zero traces give 0 or inf."""
    got = np.asarray(got, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    assert got.shape == ref.shape, (got.shape, ref.shape)
    peak = np.max(np.abs(ref), axis=-1)
    err = np.max(np.abs(got - ref), axis=-1)
    r = np.where(peak > 0, err / np.where(peak > 0, peak, 1.0), np.where(err > 0, np.inf, 0.0))
    return r


def station_errors(got, ref):
    """Per station E-field trace [..][2][N]: max over both components and samples of |got - ref|,
    divided by the larger component peak of ref."""
    got = np.asarray(got, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    assert got.shape == ref.shape and got.shape[-2] == 2
    peak = np.max(np.abs(ref), axis=(-1, -2))
    err = np.max(np.abs(got - ref), axis=(-1, -2))
    return np.where(peak > 0, err / np.where(peak > 0, peak, 1.0), np.where(err > 0, np.inf, 0.0))


def assert_traces_close(got, ref, tol, what=""):
    r = trace_errors(got, ref)
    worst = float(np.max(r)) if r.size else 0.0
    assert worst <= tol, "%s: max per-trace error %.3e > %.1e (median %.3e)" % (
        what, worst, tol, float(np.median(r)))
    return r


def oracle_unfold(grid, table, volt, dirs, units=None, singular_rel=1e-12):
    """Oracle on the same values the GPU saw (float32 inputs promoted exactly)."""
    return O.unfold(grid, np.asarray(table).astype(np.complex128), np.asarray(volt, dtype=np.float64),
                    dirs, S.FS_HZ, S.BAND_LO_HZ, S.BAND_HI_HZ, singular_rel=singular_rel, units=units)
