"""Python access to the plain FP64 CPU oracle (``oracle.c``).

TEST INFRASTRUCTURE ONLY: used by the test suite, the smoke check and the
CPU-baseline leg of the benchmark.  The product path never imports it.

The oracle is compiled with gcc (``-O2 -ffp-contract=off``) into
``oracle/liboracle.so``; :func:`build` does that and :func:`lib` builds on
first use if the library is missing or older than its source.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
import threading

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "oracle.c")
SO = os.path.join(HERE, "liboracle.so")

_lock = threading.Lock()
_lib = None


class OrcGrid(C.Structure):
    _fields_ = [("n_freq", C.c_int32), ("n_zen", C.c_int32), ("n_az", C.c_int32), ("pad_", C.c_int32),
                ("f0_hz", C.c_int64), ("df_hz", C.c_int64),
                ("zen0_deg", C.c_double), ("dzen_deg", C.c_double),
                ("az0_deg", C.c_double), ("daz_deg", C.c_double)]


def build(force: bool = True) -> str:
    """Compile liboracle.so from oracle.c with gcc."""
    if force or not os.path.exists(SO) or os.path.getmtime(SO) < os.path.getmtime(SRC):
        tmp = SO + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-ffp-contract=off", "-fPIC", "-shared",
                               "-o", tmp, SRC, "-lm"])
        os.replace(tmp, SO)
    return SO


def lib():
    global _lib
    with _lock:
        if _lib is None:
            build(force=False)
            L = C.CDLL(SO)
            dp = C.POINTER(C.c_double)
            ip = C.POINTER(C.c_int64)
            L.orc_fft.argtypes = [C.c_int64, dp, dp, C.c_int]
            L.orc_fft.restype = C.c_int
            L.orc_in_band.argtypes = [C.c_int64] * 5
            L.orc_in_band.restype = C.c_int
            L.orc_pattern_at_bin.argtypes = [C.POINTER(OrcGrid), dp, C.c_int64, C.c_int64, C.c_int64,
                                             C.c_double, C.c_double, dp]
            L.orc_pattern_at_bin.restype = C.c_int
            L.orc_pattern_at_bin_quantized.argtypes = [C.POINTER(OrcGrid), dp, C.c_int64, C.c_int64, C.c_int64,
                                                       C.c_double, C.c_double, C.c_int, dp]
            L.orc_pattern_at_bin_quantized.restype = C.c_int
            L.orc_solve2.argtypes = [dp, dp, C.c_double, dp]
            L.orc_solve2.restype = C.c_int
            L.orc_unfold_units.argtypes = [C.POINTER(OrcGrid), dp, C.c_int64, C.c_int64, C.c_int64,
                                           C.c_int64, C.c_int64, C.c_double, dp, C.c_int64, dp,
                                           C.c_int64, ip, dp, ip, dp]
            L.orc_unfold_units.restype = C.c_int
            L.orc_envelope.argtypes = [C.c_int64, dp, dp]
            L.orc_envelope.restype = C.c_int
            L.orc_envelope_peaks.argtypes = [C.c_int64, C.c_int64, dp, dp, ip]
            L.orc_envelope_peaks.restype = C.c_int
            L.orc_plane_fit.argtypes = [C.c_int64, dp, ip, C.c_int64, dp]
            L.orc_plane_fit.restype = C.c_int
            L.orc_reconstruct.argtypes = [C.POINTER(OrcGrid), dp, C.c_int64, C.c_int64, C.c_int64, C.c_int64,
                                          C.c_int64, C.c_double, dp, dp, C.c_int64, dp, ip, ip, ip]
            L.orc_reconstruct.restype = C.c_int
            L.orc_direction_objective.argtypes = [C.c_int64, dp, C.c_int64, dp, ip, C.c_int64, dp, dp, dp]
            L.orc_direction_objective.restype = None
            L.orc_local_grid.argtypes = [C.c_double, C.c_double, C.c_double, C.c_double, C.c_int64, dp]
            L.orc_local_grid.restype = None
            L.orc_direction_fit.argtypes = [C.POINTER(OrcGrid), dp, C.c_int64, C.c_int64, C.c_int64, C.c_int64,
                                            C.c_int64, C.c_double, dp, dp, C.c_int64, dp, C.c_int64, C.c_int64,
                                            C.c_double, C.c_double, dp, dp, dp, ip, dp]
            L.orc_direction_fit.restype = C.c_int
            _lib = L
    return _lib


def _dp(a):
    return a.ctypes.data_as(C.POINTER(C.c_double))


def _ip(a):
    return a.ctypes.data_as(C.POINTER(C.c_int64))


def make_grid(grid) -> OrcGrid:
    return OrcGrid(grid.n_freq, grid.n_zen, grid.n_az, 0, int(grid.f0_hz), int(grid.df_hz),
                   float(grid.zen0_deg), float(grid.dzen_deg), float(grid.az0_deg), float(grid.daz_deg))


def _table128(grid, table):
    t = np.ascontiguousarray(np.asarray(table), dtype=np.complex128)
    if t.shape != (2, 2, grid.n_freq, grid.n_zen, grid.n_az):
        raise ValueError("table shape %r does not match grid" % (t.shape,))
    return t


def fft(x, sign: int = -1) -> np.ndarray:
    """Unnormalised DFT, exp(sign 2 pi i j k / n), by the oracle's radix-2 FFT."""
    x = np.asarray(x, dtype=np.complex128)
    re = np.ascontiguousarray(x.real.copy())
    im = np.ascontiguousarray(x.imag.copy())
    if lib().orc_fft(len(x), _dp(re), _dp(im), int(sign)) != 0:
        raise ValueError("length must be a power of two")
    return re + 1j * im


def in_band(k: int, n: int, fs_hz: int, lo_hz: int, hi_hz: int) -> bool:
    return bool(lib().orc_in_band(k, n, fs_hz, lo_hz, hi_hz))


def pattern_at_bin(grid, table, k: int, n: int, fs_hz: int, zen: float, az: float) -> np.ndarray:
    """Interpolated H[c][p] (2x2 complex) at FFT bin k for direction (zen, az) deg."""
    t = _table128(grid, table)
    g = make_grid(grid)
    h = np.zeros(8)
    if lib().orc_pattern_at_bin(C.byref(g), _dp(t.view(np.float64)), k, n, fs_hz, zen, az, _dp(h)) != 0:
        raise ValueError("bin outside the table's frequency range")
    return (h[0::2] + 1j * h[1::2]).reshape(2, 2)


def pattern_at_bin_quantized(grid, table, k: int, n: int, fs_hz: int, zen: float, az: float, weight_bits: int):
    """pattern_at_bin with interpolation weights rounded to weight_bits fractional bits."""
    t = _table128(grid, table)
    g = make_grid(grid)
    h = np.zeros(8)
    if lib().orc_pattern_at_bin_quantized(C.byref(g), _dp(t.view(np.float64)), k, n, fs_hz, zen, az,
                                          int(weight_bits), _dp(h)) != 0:
        raise ValueError("bin outside the table's frequency range")
    return (h[0::2] + 1j * h[1::2]).reshape(2, 2)


def solve2(h, x, singular_rel: float = 1e-12):
    """Solve the 2x2 complex system h e = x; returns (e, singular)."""
    hh = np.ascontiguousarray(np.asarray(h, dtype=np.complex128).reshape(4)).view(np.float64).copy()
    xx = np.ascontiguousarray(np.asarray(x, dtype=np.complex128).reshape(2)).view(np.float64).copy()
    e = np.zeros(4)
    s = lib().orc_solve2(_dp(hh), _dp(xx), singular_rel, _dp(e))
    return e[0::2] + 1j * e[1::2], bool(s)


def unfold(grid, table, volt, dirs, fs_hz: int, lo_hz: int, hi_hz: int,
           singular_rel: float = 1e-12, units=None):
    """Unfold E-field traces.

    volt [S][2][N] (any real dtype, promoted to float64), dirs [D][2] degrees.
    With ``units`` = None every (direction, station) pair is computed and E
    has shape [D][S][2][N]; otherwise ``units`` is an int array [U][2] of
    (direction, station) pairs and E has shape [U][2][N].
    Returns (E, singular_bins per unit, max |Im|/peak after the inverse).
    """
    t = _table128(grid, table)
    v = np.ascontiguousarray(np.asarray(volt), dtype=np.float64)
    d = np.ascontiguousarray(np.asarray(dirs, dtype=np.float64).reshape(-1, 2))
    n_st, two, n = v.shape
    assert two == 2
    full = units is None
    if full:
        dd, ss = np.meshgrid(np.arange(len(d)), np.arange(n_st), indexing="ij")
        units = np.stack([dd.ravel(), ss.ravel()], axis=1)
    u = np.ascontiguousarray(np.asarray(units, dtype=np.int64).reshape(-1, 2))
    e = np.zeros((len(u), 2, n))
    sing = np.zeros(len(u), dtype=np.int64)
    mi = np.zeros(1)
    g = make_grid(grid)
    rc = lib().orc_unfold_units(C.byref(g), _dp(t.view(np.float64)), n_st, n, fs_hz, lo_hz, hi_hz,
                                singular_rel, _dp(v), len(d), _dp(d), len(u), _ip(u),
                                _dp(e), _ip(sing), _dp(mi))
    if rc != 0:
        raise ValueError("orc_unfold_units failed with %d" % rc)
    if full:
        e = e.reshape(len(d), n_st, 2, n)
        sing = sing.reshape(len(d), n_st)
    return e, sing, float(mi[0])


def envelope(x) -> np.ndarray:
    """Hilbert envelope sqrt(x^2 + H(x)^2) of a real trace (length a power of two)."""
    x = np.ascontiguousarray(np.asarray(x, dtype=np.float64))
    env = np.empty_like(x)
    if lib().orc_envelope(len(x), _dp(x), _dp(env)) != 0:
        raise ValueError("length must be a power of two >= 2")
    return env


def envelope_peaks(traces):
    """(peak value, first index of the peak) of the envelope of every trace along the last axis."""
    t = np.ascontiguousarray(np.asarray(traces, dtype=np.float64))
    n = t.shape[-1]
    flat = t.reshape(-1, n)
    peak = np.empty(len(flat))
    arg = np.empty(len(flat), dtype=np.int64)
    if lib().orc_envelope_peaks(len(flat), n, _dp(flat), _dp(peak), _ip(arg)) != 0:
        raise ValueError("bad trace length")
    return peak.reshape(t.shape[:-1]), arg.reshape(t.shape[:-1])


def plane_fit(positions, times, fs_hz: int):
    """(zenith, azimuth) degrees of the least-squares plane wave through station times (samples)."""
    p = np.ascontiguousarray(np.asarray(positions, dtype=np.float64).reshape(-1, 2))
    t = np.ascontiguousarray(np.asarray(times, dtype=np.int64))
    d = np.zeros(2)
    if lib().orc_plane_fit(len(p), _dp(p), _ip(t), fs_hz, _dp(d)) != 0:
        raise ValueError("singular station geometry")
    return d


def reconstruct(grid, table, volt, positions, fs_hz: int, lo_hz: int, hi_hz: int, max_iter: int = 8,
                singular_rel: float = 1e-12):
    """The reconstruction loop.

    Returns (directions [K][2], station times [K+1][S] per pass (row 0 the
    voltage maxima, row i+1 the envelope maxima after direction i), converged).
    """
    tb = _table128(grid, table)
    v = np.ascontiguousarray(np.asarray(volt), dtype=np.float64)
    p = np.ascontiguousarray(np.asarray(positions, dtype=np.float64).reshape(-1, 2))
    n_st, two, n = v.shape
    dirs = np.zeros((max_iter, 2))
    times = np.zeros((max_iter + 1, n_st), dtype=np.int64)
    nd = np.zeros(1, dtype=np.int64)
    conv = np.zeros(1, dtype=np.int64)
    g = make_grid(grid)
    rc = lib().orc_reconstruct(C.byref(g), _dp(tb.view(np.float64)), n_st, n, fs_hz, lo_hz, hi_hz, singular_rel,
                               _dp(v), _dp(p), max_iter, _dp(dirs), _ip(times), _ip(nd), _ip(conv))
    if rc != 0:
        raise ValueError("orc_reconstruct failed with %d" % rc)
    return dirs[:nd[0]], times[:nd[0] + 1], bool(conv[0])


def direction_objective(positions, dirs, times, fs_hz: int, peaks=None):
    """(chi2 [D], power [D] or None): plane-wave timing inconsistency of station times [D][S] per direction."""
    p = np.ascontiguousarray(np.asarray(positions, dtype=np.float64).reshape(-1, 2))
    d = np.ascontiguousarray(np.asarray(dirs, dtype=np.float64).reshape(-1, 2))
    t = np.ascontiguousarray(np.asarray(times, dtype=np.int64).reshape(len(d), len(p)))
    chi2 = np.zeros(len(d))
    pw = None
    pk = None
    if peaks is not None:
        pk = np.ascontiguousarray(np.asarray(peaks, dtype=np.float64).reshape(len(d), len(p)))
        pw = np.zeros(len(d))
    lib().orc_direction_objective(len(p), _dp(p), len(d), _dp(d), _ip(t), fs_hz,
                                  _dp(pk) if pk is not None else None, _dp(chi2),
                                  _dp(pw) if pw is not None else None)
    return chi2, pw


def local_grid(zc: float, ac: float, hz: float, ha: float, k: int):
    """k x k refinement directions [k*k][2] around (zc, ac)."""
    d = np.zeros((k * k, 2))
    lib().orc_local_grid(zc, ac, hz, ha, k, _dp(d))
    return d


def direction_fit(grid, table, volt, positions, dirs, fs_hz: int, lo_hz: int, hi_hz: int, levels: int = 2,
                  k: int = 5, step=(5.0, 5.0), singular_rel: float = 1e-12):
    """Coarse scan + local refinements; returns dict(level_dirs, chi2, power, best, result)."""
    tb = _table128(grid, table)
    v = np.ascontiguousarray(np.asarray(volt), dtype=np.float64)
    p = np.ascontiguousarray(np.asarray(positions, dtype=np.float64).reshape(-1, 2))
    d = np.ascontiguousarray(np.asarray(dirs, dtype=np.float64).reshape(-1, 2))
    n_st, _, n = v.shape
    tot = len(d) + levels * k * k
    ld = np.zeros((max(levels, 1), k * k, 2))
    chi2 = np.zeros(tot)
    pw = np.zeros(tot)
    best = np.zeros(levels + 1, dtype=np.int64)
    res = np.zeros(2)
    g = make_grid(grid)
    rc = lib().orc_direction_fit(C.byref(g), _dp(tb.view(np.float64)), n_st, n, fs_hz, lo_hz, hi_hz, singular_rel,
                                 _dp(v), _dp(p), len(d), _dp(d), levels, k, float(step[0]), float(step[1]),
                                 _dp(ld), _dp(chi2), _dp(pw), _ip(best), _dp(res))
    if rc != 0:
        raise ValueError("orc_direction_fit failed with %d" % rc)
    return {"level_dirs": ld[:levels], "chi2": chi2, "power": pw, "best": best, "result": res}
