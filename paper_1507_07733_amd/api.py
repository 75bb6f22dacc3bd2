"""Python binding of libaeraunfold.so (argument marshalling only).

Every computation runs in the HIP library; PyTorch is used here only to
allocate device memory and to name the stream work is enqueued on.  The
functions mirror the C ABI in include/aeraunfold.h.  If the library has not
been built, :func:`lib` raises -- there is no fallback.
"""
from __future__ import annotations

import ctypes as C
import os
import threading

import numpy as np

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG, "libaeraunfold.so")

AU_OK = 0
AU_EINVAL = -1
AU_ENOMEM = -2
AU_EDEVICE = -3
AU_EAGAIN = -4
AU_ENOTFOUND = -5

AU_F32 = 1
AU_F64 = 2
AU_PREC_FP64 = 0
AU_PREC_FP32 = 1
AU_PLAN_GRAPH = 1
AU_PLAN_PERSISTENT = 2
AU_PLAN_XCD = 4
AU_PLAN_FUSED = 8

FS_HZ = 200_000_000
BAND_LO_HZ = 30_000_000
BAND_HI_HZ = 80_000_000


class AuGrid(C.Structure):
    _fields_ = [("n_freq", C.c_int32), ("n_zen", C.c_int32), ("n_az", C.c_int32), ("reserved", C.c_int32),
                ("f0_hz", C.c_int64), ("df_hz", C.c_int64),
                ("zen0_deg", C.c_double), ("dzen_deg", C.c_double),
                ("az0_deg", C.c_double), ("daz_deg", C.c_double)]


class AuEvent(C.Structure):
    _fields_ = [("n_stations", C.c_int32), ("n_samples", C.c_int32),
                ("fs_hz", C.c_int64), ("band_lo_hz", C.c_int64), ("band_hi_hz", C.c_int64),
                ("trace_dtype", C.c_int32), ("prec", C.c_int32),
                ("fallback_rel", C.c_double), ("singular_rel", C.c_double)]


class AuBatch(C.Structure):
    _fields_ = [("n_events", C.c_int32), ("prec", C.c_int32), ("trace_dtype", C.c_int32), ("flags", C.c_int32),
                ("fs_hz", C.c_int64), ("band_lo_hz", C.c_int64), ("band_hi_hz", C.c_int64),
                ("fallback_rel", C.c_double), ("singular_rel", C.c_double),
                ("n_stations", C.POINTER(C.c_int32)), ("n_samples", C.POINTER(C.c_int32)),
                ("n_dirs", C.POINTER(C.c_int32)), ("h_dirs", C.POINTER(C.c_double)),
                ("volt_offset", C.POINTER(C.c_int64)), ("efield_offset", C.POINTER(C.c_int64))]


class AuServerCfg(C.Structure):
    _fields_ = [("hbm_budget_bytes", C.c_uint64), ("staging_bytes", C.c_uint64), ("max_inflight", C.c_int32),
                ("n_streams", C.c_int32), ("max_batch_events", C.c_int32), ("prec", C.c_int32),
                ("trace_dtype", C.c_int32), ("reserved", C.c_int32),
                ("fs_hz", C.c_int64), ("band_lo_hz", C.c_int64), ("band_hi_hz", C.c_int64),
                ("fallback_rel", C.c_double), ("singular_rel", C.c_double), ("tick_s", C.c_double)]


class AuRequest(C.Structure):
    _fields_ = [("n_stations", C.c_int32), ("n_samples", C.c_int32), ("n_dirs", C.c_int32), ("reserved", C.c_int32),
                ("h_volt", C.c_void_p), ("h_dirs", C.POINTER(C.c_double)), ("t_arrival", C.c_double)]


class AuResult(C.Structure):
    _fields_ = [("d_efield", C.c_void_p), ("efield_bytes", C.c_uint64), ("n_stations", C.c_int32),
                ("n_samples", C.c_int32), ("n_dirs", C.c_int32), ("batch_events", C.c_int32),
                ("t_arrival", C.c_double), ("t_submit", C.c_double), ("t_admit", C.c_double),
                ("t_launch", C.c_double), ("t_complete", C.c_double), ("batch_id", C.c_uint64)]


class AuServerStats(C.Structure):
    _fields_ = [(n, C.c_uint64) for n in ("submitted", "completed", "rejected", "batches", "queued", "in_flight",
                                          "arena_bytes", "arena_in_use", "arena_peak", "fallback_bins",
                                          "singular_bins")]


class AuError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__("aeraunfold status %d: %s" % (status, msg))
        self.status = status


_lock = threading.Lock()
_lib = None

# exported symbol -> (restype, argtypes)
_VP = C.c_void_p
_SIG = {
    "au_last_error": (C.c_char_p, []),
    "au_version": (C.c_char_p, []),
    "au_load_pattern_table": (C.c_int32, [C.POINTER(AuGrid), C.c_int32, _VP, C.POINTER(_VP)]),
    "au_free_pattern_table": (C.c_int32, [_VP]),
    "au_workspace_bytes": (C.c_int32, [_VP, C.POINTER(AuEvent), C.c_int32, C.POINTER(C.c_uint64)]),
    "au_band_bins": (C.c_int32, [C.POINTER(AuEvent), C.POINTER(C.c_int32), C.POINTER(C.c_int32)]),
    "au_unfold_event": (C.c_int32, [_VP, C.POINTER(AuEvent), _VP, C.c_double, C.c_double, _VP, _VP,
                                    C.c_uint64, _VP, _VP]),
    "au_unfold_direction_scan": (C.c_int32, [_VP, C.POINTER(AuEvent), _VP, C.c_int32, C.POINTER(C.c_double),
                                             _VP, _VP, C.c_uint64, _VP, _VP]),
    "au_unfold_envelope_scan": (C.c_int32, [_VP, C.POINTER(AuEvent), _VP, C.c_int32, C.POINTER(C.c_double),
                                            _VP, _VP, _VP, _VP, C.c_uint64, _VP, _VP]),
    "au_pattern_response": (C.c_int32, [_VP, C.POINTER(AuEvent), C.c_int32, C.POINTER(C.c_double), _VP, _VP]),
    "au_pattern_response_quantized": (C.c_int32, [_VP, C.POINTER(AuEvent), C.c_int32, C.POINTER(C.c_double),
                                                  C.c_int32, _VP, _VP]),
    "au_direction_fit_workspace_bytes": (C.c_int32, [_VP, C.POINTER(AuEvent), C.c_int32, C.c_int32, C.c_int32,
                                                     C.POINTER(C.c_uint64)]),
    "au_direction_fit": (C.c_int32, [_VP, C.POINTER(AuEvent), _VP, C.POINTER(C.c_double), C.c_int32,
                                     C.POINTER(C.c_double), C.c_int32, C.c_int32, C.c_double, C.c_double,
                                     C.POINTER(C.c_double), C.POINTER(C.c_double), C.POINTER(C.c_double),
                                     C.POINTER(C.c_int32), C.POINTER(C.c_double), _VP, C.c_uint64, _VP]),
    "au_reconstruct_batch_workspace_bytes": (C.c_int32, [_VP, C.POINTER(AuEvent), C.c_int32, C.POINTER(C.c_int32),
                                                         C.POINTER(C.c_int64), C.c_int32, C.POINTER(C.c_uint64)]),
    "au_reconstruct_batch": (C.c_int32, [_VP, C.POINTER(AuEvent), C.c_int32, C.POINTER(C.c_int32),
                                         C.POINTER(C.c_int64), _VP, C.POINTER(C.c_double), C.c_int32,
                                         C.POINTER(C.c_double), C.POINTER(C.c_int32), C.POINTER(C.c_int32),
                                         C.POINTER(C.c_int32), _VP, C.c_uint64, _VP]),
    "au_reconstruct_workspace_bytes": (C.c_int32, [_VP, C.POINTER(AuEvent), C.c_int32, C.POINTER(C.c_uint64)]),
    "au_reconstruct": (C.c_int32, [_VP, C.POINTER(AuEvent), _VP, C.POINTER(C.c_double), C.c_int32,
                                   C.POINTER(C.c_double), C.POINTER(C.c_int32), C.POINTER(C.c_int32),
                                   C.POINTER(C.c_int32), _VP, _VP, _VP, C.c_uint64, _VP]),
    "au_plan_create": (C.c_int32, [_VP, C.POINTER(AuBatch), C.POINTER(_VP)]),
    "au_plan_units": (C.c_int32, [_VP, C.POINTER(C.c_uint64)]),
    "au_plan_run": (C.c_int32, [_VP, _VP, _VP, _VP, _VP]),
    "au_plan_free": (C.c_int32, [_VP]),
    "au_plan_autotune": (C.c_int32, [_VP, _VP, _VP, C.c_int32, _VP, C.POINTER(C.c_double), C.POINTER(C.c_int32)]),
    "au_plan_timing": (C.c_int32, [_VP, C.c_int32]),
    "au_plan_classes": (C.c_int32, [_VP, C.c_int32, C.POINTER(C.c_int32), C.POINTER(C.c_uint64),
                                    C.POINTER(C.c_int32), C.POINTER(C.c_int32)]),
    "au_hbm_copy": (C.c_int32, [_VP, _VP, C.c_uint64, _VP]),
    "au_hbm_fill": (C.c_int32, [_VP, C.c_uint64, C.c_uint32, _VP]),
    "au_plan_stage_ms": (C.c_int32, [_VP, C.c_int32, C.POINTER(C.c_double), C.POINTER(C.c_uint64)]),
    "au_unfold_variant_count": (C.c_int32, [C.POINTER(C.c_int32)] * 7),
    "au_set_unfold_variant": (C.c_int32, [C.c_int32, C.c_int32, C.c_int32]),
    "au_get_unfold_variant": (C.c_int32, [C.c_int32, C.c_int32, C.POINTER(C.c_int32)]),
    "au_autotune": (C.c_int32, [_VP, C.POINTER(AuEvent), C.c_int32, C.c_int32, C.POINTER(C.c_double),
                                C.POINTER(C.c_int32)]),
    "au_server_create": (C.c_int32, [_VP, C.POINTER(AuServerCfg), C.POINTER(_VP)]),
    "au_server_destroy": (C.c_int32, [_VP]),
    "au_server_now": (C.c_int32, [_VP, C.POINTER(C.c_double)]),
    "au_submit": (C.c_int32, [_VP, C.POINTER(AuRequest), C.POINTER(C.c_uint64)]),
    "au_unfold_direction_scan_noalloc": (C.c_int32, [_VP, C.POINTER(AuEvent), _VP, C.c_int32, _VP, _VP, _VP, _VP]),
    "au_poll": (C.c_int32, [_VP, C.c_uint64, C.POINTER(AuResult)]),
    "au_wait": (C.c_int32, [_VP, C.c_uint64, C.c_double, C.POINTER(AuResult)]),
    "au_server_request_bytes": (C.c_int32, [_VP, C.c_int32, C.c_int32, C.c_int32, C.POINTER(C.c_uint64)]),
    "au_copy_result": (C.c_int32, [_VP, C.c_uint64, _VP, C.c_uint64]),
    "au_release": (C.c_int32, [_VP, C.c_uint64]),
    "au_server_stats": (C.c_int32, [_VP, C.POINTER(AuServerStats)]),
}


def lib():
    """Load libaeraunfold.so (raises if it has not been built)."""
    global _lib
    with _lock:
        if _lib is None:
            if not os.path.exists(LIB_PATH):
                raise RuntimeError("libaeraunfold.so is not built; run __graft_entry__.build() "
                                   "or python paper_1507_07733_amd/build.py")
            L = C.CDLL(LIB_PATH)
            for name, (res, args) in _SIG.items():
                f = getattr(L, name)
                f.restype = res
                f.argtypes = args
            _lib = L
    return _lib


def declared_symbols():
    return sorted(_SIG)


def _check(rc: int):
    if rc != AU_OK:
        raise AuError(rc, lib().au_last_error().decode(errors="replace"))


def _stream_handle(stream):
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return C.c_void_p(stream.cuda_stream)


def _ptr(t):
    return C.c_void_p(0 if t is None else t.data_ptr())


def make_grid(g) -> AuGrid:
    return AuGrid(g.n_freq, g.n_zen, g.n_az, 0, int(g.f0_hz), int(g.df_hz),
                  float(g.zen0_deg), float(g.dzen_deg), float(g.az0_deg), float(g.daz_deg))


def make_event(n_stations: int, n_samples: int, prec: int = AU_PREC_FP64, trace_dtype: int = AU_F64,
               fs_hz: int = FS_HZ, band_lo_hz: int = BAND_LO_HZ, band_hi_hz: int = BAND_HI_HZ,
               fallback_rel: float = 1e-6, singular_rel: float = 1e-12) -> AuEvent:
    return AuEvent(int(n_stations), int(n_samples), int(fs_hz), int(band_lo_hz), int(band_hi_hz),
                   int(trace_dtype), int(prec), float(fallback_rel), float(singular_rel))


def out_dtype(prec: int):
    import torch
    return torch.float64 if prec == AU_PREC_FP64 else torch.float32


def trace_code(t) -> int:
    import torch
    if t.dtype == torch.float64:
        return AU_F64
    if t.dtype == torch.float32:
        return AU_F32
    raise TypeError("traces must be float32 or float64")


class Table:
    """A pattern table resident on the current device."""

    def __init__(self, grid, table: np.ndarray):
        t = np.asarray(table)
        if t.dtype == np.complex128:
            code = AU_F64
        elif t.dtype == np.complex64:
            code = AU_F32
        else:
            raise TypeError("pattern table must be complex64 or complex128")
        t = np.ascontiguousarray(t)
        h = C.c_void_p()
        g = make_grid(grid)
        _check(lib().au_load_pattern_table(C.byref(g), code, t.ctypes.data_as(C.c_void_p), C.byref(h)))
        self.handle = h
        self.grid = grid
        self.dtype = code

    def free(self):
        if getattr(self, "handle", None) is not None and self.handle.value:
            _check(lib().au_free_pattern_table(self.handle))
            self.handle = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


def load_pattern_table(grid, table) -> Table:
    return Table(grid, table)


def band_bins(ev: AuEvent):
    a, b = C.c_int32(), C.c_int32()
    _check(lib().au_band_bins(C.byref(ev), C.byref(a), C.byref(b)))
    return a.value, b.value


def workspace_bytes(table: Table, ev: AuEvent, n_dir: int) -> int:
    n = C.c_uint64()
    _check(lib().au_workspace_bytes(table.handle, C.byref(ev), int(n_dir), C.byref(n)))
    return n.value


def _check_traces(volt, ev: AuEvent):
    if not volt.is_cuda or not volt.is_contiguous():
        raise ValueError("traces must be a contiguous device tensor")
    if tuple(volt.shape) != (ev.n_stations, 2, ev.n_samples):
        raise ValueError("traces must have shape [S][2][N]")
    if trace_code(volt) != ev.trace_dtype:
        raise ValueError("trace dtype does not match the event")


def _work(work):
    if work is None:
        return C.c_void_p(0), 0
    return C.c_void_p(work.data_ptr()), work.numel() * work.element_size()


def unfold_event(table: Table, ev: AuEvent, volt, zen_deg: float, az_deg: float, out=None, work=None,
                 counts=None, stream=None):
    """E-field [S][2][N] for one direction; see au_unfold_event."""
    import torch
    _check_traces(volt, ev)
    if out is None:
        out = torch.empty((ev.n_stations, 2, ev.n_samples), dtype=out_dtype(ev.prec), device=volt.device)
    wp, wb = _work(work)
    _check(lib().au_unfold_event(table.handle, C.byref(ev), _ptr(volt), float(zen_deg), float(az_deg),
                                 _ptr(out), wp, wb, _stream_handle(stream), _ptr(counts)))
    return out


def unfold_direction_scan(table: Table, ev: AuEvent, volt, dirs, out=None, work=None, counts=None,
                          stream=None):
    """E-field [D][S][2][N] for every direction of dirs [D][2] (degrees)."""
    import torch
    _check_traces(volt, ev)
    d = np.ascontiguousarray(np.asarray(dirs, dtype=np.float64).reshape(-1, 2))
    if out is None:
        out = torch.empty((len(d), ev.n_stations, 2, ev.n_samples), dtype=out_dtype(ev.prec),
                          device=volt.device)
    wp, wb = _work(work)
    _check(lib().au_unfold_direction_scan(table.handle, C.byref(ev), _ptr(volt), len(d),
                                          d.ctypes.data_as(C.POINTER(C.c_double)), _ptr(out), wp, wb,
                                          _stream_handle(stream), _ptr(counts)))
    return out


def unfold_direction_scan_noalloc(table: Table, ev: AuEvent, volt, d_dirs, out, counts=None, stream=None):
    """au_unfold_direction_scan_noalloc: directions d_dirs [D][2] float64 and the output out [D][S][2][N]
    are device tensors the caller allocated; the call itself allocates nothing."""
    _check_traces(volt, ev)
    n_dir = int(d_dirs.shape[0])
    if d_dirs.dim() != 2 or d_dirs.shape[1] != 2 or not d_dirs.is_contiguous() or not d_dirs.is_cuda:
        raise ValueError("d_dirs must be a contiguous device tensor [D][2]")
    import torch
    if d_dirs.dtype != torch.float64:
        raise ValueError("d_dirs must be float64")
    want = (n_dir, ev.n_stations, 2, ev.n_samples)
    if tuple(out.shape) != want or out.dtype != out_dtype(ev.prec) or not out.is_contiguous():
        raise ValueError("out must be a contiguous %s tensor of shape %s" % (out_dtype(ev.prec), want))
    _check(lib().au_unfold_direction_scan_noalloc(table.handle, C.byref(ev), _ptr(volt), n_dir, _ptr(d_dirs),
                                                  _ptr(out), _stream_handle(stream), _ptr(counts)))
    return out


def unfold_envelope_scan(table: Table, ev: AuEvent, volt, dirs, efield=False, work=None, counts=None,
                         stream=None):
    """Envelope peaks for every (direction, station) of the theta, phi and total-field envelopes.

    Returns (peak [D][S][3], arg [D][S][3] int32, E or None) where E
    [D][S][2][N] is also produced when ``efield`` is True (or a tensor).
    """
    import torch
    _check_traces(volt, ev)
    d = np.ascontiguousarray(np.asarray(dirs, dtype=np.float64).reshape(-1, 2))
    dt = out_dtype(ev.prec)
    peak = torch.empty((len(d), ev.n_stations, 3), dtype=dt, device=volt.device)
    arg = torch.empty((len(d), ev.n_stations, 3), dtype=torch.int32, device=volt.device)
    out = None
    if efield is True:
        out = torch.empty((len(d), ev.n_stations, 2, ev.n_samples), dtype=dt, device=volt.device)
    elif efield is not False and efield is not None:
        out = efield
    wp, wb = _work(work)
    _check(lib().au_unfold_envelope_scan(table.handle, C.byref(ev), _ptr(volt), len(d),
                                         d.ctypes.data_as(C.POINTER(C.c_double)), _ptr(out), _ptr(peak),
                                         _ptr(arg), wp, wb, _stream_handle(stream), _ptr(counts)))
    return peak, arg, out


def reconstruct_workspace_bytes(table: Table, ev: AuEvent, max_iter: int) -> int:
    n = C.c_uint64()
    _check(lib().au_reconstruct_workspace_bytes(table.handle, C.byref(ev), int(max_iter), C.byref(n)))
    return n.value


class Reconstruction:
    """Result of :func:`reconstruct`: directions per pass, station times per pass, final traces."""

    def __init__(self, dirs, times, converged, efield, peak):
        self.dirs = dirs            # [K][2] degrees, last = result
        self.times = times          # [K+1][S] samples: voltage maxima, then envelope maxima per pass
        self.converged = converged
        self.efield = efield        # [S][2][N] at the final direction, or None
        self.peak = peak            # [S][3] envelope maxima at the final direction

    @property
    def direction(self):
        return self.dirs[-1]


def reconstruct(table: Table, ev: AuEvent, volt, positions, max_iter: int = 8, efield=False, work=None,
                stream=None) -> Reconstruction:
    """The reconstruction loop of one event on the device; see au_reconstruct."""
    import torch
    _check_traces(volt, ev)
    pos = np.ascontiguousarray(np.asarray(positions, dtype=np.float64).reshape(-1, 2))
    if len(pos) != ev.n_stations:
        raise ValueError("positions must have shape [S][2]")
    dt = out_dtype(ev.prec)
    out = None
    if efield is True:
        out = torch.empty((ev.n_stations, 2, ev.n_samples), dtype=dt, device=volt.device)
    elif efield is not False and efield is not None:
        out = efield
    peak = torch.empty((ev.n_stations, 3), dtype=dt, device=volt.device)
    dirs = np.zeros((max_iter, 2))
    times = np.zeros((max_iter + 1, ev.n_stations), dtype=np.int32)
    nd = C.c_int32()
    conv = C.c_int32()
    wp, wb = _work(work)
    _check(lib().au_reconstruct(table.handle, C.byref(ev), _ptr(volt), pos.ctypes.data_as(C.POINTER(C.c_double)),
                                int(max_iter), dirs.ctypes.data_as(C.POINTER(C.c_double)),
                                times.ctypes.data_as(C.POINTER(C.c_int32)), C.byref(nd), C.byref(conv),
                                _ptr(out), _ptr(peak), wp, wb, _stream_handle(stream)))
    k = nd.value
    return Reconstruction(dirs[:k], times[:k + 1], bool(conv.value), out, peak)


def direction_fit_workspace_bytes(table: Table, ev: AuEvent, n_dir: int, levels: int, k: int) -> int:
    n = C.c_uint64()
    _check(lib().au_direction_fit_workspace_bytes(table.handle, C.byref(ev), int(n_dir), int(levels), int(k),
                                                  C.byref(n)))
    return n.value


def direction_fit(table: Table, ev: AuEvent, volt, positions, dirs, levels: int = 3, k: int = 5,
                  step=(5.0, 5.0), work=None, stream=None):
    """Coarse scan + device refinements; see au_direction_fit.

    Returns dict(result [2], best [levels+1], chi2, power [n_dir + levels*k*k], level_dirs [levels][k*k][2]).
    """
    _check_traces(volt, ev)
    pos = np.ascontiguousarray(np.asarray(positions, dtype=np.float64).reshape(-1, 2))
    if len(pos) != ev.n_stations:
        raise ValueError("positions must have shape [S][2]")
    d = np.ascontiguousarray(np.asarray(dirs, dtype=np.float64).reshape(-1, 2))
    tot = len(d) + levels * k * k
    ld = np.zeros((max(levels, 1), k * k, 2))
    chi2 = np.zeros(tot)
    pw = np.zeros(tot)
    best = np.zeros(levels + 1, dtype=np.int32)
    res = np.zeros(2)
    dp = C.POINTER(C.c_double)
    wp, wb = _work(work)
    _check(lib().au_direction_fit(table.handle, C.byref(ev), _ptr(volt), pos.ctypes.data_as(dp), len(d),
                                  d.ctypes.data_as(dp), int(levels), int(k), float(step[0]), float(step[1]),
                                  ld.ctypes.data_as(dp), chi2.ctypes.data_as(dp), pw.ctypes.data_as(dp),
                                  best.ctypes.data_as(C.POINTER(C.c_int32)), res.ctypes.data_as(dp), wp, wb,
                                  _stream_handle(stream)))
    return {"result": res, "best": best, "chi2": chi2, "power": pw, "level_dirs": ld[:levels]}


def reconstruct_batch(table: Table, ev: AuEvent, volt, n_stations, volt_offsets, positions, max_iter: int = 8,
                      work=None, stream=None):
    """The reconstruction loop for many events at once; see au_reconstruct_batch.

    volt: flat device tensor holding every event's [S][2][N] traces at volt_offsets[e];
    positions: [sum S][2].  Returns a list of Reconstruction (efield and peak None).
    """
    if not volt.is_cuda or not volt.is_contiguous() or trace_code(volt) != ev.trace_dtype:
        raise ValueError("traces must be a contiguous device tensor of the event's trace type")
    ns = np.ascontiguousarray(np.asarray(n_stations, dtype=np.int32))
    vo = np.ascontiguousarray(np.asarray(volt_offsets, dtype=np.int64))
    pos = np.ascontiguousarray(np.asarray(positions, dtype=np.float64).reshape(-1, 2))
    n_ev = len(ns)
    if len(vo) != n_ev or len(pos) != int(ns.sum()):
        raise ValueError("one offset per event and one position per station")
    if np.any(vo + ns.astype(np.int64) * 2 * ev.n_samples > volt.numel()):
        raise ValueError("trace offsets exceed the trace buffer")
    stot = int(ns.sum())
    dirs = np.zeros((n_ev, max_iter, 2))
    times = np.zeros((max_iter + 1, stot), dtype=np.int32)
    nd = np.zeros(n_ev, dtype=np.int32)
    conv = np.zeros(n_ev, dtype=np.int32)
    i32 = C.POINTER(C.c_int32)
    wp, wb = _work(work)
    _check(lib().au_reconstruct_batch(table.handle, C.byref(ev), n_ev, ns.ctypes.data_as(i32),
                                      vo.ctypes.data_as(C.POINTER(C.c_int64)), _ptr(volt),
                                      pos.ctypes.data_as(C.POINTER(C.c_double)), int(max_iter),
                                      dirs.ctypes.data_as(C.POINTER(C.c_double)), times.ctypes.data_as(i32),
                                      nd.ctypes.data_as(i32), conv.ctypes.data_as(i32), wp, wb,
                                      _stream_handle(stream)))
    out = []
    so = 0
    for e in range(n_ev):
        k = int(nd[e])
        out.append(Reconstruction(dirs[e, :k], times[:k + 1, so:so + ns[e]], int(conv[e]), None, None))
        so += int(ns[e])
    return out


def pattern_response(table: Table, ev: AuEvent, dirs, device=None, stream=None, weight_bits: int = 0):
    """Interpolated H at every in-band bin: complex tensor [D][n_band][2][2].

    weight_bits > 0 rounds the interpolation weights to that many fractional
    bits (au_pattern_response_quantized)."""
    import torch
    d = np.ascontiguousarray(np.asarray(dirs, dtype=np.float64).reshape(-1, 2))
    _, nb = band_bins(ev)
    rd = out_dtype(ev.prec)
    out = torch.zeros((len(d), nb, 2, 2, 2), dtype=rd, device=device or "cuda")
    dp = d.ctypes.data_as(C.POINTER(C.c_double))
    if weight_bits:
        _check(lib().au_pattern_response_quantized(table.handle, C.byref(ev), len(d), dp, int(weight_bits),
                                                   _ptr(out), _stream_handle(stream)))
    else:
        _check(lib().au_pattern_response(table.handle, C.byref(ev), len(d), dp, _ptr(out), _stream_handle(stream)))
    return torch.view_as_complex(out)


def hbm_copy(dst, src, nbytes: int = None, stream=None):
    """Device-to-device copy with the library's bandwidth probe kernel."""
    n = nbytes if nbytes is not None else min(dst.numel() * dst.element_size(), src.numel() * src.element_size())
    _check(lib().au_hbm_copy(_ptr(dst), _ptr(src), int(n), _stream_handle(stream)))


def hbm_fill(dst, nbytes: int = None, value: int = 0, stream=None):
    """Write-only bandwidth probe (non-temporal stores)."""
    n = nbytes if nbytes is not None else dst.numel() * dst.element_size()
    _check(lib().au_hbm_fill(_ptr(dst), int(n), int(value), _stream_handle(stream)))


def unfold_kernel_name(prec: int, n: int, variant: int) -> str:
    """Template name of the unfold kernel a (precision, N, variant) launches."""
    e, rmax, tw, wave, pair, pp = unfold_variants()[variant]
    e = n // 64 if e == 0 else e
    e = min(e, n)
    rmax = min(rmax, e)
    t = "double" if prec == AU_PREC_FP64 else "float"
    b = lambda x: "true" if x else "false"
    return "k_unfold<%s, %d, %d, %d, %d, %s, %s, %s>" % (t, n, e, rmax, tw, b(wave), b(pair), b(pp))


def unfold_variants():
    """[(E, rmax, twmode, wave, pair, pp)] of the unfold-kernel shapes the library is built in."""
    n = C.c_int32()
    e, r, t, w, p, q = ((C.c_int32 * 32)() for _ in range(6))
    _check(lib().au_unfold_variant_count(C.byref(n), e, r, t, w, p, q))
    return [(e[i], r[i], t[i], bool(w[i]), bool(p[i]), bool(q[i])) for i in range(n.value)]


def set_unfold_variant(prec: int, n_samples: int, variant: int):
    _check(lib().au_set_unfold_variant(int(prec), int(n_samples), int(variant)))


def get_unfold_variant(prec: int, n_samples: int) -> int:
    v = C.c_int32()
    _check(lib().au_get_unfold_variant(int(prec), int(n_samples), C.byref(v)))
    return v.value


def autotune(table: Table, ev: AuEvent, n_dir: int = 16, reps: int = 3):
    """Time every unfold variant for ev's sizes, select the fastest; returns (best, ms list)."""
    nv = len(unfold_variants())
    ms = (C.c_double * nv)()
    best = C.c_int32()
    _check(lib().au_autotune(table.handle, C.byref(ev), int(n_dir), int(reps), ms, C.byref(best)))
    return best.value, list(ms)


class Plan:
    """A batched unfolding plan over events of uneven size (au_plan_*).

    events: list of (n_stations, n_samples, dirs[D][2]); traces of event e
    live at element offset volt_offsets[e] of one flat trace buffer and its
    output [D][S][2][N] at efield_offsets[e] of one flat output buffer.
    """

    def __init__(self, table: Table, events, prec: int, trace_dtype: int, flags: int = 0,
                 volt_offsets=None, efield_offsets=None, fs_hz: int = FS_HZ,
                 band_lo_hz: int = BAND_LO_HZ, band_hi_hz: int = BAND_HI_HZ,
                 fallback_rel: float = 1e-6, singular_rel: float = 1e-12):
        self.table = table
        s = np.array([e[0] for e in events], dtype=np.int32)
        n = np.array([e[1] for e in events], dtype=np.int32)
        dl = [np.asarray(e[2], dtype=np.float64).reshape(-1, 2) for e in events]
        dcount = np.array([len(x) for x in dl], dtype=np.int32)
        dirs = np.ascontiguousarray(np.concatenate(dl, axis=0))
        vsz = s.astype(np.int64) * 2 * n
        esz = dcount.astype(np.int64) * s * 2 * n
        if volt_offsets is None:
            volt_offsets = np.concatenate([[0], np.cumsum(vsz)[:-1]]).astype(np.int64)
        if efield_offsets is None:
            efield_offsets = np.concatenate([[0], np.cumsum(esz)[:-1]]).astype(np.int64)
        self.volt_offsets = np.ascontiguousarray(volt_offsets, dtype=np.int64)
        self.efield_offsets = np.ascontiguousarray(efield_offsets, dtype=np.int64)
        self.volt_elems = int((self.volt_offsets + vsz).max())
        self.efield_elems = int((self.efield_offsets + esz).max())
        self.n_stations, self.n_samples, self.n_dirs, self.dirs = s, n, dcount, dirs
        self.prec, self.trace_dtype = prec, trace_dtype
        b = AuBatch(len(events), int(prec), int(trace_dtype), int(flags), int(fs_hz), int(band_lo_hz),
                    int(band_hi_hz), float(fallback_rel), float(singular_rel),
                    s.ctypes.data_as(C.POINTER(C.c_int32)), n.ctypes.data_as(C.POINTER(C.c_int32)),
                    dcount.ctypes.data_as(C.POINTER(C.c_int32)), dirs.ctypes.data_as(C.POINTER(C.c_double)),
                    self.volt_offsets.ctypes.data_as(C.POINTER(C.c_int64)),
                    self.efield_offsets.ctypes.data_as(C.POINTER(C.c_int64)))
        h = C.c_void_p()
        _check(lib().au_plan_create(table.handle, C.byref(b), C.byref(h)))
        self.handle = h
        u = C.c_uint64()
        _check(lib().au_plan_units(h, C.byref(u)))
        self.station_unfolds = u.value

    def run(self, volt, efield, counts=None, stream=None):
        if volt.numel() < self.volt_elems or efield.numel() < self.efield_elems:
            raise ValueError("buffers smaller than the plan's offsets require")
        if trace_code(volt) != self.trace_dtype or efield.dtype != out_dtype(self.prec):
            raise ValueError("buffer dtypes do not match the plan")
        _check(lib().au_plan_run(self.handle, _ptr(volt), _ptr(efield), _stream_handle(stream), _ptr(counts)))

    def autotune(self, volt, efield, reps: int = 3, stream=None):
        """Pick the fastest unfold variant per class inside this plan.

        Returns [(n_samples, best variant, [ms per variant, -1 if not built])].
        """
        if volt.numel() < self.volt_elems or efield.numel() < self.efield_elems:
            raise ValueError("buffers smaller than the plan's offsets require")
        nc = len(self.classes())
        nv = len(unfold_variants())
        ms = (C.c_double * (nc * nv))()
        best = (C.c_int32 * nc)()
        _check(lib().au_plan_autotune(self.handle, _ptr(volt), _ptr(efield), int(reps), _stream_handle(stream),
                                      ms, best))
        cls = self.classes()
        return [(cls[i][0], best[i], list(ms[i * nv:(i + 1) * nv])) for i in range(nc)]

    def set_timing(self, enable: bool):
        _check(lib().au_plan_timing(self.handle, 1 if enable else 0))

    def classes(self):
        """[(n_samples, station_unfolds, unfold variant)] per trace-length class, in stage order."""
        nc = C.c_int32()
        _check(lib().au_plan_classes(self.handle, 0, None, None, None, C.byref(nc)))
        ns = (C.c_int32 * max(nc.value, 1))()
        su = (C.c_uint64 * max(nc.value, 1))()
        va = (C.c_int32 * max(nc.value, 1))()
        _check(lib().au_plan_classes(self.handle, nc.value, ns, su, va, C.byref(nc)))
        return [(ns[i], su[i], va[i]) for i in range(nc.value)]

    def stage_ms(self):
        """(per-class [spectrum, coef, unfold] summed ms, number of timed runs)."""
        nc = len(self.classes())
        ms = (C.c_double * (3 * nc))()
        runs = C.c_uint64()
        _check(lib().au_plan_stage_ms(self.handle, 3 * nc, ms, C.byref(runs)))
        return np.array(ms[:]).reshape(nc, 3), runs.value

    def event_output(self, efield, e: int):
        n, s, d = int(self.n_samples[e]), int(self.n_stations[e]), int(self.n_dirs[e])
        o = int(self.efield_offsets[e])
        return efield[o:o + d * s * 2 * n].view(d, s, 2, n)

    def free(self):
        if getattr(self, "handle", None) is not None and self.handle.value:
            _check(lib().au_plan_free(self.handle))
            self.handle = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


class Server:
    """Continuous-batching unfolding server (au_server_*)."""

    def __init__(self, table: Table, hbm_budget_bytes: int, staging_bytes: int = 1 << 30,
                 max_inflight: int = 64, n_streams: int = 4, max_batch_events: int = 16,
                 prec: int = AU_PREC_FP32, trace_dtype: int = AU_F32, tick_s: float = 0.0,
                 fs_hz: int = FS_HZ, band_lo_hz: int = BAND_LO_HZ, band_hi_hz: int = BAND_HI_HZ,
                 fallback_rel: float = 1e-6, singular_rel: float = 1e-12):
        self.table = table
        self.prec, self.trace_dtype = prec, trace_dtype
        cfg = AuServerCfg(int(hbm_budget_bytes), int(staging_bytes), int(max_inflight), int(n_streams),
                          int(max_batch_events), int(prec), int(trace_dtype), 0, int(fs_hz), int(band_lo_hz),
                          int(band_hi_hz), float(fallback_rel), float(singular_rel), float(tick_s))
        h = C.c_void_p()
        _check(lib().au_server_create(table.handle, C.byref(cfg), C.byref(h)))
        self.handle = h

    def now(self) -> float:
        t = C.c_double()
        _check(lib().au_server_now(self.handle, C.byref(t)))
        return t.value

    def submit(self, volt, dirs, t_arrival: float = 0.0) -> int:
        """Queue one event (host traces [S][2][N]: a numpy array, or a CPU torch tensor, e.g. in
        pinned memory); returns its ticket.  Raises AuError with status AU_EAGAIN when the staging
        area is full."""
        want = np.float64 if self.trace_dtype == AU_F64 else np.float32
        d = np.ascontiguousarray(np.asarray(dirs, dtype=np.float64).reshape(-1, 2))
        if hasattr(volt, "data_ptr"):
            import torch
            tw = torch.float64 if self.trace_dtype == AU_F64 else torch.float32
            if volt.device.type != "cpu" or volt.dtype != tw or not volt.is_contiguous() or volt.dim() != 3:
                raise ValueError("traces must be a contiguous CPU tensor [S][2][N] of the server's dtype")
            s, two, n = volt.shape
            ptr = C.c_void_p(volt.data_ptr())
        else:
            v = np.ascontiguousarray(volt, dtype=want)
            s, two, n = v.shape
            ptr = v.ctypes.data_as(C.c_void_p)
        if two != 2:
            raise ValueError("traces must have shape [S][2][N]")
        rq = AuRequest(s, n, len(d), 0, ptr, d.ctypes.data_as(C.POINTER(C.c_double)), float(t_arrival))
        t = C.c_uint64()
        _check(lib().au_submit(self.handle, C.byref(rq), C.byref(t)))
        return t.value

    def request_bytes(self, n_stations: int, n_samples: int, n_dirs: int) -> int:
        """Arena bytes one request of these sizes occupies."""
        b = C.c_uint64()
        _check(lib().au_server_request_bytes(self.handle, int(n_stations), int(n_samples), int(n_dirs),
                                             C.byref(b)))
        return b.value

    def poll(self, ticket: int):
        """AuResult when complete, None while pending."""
        r = AuResult()
        rc = lib().au_poll(self.handle, C.c_uint64(ticket), C.byref(r))
        if rc == AU_EAGAIN:
            return None
        _check(rc)
        return r

    def wait(self, ticket: int, timeout_s: float = 60.0):
        """Block until the ticket completes (au_wait); TimeoutError after timeout_s."""
        r = AuResult()
        rc = lib().au_wait(self.handle, C.c_uint64(ticket), float(timeout_s), C.byref(r))
        if rc == AU_EAGAIN:
            raise TimeoutError("ticket %d not complete after %.1f s" % (ticket, timeout_s))
        _check(rc)
        return r

    def result(self, ticket: int) -> np.ndarray:
        """Copy a completed result to a host array [D][S][2][N]."""
        r = self.poll(ticket)
        if r is None:
            raise AuError(AU_EAGAIN, "not complete")
        dt = np.float64 if self.prec == AU_PREC_FP64 else np.float32
        out = np.empty((r.n_dirs, r.n_stations, 2, r.n_samples), dtype=dt)
        _check(lib().au_copy_result(self.handle, C.c_uint64(ticket), out.ctypes.data_as(C.c_void_p), out.nbytes))
        return out

    def release(self, ticket: int):
        _check(lib().au_release(self.handle, C.c_uint64(ticket)))

    def stats(self) -> dict:
        st = AuServerStats()
        _check(lib().au_server_stats(self.handle, C.byref(st)))
        return {n: getattr(st, n) for n, _ in AuServerStats._fields_}

    def close(self):
        if getattr(self, "handle", None) is not None and self.handle.value:
            _check(lib().au_server_destroy(self.handle))
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
