"""Seeded synthetic inputs shaped like AERA radio events.

This module only *generates data*: pattern tables, voltage traces, event
size mixes, candidate-direction grids and arrival times.  It holds none of
the unfolding arithmetic, so both the HIP path and the CPU oracle can take
their inputs from it without sharing any of the method's code.

The shapes follow the paper: up to 124 stations with two polarised channels
each and an antenna band of 30-80 MHz (section 1, AERA description; section
2, two-channel read-out), and a vector-effective-length table of complex
(theta, phi) pairs on a discrete (frequency, zenith, azimuth) grid (section
3).  Measured AERA patterns and traces are not available, so the generators
below stand in for them:

* pattern table: a crossed-dipole response with smooth low-order angular
  harmonics, multiplied by a per-channel frequency resonance;
* traces: unit Gaussian noise plus a pulse that is band-limited exactly to
  the in-band FFT bins of the trace, at a continuous random time;
* directions: cell-centred zenith/azimuth grids.

All randomness comes from ``numpy.random.default_rng`` seeded with
``SeedSequence([7733, cfg, stream, ...])`` so a run can be repeated bit for
bit on any machine with the same numpy.
"""
from __future__ import annotations

from dataclasses import dataclass, field
import numpy as np

SEED_ROOT = 7733
STREAM_TABLE = 0
STREAM_TRACES = 1
STREAM_EVENTS = 2
STREAM_ARRIVALS = 3

FS_HZ = 200_000_000
BAND_LO_HZ = 30_000_000
BAND_HI_HZ = 80_000_000


def rng(cfg: int, stream: int, *extra: int) -> np.random.Generator:
    """Deterministic generator for (configuration, stream, extra keys)."""
    return np.random.default_rng(np.random.SeedSequence([SEED_ROOT, cfg, stream, *extra]))


@dataclass(frozen=True)
class Grid:
    """Node grid of a pattern table.

    Frequencies are integers in Hz so that the bin-to-node mapping can be
    evaluated exactly; angles are in degrees.  The azimuth axis is periodic:
    ``n_az * daz_deg == 360`` and node ``n_az - 1`` wraps to node 0.
    """
    n_freq: int
    n_zen: int
    n_az: int
    f0_hz: int
    df_hz: int
    zen0_deg: float
    dzen_deg: float
    az0_deg: float
    daz_deg: float

    @property
    def shape(self):
        return (2, 2, self.n_freq, self.n_zen, self.n_az)

    def freqs_hz(self):
        return self.f0_hz + self.df_hz * np.arange(self.n_freq, dtype=np.int64)

    def zeniths_deg(self):
        return self.zen0_deg + self.dzen_deg * np.arange(self.n_zen)

    def azimuths_deg(self):
        return self.az0_deg + self.daz_deg * np.arange(self.n_az)


# 0-100 MHz in 1 MHz steps, zenith 0-90 deg in 5 deg, azimuth 0-355 deg in 5 deg.
GRID_COARSE = Grid(101, 19, 72, 0, 1_000_000, 0.0, 5.0, 0.0, 5.0)
# 0-100 MHz in 0.5 MHz steps, zenith 0-90 deg in 1 deg, azimuth 0-359 deg in 1 deg.
GRID_FINE = Grid(201, 91, 360, 0, 500_000, 0.0, 1.0, 0.0, 1.0)


def resonance(f_hz: np.ndarray, f_c: float, q: float) -> np.ndarray:
    """Series-resonance response 1 / (1 + iQ(f/f_c - f_c/f)); zero at DC."""
    f = np.asarray(f_hz, dtype=np.float64)
    out = np.zeros(f.shape, dtype=np.complex128)
    nz = f > 0
    out[nz] = 1.0 / (1.0 + 1j * q * (f[nz] / f_c - f_c / f[nz]))
    return out


def pattern_table(grid: Grid, cfg: int = 0, eps: float = 0.05, q: float = 2.0,
                  f_res=(55e6, 60e6)) -> np.ndarray:
    """Synthetic vector-effective-length table, complex128 [2 ch][2 comp][nf][nz][na].

    H[c][theta] = R_c(f) cos(theta) (d_c(phi) + eps h_c,theta(theta, phi))
    H[c][phi]   = R_c(f)            (d'_c(phi) + eps h_c,phi(theta, phi))
    with the crossed-dipole base d_0 = cos phi, d'_0 = -sin phi,
    d_1 = sin phi, d'_1 = cos phi, and h = sum_{l<=2, |m|<=2} a_lm cos^l(theta) e^{i m phi},
    a_lm complex normal with variance 1/15 (one independent set per (c, comp)).
    cos(90 deg) is set to exactly zero, so the horizon row is exactly singular.
    """
    r = rng(cfg, STREAM_TABLE)
    th = np.deg2rad(grid.zeniths_deg())
    ph = np.deg2rad(grid.azimuths_deg())
    cth = np.cos(th)
    cth[grid.zeniths_deg() == 90.0] = 0.0
    ls = np.arange(3)
    ms = np.arange(-2, 3)
    # [nz][l] and [na][m]
    cpow = cth[:, None] ** ls[None, :]
    eim = np.exp(1j * ms[None, :] * ph[:, None])
    base = {
        (0, 0): np.cos(ph), (0, 1): -np.sin(ph),
        (1, 0): np.sin(ph), (1, 1): np.cos(ph),
    }
    f = grid.freqs_hz()
    out = np.empty(grid.shape, dtype=np.complex128)
    for c in range(2):
        rc = resonance(f, f_res[c], q)
        for p in range(2):
            a = (r.standard_normal((3, 5)) + 1j * r.standard_normal((3, 5))) * np.sqrt(1.0 / 30.0)
            h = cpow @ a @ eim.T                      # [nz][na]
            ang = base[(c, p)][None, :] + eps * h     # [nz][na]
            if p == 0:
                ang = cth[:, None] * ang
            out[c, p] = rc[:, None, None] * ang[None, :, :]
    return out


def identity_table(grid: Grid) -> np.ndarray:
    """Pattern H = I at every node: unfolding reduces to a band-pass filter."""
    out = np.zeros(grid.shape, dtype=np.complex128)
    out[0, 0] = 1.0
    out[1, 1] = 1.0
    return out


def band_bins(n: int, fs_hz: int = FS_HZ, lo_hz: int = BAND_LO_HZ, hi_hz: int = BAND_HI_HZ) -> np.ndarray:
    """Integer FFT bins k in [0, n/2] whose frequency k*fs/n lies in [lo, hi].

    Used here only to shape the synthetic pulse; the band test is integer
    arithmetic in Hz so it has no rounding.
    """
    k = np.arange(n // 2 + 1, dtype=np.int64)
    return k[(lo_hz * n <= k * fs_hz) & (k * fs_hz <= hi_hz * n)]


def pulse(n: int, t0: np.ndarray, amp: np.ndarray, fs_hz: int = FS_HZ,
          lo_hz: int = BAND_LO_HZ, hi_hz: int = BAND_HI_HZ) -> np.ndarray:
    """(A/|K|) sum_{k in K} cos(2 pi k (t - t0) / n) for t = 0..n-1, in float64.

    ``t0`` and ``amp`` broadcast against each other; the result has their
    shape plus a trailing axis of length ``n``.  The band K is a contiguous
    run of bins k1..k2, so the sum has the Dirichlet closed form
    [sin((k2+1/2)x) - sin((k1-1/2)x)] / (2 sin(x/2)) with x = 2 pi (t - t0)/n.
    """
    kb = band_bins(n, fs_hz, lo_hz, hi_hz)
    k1, k2, nk = float(kb[0]), float(kb[-1]), len(kb)
    t0 = np.asarray(t0, dtype=np.float64)[..., None]
    amp = np.asarray(amp, dtype=np.float64)[..., None]
    x = 2.0 * np.pi * (np.arange(n, dtype=np.float64) - t0) / n
    s = np.sin(0.5 * x)
    small = np.abs(s) < 1e-12
    ssafe = np.where(small, 1.0, s)
    val = (np.sin((k2 + 0.5) * x) - np.sin((k1 - 0.5) * x)) / (2.0 * ssafe)
    val = np.where(small, float(nk), val)
    return amp * val / nk


def traces(n_st: int, n: int, cfg: int, event: int = 0, dtype=np.float64,
           noise_sigma: float = 1.0, amp_range=(5.0, 20.0)) -> np.ndarray:
    """Voltage traces [S][2][N]: Gaussian noise (sigma 1) plus an in-band pulse.

    Amplitude is uniform in [5, 20] per (station, channel); the pulse time is
    uniform in [0, N) per station and shared by both channels.  Generated in
    float64 and rounded to nearest-even when ``dtype`` is float32.
    """
    r = rng(cfg, STREAM_TRACES, event)
    noise = r.standard_normal((n_st, 2, n)) * noise_sigma
    amp = r.uniform(amp_range[0], amp_range[1], size=(n_st, 2))
    t0 = r.uniform(0.0, n, size=(n_st, 1))
    v = noise + pulse(n, np.broadcast_to(t0, (n_st, 2)), amp)
    return np.ascontiguousarray(v.astype(dtype))


def direction_grid(n_zen: int, n_az: int) -> np.ndarray:
    """Cell-centred candidate directions [D][2] (zenith, azimuth) in degrees.

    theta_i = (i + 1/2) * 90 / n_zen, phi_j = j * 360 / n_az, zenith-major.
    """
    th = (np.arange(n_zen) + 0.5) * 90.0 / n_zen
    ph = np.arange(n_az) * 360.0 / n_az
    d = np.empty((n_zen * n_az, 2))
    d[:, 0] = np.repeat(th, n_az)
    d[:, 1] = np.tile(ph, n_zen)
    return d


# Horizon stress set: wrap, FP32-determinant fallback and exactly singular cases.
STRESS_ZENITHS = (0.0, 45.0, 89.0, 89.9, 89.99, 89.999, 89.9999, 89.99999, 90.0)
STRESS_AZIMUTHS = (0.0, 2.5, 357.5, 359.999)


def stress_directions() -> np.ndarray:
    d = [(z, a) for z in STRESS_ZENITHS for a in STRESS_AZIMUTHS]
    return np.asarray(d, dtype=np.float64)


@dataclass
class EventSpec:
    n_stations: int
    n_samples: int
    seed_event: int
    dirs: np.ndarray = field(repr=False)


def event_mix(n_events: int, cfg: int, s_range=(3, 124), n_choices=(2048, 4096),
              dirs: np.ndarray | None = None) -> list:
    """Uneven event list: S uniform in s_range (inclusive), N drawn with equal probability."""
    r = rng(cfg, STREAM_EVENTS)
    s = r.integers(s_range[0], s_range[1] + 1, size=n_events)
    n = r.choice(np.asarray(n_choices), size=n_events)
    if dirs is None:
        dirs = direction_grid(16, 16)
    return [EventSpec(int(s[i]), int(n[i]), i, dirs) for i in range(n_events)]


def poisson_arrivals(rate_hz: float, duration_s: float, cfg: int = 3) -> np.ndarray:
    """Open-loop arrival times (s): exponential gaps at ``rate_hz`` over ``duration_s``."""
    r = rng(cfg, STREAM_ARRIVALS)
    n = int(rate_hz * duration_s * 1.2) + 16
    t = np.cumsum(r.exponential(1.0 / rate_hz, size=n))
    return t[t < duration_s]


# ---------------------------------------------------------------------------
# Station layout and plane-wave events (for the reconstruction loop)
# ---------------------------------------------------------------------------

C_M_PER_NS = 0.299792458


def station_positions(n: int = 124, area_km2: float = 6.0) -> np.ndarray:
    """[n][2] (east, north) metres of n stations on a hexagonal grid covering
    about area_km2 (AERA: 124 stations over about 6 km^2), centred on 0."""
    a = np.sqrt(2.0 * area_km2 * 1e6 / (np.sqrt(3.0) * n))
    rings = int(np.ceil(np.sqrt(n))) + 2
    pts = []
    for i in range(-rings, rings + 1):
        for j in range(-rings, rings + 1):
            pts.append((a * (i + 0.5 * j), a * (np.sqrt(3.0) / 2.0) * j))
    pts = np.array(pts)
    r = np.hypot(pts[:, 0], pts[:, 1])
    order = np.lexsort((np.arctan2(pts[:, 1], pts[:, 0]), np.round(r, 6)))
    return np.ascontiguousarray(pts[order[:n]])


def plane_wave_delays(positions: np.ndarray, zen_deg: float, az_deg: float, fs_hz: int = FS_HZ) -> np.ndarray:
    """Arrival-time offsets in samples of a plane wave from (zen, az) at ground
    positions: t = -(n . x) / c with n the unit vector towards the source."""
    th, ph = np.deg2rad(zen_deg), np.deg2rad(az_deg)
    nx, ny = np.sin(th) * np.cos(ph), np.sin(th) * np.sin(ph)
    t_ns = -(nx * positions[:, 0] + ny * positions[:, 1]) / C_M_PER_NS
    return t_ns * fs_hz / 1e9


def plane_wave_traces(positions: np.ndarray, n: int, zen_deg: float, az_deg: float, cfg: int, event: int = 0,
                      dtype=np.float64, noise_sigma: float = 1.0, amp_range=(5.0, 20.0)):
    """Voltage traces [S][2][N] whose in-band pulses arrive as a plane wave from
    (zen, az), centred on sample N/2, plus Gaussian noise.  Returns (traces,
    true arrival samples [S])."""
    r = rng(cfg, STREAM_TRACES, 1000 + event)
    s = len(positions)
    t0 = n / 2.0 + plane_wave_delays(positions, zen_deg, az_deg)
    amp = r.uniform(amp_range[0], amp_range[1], size=(s, 2))
    v = r.standard_normal((s, 2, n)) * noise_sigma + pulse(n, np.broadcast_to(t0[:, None], (s, 2)), amp)
    return np.ascontiguousarray(v.astype(dtype)), t0


# ---------------------------------------------------------------------------
# Counter-based trace stream for workloads too large to generate on the host
# (10 000 events x 124 stations x 2 x 4096 float32 samples = 40.6 GB).  The
# same definition is implemented here (numpy, for the sampled events the
# oracle checks) and as a device kernel (csrc/au_synth.hip, for the whole
# stream); every step is integer arithmetic or a single IEEE float32
# operation, so both give bit-identical traces.
#
#   r = Philox4x32-10(counter, key)  (Salmon, Moraes, Dror, Shaw, "Parallel
#       random numbers: as easy as 1, 2, 3", SC'11): 10 rounds of
#       (L0, R0, L1, R1) <- (hi(M1 R1) ^ L1... see philox4x32 below), the
#       key bumped by the Weyl constants between rounds;
#   key = (seed, 0x7733);
#   noise[n] = (sum of four 22-bit uniforms of r(counter = (n, 2 s + c, e, 0))
#              - 2) * f32(sqrt(3))   (Irwin-Hall: mean 0, variance 1, exact sums);
#   per (e, s): t0 = r(0, s, e, 1)[0] mod N (integer sample), per (e, s, c):
#   A = 5 + 15 u, u = 24-bit uniform of r(0, 2 s + c, e, 2)[0];
#   V[e][s][c][n] = noise[n] + A * D[(n - t0) mod N], D the unit-amplitude
#   in-band pulse (Dirichlet kernel of the 30-80 MHz bins, float32 table).
# ---------------------------------------------------------------------------
PHILOX_M = (0xD2511F53, 0xCD9E8D57)
PHILOX_W = (0x9E3779B9, 0xBB67AE85)
STREAM_KEY1 = 0x7733


def philox4x32(c0, c1, c2, c3, k0, k1):
    """Philox4x32-10 of uint32 counter words (numpy arrays, broadcast) and a key; returns four uint32 arrays."""
    c0, c1, c2, c3 = (np.asarray(x, dtype=np.uint64) & 0xFFFFFFFF for x in (c0, c1, c2, c3))
    k0 = np.uint64(k0 & 0xFFFFFFFF)
    k1 = np.uint64(k1 & 0xFFFFFFFF)
    m0, m1 = np.uint64(PHILOX_M[0]), np.uint64(PHILOX_M[1])
    mask = np.uint64(0xFFFFFFFF)
    for rnd in range(10):
        if rnd:
            k0 = (k0 + np.uint64(PHILOX_W[0])) & mask
            k1 = (k1 + np.uint64(PHILOX_W[1])) & mask
        p0 = m0 * c0
        p1 = m1 * c2
        hi0, lo0 = p0 >> np.uint64(32), p0 & mask
        hi1, lo1 = p1 >> np.uint64(32), p1 & mask
        c0, c1, c2, c3 = hi1 ^ c1 ^ k0, lo1, hi0 ^ c3 ^ k1, lo0
    return tuple(x.astype(np.uint32) for x in (c0, c1, c2, c3))


def dirichlet_table(n: int) -> np.ndarray:
    """Unit-amplitude in-band pulse D[m] = (1/|K|) sum_{k in K} cos(2 pi k m / n), float32."""
    return pulse(n, np.zeros(()), np.ones(()))[...].astype(np.float32)


def stream_traces(events, n_st: int, n: int, seed: int = 7733, stations=None) -> np.ndarray:
    """Traces [len(events)][S][2][N] float32 of the counter-based stream (see above); with ``stations``
    (a list of station indices) only those, [len(events)][len(stations)][2][N]."""
    ev = np.asarray(events, dtype=np.int64).reshape(-1)
    st = list(range(n_st)) if stations is None else [int(x) for x in stations]
    d = dirichlet_table(n)
    sqrt3 = np.float32(np.sqrt(3.0))
    out = np.empty((len(ev), len(st), 2, n), dtype=np.float32)
    smp = np.arange(n, dtype=np.uint64)
    for i, e in enumerate(ev):
        for si, s in enumerate(st):
            t0 = int(philox4x32(0, s, e, 1, seed, STREAM_KEY1)[0]) & (n - 1)
            for c in range(2):
                r = philox4x32(smp, 2 * s + c, e, 0, seed, STREAM_KEY1)
                u = [(x >> np.uint32(10)).astype(np.float32) * np.float32(2.0 ** -22) for x in r]
                noise = (((u[0] + u[1]) + (u[2] + u[3])) - np.float32(2.0)) * sqrt3
                ua = np.float32(int(philox4x32(0, 2 * s + c, e, 2, seed, STREAM_KEY1)[0]) >> 8) * np.float32(2.0 ** -24)
                a = np.float32(np.float32(5.0) + np.float32(np.float32(15.0) * ua))
                idx = (np.arange(n) - t0) & (n - 1)
                out[i, si, c] = noise + a * d[idx]
    return out


_synth_lib = None


def synth_lib():
    """The device generator library (built beside the unfolding library)."""
    global _synth_lib
    if _synth_lib is None:
        import ctypes as C
        import os
        path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libausynth.so")
        if not os.path.exists(path):
            raise RuntimeError("libausynth.so is not built; run __graft_entry__.build()")
        lib = C.CDLL(path)
        lib.ausynth_traces.restype = C.c_int32
        lib.ausynth_traces.argtypes = [C.c_void_p, C.c_int32, C.c_int32, C.c_int32, C.c_int32, C.c_uint32,
                                       C.c_void_p, C.c_void_p]
        _synth_lib = lib
    return _synth_lib


def device_stream_traces(out, event0: int, n_events: int, n_st: int, n: int, seed: int = 7733, stream=None):
    """Fill the device tensor out [n_events][S][2][N] float32 with events event0 .. event0 + n_events - 1 of
    the counter-based stream (the same values as stream_traces)."""
    import ctypes as C
    import torch
    assert out.is_cuda and out.dtype == torch.float32 and out.is_contiguous()
    assert out.numel() == n_events * n_st * 2 * n
    d = torch.from_numpy(dirichlet_table(n)).to(out.device)
    st = torch.cuda.current_stream() if stream is None else stream
    rc = synth_lib().ausynth_traces(C.c_void_p(out.data_ptr()), int(n_events), int(event0), int(n_st), int(n),
                                    int(seed) & 0xFFFFFFFF, C.c_void_p(d.data_ptr()), C.c_void_p(st.cuda_stream))
    if rc != 0:
        raise RuntimeError("ausynth_traces failed with %d" % rc)
    torch.cuda.current_stream().synchronize() if stream is None else st.synchronize()
    return out
