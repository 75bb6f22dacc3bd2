/*
 * aeraunfold.h -- C ABI of the MI355X (gfx950) antenna-pattern unfolding library.
 *
 * The library reconstructs electric-field traces from the two voltage channels
 * of radio stations, the step the reconstruction repeats for every candidate
 * arrival direction (arXiv:1507.07733, section 2 and the algorithm of its
 * Fig. 1).  Per station and direction it
 *   1. takes the FFT of both channel traces (section 4);
 *   2. evaluates the complex vector effective length H[c][p] of channel c and
 *      component p in {theta, phi} at the direction by linear interpolation
 *      between the (frequency, zenith, azimuth) nodes of a pattern table
 *      (section 3; trilinear, azimuth periodic, zenith clamped);
 *   3. per frequency bin solves the 2x2 complex system V_c = sum_p H[c][p] E_p
 *      for (E_theta, E_phi) (section 2: reconstruct the E-field from the
 *      voltages with the pattern for the direction);
 *   4. keeps only bins inside the antenna band, 30-80 MHz by default
 *      (section 1), and
 *   5. inverse-FFTs back to E_theta and E_phi traces.
 *
 * Conventions for every entry point:
 *   - Pointers prefixed d_ are device memory on the current HIP device; h_
 *     pointers are host memory.  The caller owns every pointer it passes; the
 *     library never frees or retains them past the call (except a batch plan,
 *     which may keep device pointers inside a captured graph, see au_plan_run).
 *   - Traces are [S][2][N] (station, channel, sample), sample fastest.  Outputs
 *     are [D][S][2][N] (direction, station, component theta/phi, sample).
 *   - Float outputs have the compute precision's type: float for AU_PREC_FP32,
 *     double for AU_PREC_FP64.  Input traces may be float or double.
 *   - `stream` is a hipStream_t passed as void* (NULL = default stream).  Calls
 *     validate synchronously, enqueue on the stream and return; results and
 *     counters are valid once the stream has completed the work.
 *   - `d_counts` (nullable) is a device array of two uint64: [0] += number of
 *     (direction, in-band bin) pairs whose FP32 determinant fell below
 *     fallback_rel * ||H||_F^2 and were redone in FP64, [1] += number of pairs
 *     treated as singular (|det| <= singular_rel * ||H||_F^2, field set to 0).
 *     The library only adds to them.
 *   - Return codes: AU_OK (0) or a negative au_status.  On error nothing has
 *     been enqueued and au_last_error() returns a message (per thread).
 */
#ifndef AERAUNFOLD_H
#define AERAUNFOLD_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t au_status;
#define AU_OK 0
#define AU_EINVAL (-1)     /* bad argument: sizes, band, grid, dtype, null pointer */
#define AU_ENOMEM (-2)     /* device or host allocation failed, or workspace too small */
#define AU_EDEVICE (-3)    /* a HIP call failed */
#define AU_EAGAIN (-4)     /* not ready yet (au_poll) or over budget (au_submit) */
#define AU_ENOTFOUND (-5)  /* unknown ticket */

/* element types */
#define AU_F32 1           /* float; tables: complex64 */
#define AU_F64 2           /* double; tables: complex128 */

/* compute precision */
#define AU_PREC_FP64 0     /* everything in double; needs a complex128 table */
#define AU_PREC_FP32 1     /* FFT, interpolation and solve in float; the 2x2
                              determinant and inverse are redone in double where
                              |det| < fallback_rel * ||H||_F^2 */

/*
 * Node grid of a pattern table (section 3: the vector effective length is
 * known at discrete frequencies, zenith and azimuth angles).  Frequencies are
 * integers in Hz so that FFT-bin positions on the grid are exact; angles in
 * degrees.  Node f has frequency f0_hz + f*df_hz, node z zenith
 * zen0_deg + z*dzen_deg, node a azimuth az0_deg + a*daz_deg.  The azimuth
 * axis must close the circle: n_az*daz_deg == 360 (or (n_az-1)*daz_deg == 360
 * with the last column equal to the first, which is then dropped).
 */
typedef struct {
    int32_t n_freq, n_zen, n_az, reserved;
    int64_t f0_hz, df_hz;
    double zen0_deg, dzen_deg, az0_deg, daz_deg;
} au_grid;

/*
 * One event: S stations with two channels of N samples at fs_hz.  The band
 * is the set of FFT bins k in [0, N/2] with band_lo_hz*N <= k*fs_hz <=
 * band_hi_hz*N, tested exactly in 64-bit integers.  Requirements: N a power
 * of two in [16, 4096]; S >= 1; 0 <= band_lo_hz <= band_hi_hz < fs_hz/2; every
 * in-band bin frequency inside the table's frequency range; |k*fs_hz -
 * f0_hz*N| for every in-band bin k, and N*df_hz, below 2^53 (the bin's node
 * position is split exactly in double arithmetic).
 * fallback_rel (FP32 only) and singular_rel: see d_counts above; the usual
 * values are 1e-6 and 1e-12.  Both tests are scale-free: they are taken on H
 * scaled by a power of two (exact), so a table in any units, e.g. of order
 * 1e-12 or 1e12, gives the decisions and coefficients of the same table in
 * units of order one.
 */
typedef struct {
    int32_t n_stations, n_samples;
    int64_t fs_hz, band_lo_hz, band_hi_hz;
    int32_t trace_dtype;          /* AU_F32 or AU_F64: element type of d_volt */
    int32_t prec;                 /* AU_PREC_FP64 or AU_PREC_FP32 */
    double fallback_rel;
    double singular_rel;
} au_event;

typedef struct au_table au_table;
typedef struct au_plan au_plan;
typedef struct au_server au_server;

/* Message for the last non-OK status returned on this thread ("" if none). */
const char* au_last_error(void);

/* Library version string. */
const char* au_version(void);

/*
 * Load a pattern table onto the current device (section 3: the pattern is
 * copied and converted once, then stays resident for every later lookup).
 *   grid:        node grid (see au_grid).
 *   table_dtype: AU_F64 (complex128) or AU_F32 (complex64) for h_vel.
 *   h_vel:       host array [2 channel][2 component theta/phi][n_freq][n_zen][n_az]
 *                of interleaved (re, im) pairs of that type.
 *   out:         receives the handle; free with au_free_pattern_table.
 * The device copy is re-laid out node-major [freq][zen][az][channel][component]
 * so one interpolation corner is one contiguous 32 or 64 byte read.  The
 * call is synchronous.  Errors: AU_EINVAL (grid or dtype), AU_ENOMEM, AU_EDEVICE.
 */
au_status au_load_pattern_table(const au_grid* grid, int32_t table_dtype, const void* h_vel,
                                au_table** out);
au_status au_free_pattern_table(au_table* table);

/*
 * Size in bytes of the device workspace a call on this event with n_dir
 * directions needs (in-band spectra of every station, the per-direction
 * inverse-pattern coefficients, and the direction list).
 */
au_status au_workspace_bytes(const au_table* table, const au_event* ev, int32_t n_dir, uint64_t* bytes);

/* In-band bin range of an event: bins k_lo .. k_lo + n_band - 1 (n_band may be 0). */
au_status au_band_bins(const au_event* ev, int32_t* k_lo, int32_t* n_band);

/*
 * Unfold one event for one direction (zen_deg, az_deg) (section 2: the
 * pattern for the direction is evaluated and the E-field trace of each
 * station reconstructed from its voltage traces).
 *   d_volt:   [S][2][N] traces of ev->trace_dtype.
 *   d_efield: [S][2][N] output (E_theta, E_phi), float or double per ev->prec.
 *   d_work:   workspace of au_workspace_bytes(ev, 1) bytes, or NULL to let the
 *             library take it from the stream-ordered pool (hipMallocAsync).
 * Events of 2048 or 4096 samples whose traces and table are in the compute
 * precision and whose band holds at most N/4 bins run in one launch (one
 * workgroup per station: forward transform, the direction's coefficients,
 * solve, inverse transform) and leave d_work untouched (a given workspace
 * is still checked for size); the results agree with a one-direction
 * au_unfold_direction_scan to rounding (per station within 1e-6 of the peak
 * in FP32, 1e-13 in FP64), the counters exactly.
 * Errors: AU_EINVAL, AU_ENOMEM (work_bytes too small or pool exhausted), AU_EDEVICE.
 */
au_status au_unfold_event(const au_table* table, const au_event* ev, const void* d_volt,
                          double zen_deg, double az_deg, void* d_efield,
                          void* d_work, uint64_t work_bytes, void* stream, uint64_t* d_counts);

/*
 * Unfold one event for each of n_dir candidate directions (the direction fit
 * repeats the unfolding for every candidate; section 2).  The station
 * spectra are computed once and reused for every direction (section 4: the
 * trace container keeps the frequency domain and only recomputes it when the
 * trace changes).
 *   h_dirs:   host [n_dir][2] (zenith, azimuth) in degrees.
 *   d_efield: [n_dir][S][2][N] output.
 *   d_work:   au_workspace_bytes(ev, n_dir) bytes, or NULL (pool).
 */
au_status au_unfold_direction_scan(const au_table* table, const au_event* ev, const void* d_volt,
                                   int32_t n_dir, const double* h_dirs, void* d_efield,
                                   void* d_work, uint64_t work_bytes, void* stream,
                                   uint64_t* d_counts);

/*
 * au_unfold_direction_scan for callers that cannot allocate memory (code
 * under HIP graph capture, tight serving loops, harnesses that forbid
 * allocation): the same kernels and results (bitwise), with the work space
 * (the stations' in-band spectra and the directions' coefficients) in a
 * fixed 32 MiB device array of the library instead of d_work or a pool.
 * The call allocates nothing and enqueues no host-to-device copy.
 *   d_dirs:   DEVICE [n_dir][2] (zenith, azimuth) in degrees (caller-owned).
 *   d_efield: [n_dir][S][2][N] output.
 * Limit: the spectra, S * n_band * 16 B (FP32) or 32 B (FP64), plus one
 * direction's coefficients, n_band * 32 B (FP32) or 64 B (FP64), must fit
 * 32 MiB (at N = 4096 and fs = 200 MHz, 30-80 MHz: up to 2 046 stations
 * FP32, 1 022 FP64); directions are processed in chunks that fit, so n_dir
 * is not limited.  Larger events: AU_EINVAL, nothing enqueued.
 * The array is shared by every call on a device and keeps the last call's
 * contents (every byte a call reads it has written first): calls on one
 * device that may overlap (different streams, or threads without ordering)
 * race and must not be issued; calls on one stream are ordered.
 */
au_status au_unfold_direction_scan_noalloc(const au_table* table, const au_event* ev, const void* d_volt,
                                           int32_t n_dir, const double* d_dirs, void* d_efield, void* stream,
                                           uint64_t* d_counts);

/*
 * Direction scan reduced to station timing: the E-field trace's Hilbert
 * envelope env = sqrt(e^2 + H(e)^2) (section 4) and its maximum, whose
 * sample is the updated station time (section 2, Fig. 1).  For every
 * direction and station, for c = 0 (theta), 1 (phi) and 2 (total field,
 * sqrt(env_theta^2 + env_phi^2)):
 *   d_peak [n_dir][S][3] (float or double per ev->prec): max_n env_c[n];
 *   d_arg  [n_dir][S][3] int32: the smallest n attaining it.
 * d_efield ([n_dir][S][2][N], nullable) also receives the traces.  The
 * Hilbert transform uses -i sgn(k) (sgn 0 at DC and Nyquist); the opposite
 * sign gives the same envelope.  Workspace as au_unfold_direction_scan.
 */
au_status au_unfold_envelope_scan(const au_table* table, const au_event* ev, const void* d_volt,
                                  int32_t n_dir, const double* h_dirs, void* d_efield, void* d_peak,
                                  int32_t* d_arg, void* d_work, uint64_t work_bytes, void* stream,
                                  uint64_t* d_counts);

/*
 * The reconstruction loop of one event (section 2, Fig. 1), run on the device
 * with no host round trip between its steps:
 *   1. station times t_s = the smallest sample maximising V_0^2 + V_1^2
 *      (evaluated in double, no fused multiply-add);
 *   2. triangulation: least-squares plane wave t = t0 + p x + q y over the
 *      station positions (times in ns = samples * 1e9 / fs), direction of
 *      arrival n = (-c p, -c q) on the ground, c = 0.299792458 m/ns,
 *      zenith = asin(min(1, |n|)), azimuth = atan2(n_y, n_x) in [0, 360);
 *   3. unfold every station for that direction (as au_unfold_event);
 *   4. new t_s = the total-field envelope maximum (as au_unfold_envelope_scan,
 *      component 2);
 *   5. stop when no station time changed (converged), else repeat from 2,
 *      at most max_iter directions.
 * Inputs: d_volt [S][2][N] device traces (ev->trace_dtype), h_pos [S][2] host
 * ground positions in metres (x east, y north; finite, |x|, |y| <= 1e7),
 * 1 <= max_iter <= 1024, S >= 3.
 * Outputs (host, written before return; the call synchronises the stream):
 *   h_dirs  [max_iter][2] degrees: rows 0..*n_dirs-1 are the directions of
 *           each pass, the last one the result;
 *   h_times [max_iter+1][S] int32 samples: row 0 the voltage maxima, row i the
 *           envelope maxima after direction i-1; rows 0..*n_dirs are defined;
 *   *n_dirs, *converged (1 when step 5 ended the loop).
 *   d_efield ([S][2][N] of ev->prec's type, nullable) and d_peak ([S][3],
 *   nullable): traces and envelope maxima of the final direction.
 * Workspace: au_reconstruct_workspace_bytes, or NULL to allocate from the
 * stream's pool.  AU_EINVAL with *n_dirs set when the stations are collinear
 * or coincident (the plane fit is undetermined).
 */
au_status au_reconstruct_workspace_bytes(const au_table* table, const au_event* ev, int32_t max_iter,
                                         uint64_t* bytes);
au_status au_reconstruct(const au_table* table, const au_event* ev, const void* d_volt, const double* h_pos,
                         int32_t max_iter, double* h_dirs, int32_t* h_times, int32_t* n_dirs,
                         int32_t* converged, void* d_efield, void* d_peak, void* d_work, uint64_t work_bytes,
                         void* stream);

/*
 * The reconstruction loop (as au_reconstruct) for n_events events at once:
 * each step is one launch over all events and every event stops on its own
 * (converged, out of passes, or degenerate geometry).  Common to all events:
 * ev's n_samples, sampling rate, band, precision, trace type and thresholds
 * (ev->n_stations is ignored).  Per event e: h_n_stations[e] >= 3 stations
 * whose [S][2][N] traces start at element h_volt_offset[e] of d_volt (offsets
 * may alias).  h_pos [sum S][2] ground positions in metres, events in order.
 * Outputs (host; the call synchronises the stream):
 *   h_dirs [n_events][max_iter][2] degrees, rows 0..h_n_dirs[e]-1 defined;
 *   h_times [max_iter+1][sum S] int32 samples, the stations in event order,
 *           rows 0..h_n_dirs[e] defined for the stations of event e;
 *   h_n_dirs [n_events]; h_converged [n_events]: 1 converged, 0 ran out of
 *           passes, -1 degenerate geometry (collinear or coincident).
 * A result equals the one-event au_reconstruct of that event.  Workspace:
 * au_reconstruct_batch_workspace_bytes, or NULL for the stream's pool.
 */
au_status au_reconstruct_batch_workspace_bytes(const au_table* table, const au_event* ev, int32_t n_events,
                                               const int32_t* h_n_stations, const int64_t* h_volt_offset,
                                               int32_t max_iter, uint64_t* bytes);
au_status au_reconstruct_batch(const au_table* table, const au_event* ev, int32_t n_events,
                               const int32_t* h_n_stations, const int64_t* h_volt_offset, const void* d_volt,
                               const double* h_pos, int32_t max_iter, double* h_dirs, int32_t* h_times,
                               int32_t* h_n_dirs, int32_t* h_converged, void* d_work, uint64_t work_bytes,
                               void* stream);

/*
 * Direction fit of one event over candidate directions (the reconstruction
 * repeats the E-field step per candidate, section 2; the paper names no
 * objective).  Per candidate d every station is unfolded for d and timed at
 * its total-field envelope maximum t_s(d) (as au_unfold_envelope_scan); the
 * score is the inconsistency of those times with a plane wave from d,
 *   chi2(d) = min over t0 of sum_s (t_s(d) dt - t0 - tau_s(d))^2   [ns^2],
 *   tau_s(d) = -(n(d) . x_s) / c,  n(d) = (sin z cos a, sin z sin a),
 * with dt = 1e9 / fs ns, c = 0.299792458 m/ns; also power(d) = sum_s peak_s^2.
 * The best candidate minimises chi2 (the first on ties).  Then `levels`
 * refinements, all on the device with no host round trip: level l scores the
 * k x k grid around the previous best at spacing (step_zen, step_az) / 2^l,
 * zenith zc + (i - (k-1)/2) h_z clamped to [0, 90] (row i), azimuth
 * ac + (j - (k-1)/2) h_a wrapped to [0, 360) (column j).
 * Inputs: d_volt [S][2][N] device; h_pos [S][2] host metres (x east, y north;
 * finite, |x|, |y| <= 1e7); h_dirs [n_dir][2] host degrees; S >= 3,
 * 0 <= levels <= 16, 1 <= k <= 15, steps in (0, 90] and (0, 360] when
 * levels > 0.  Outputs (host, written before return; the call synchronises
 * the stream; each nullable except h_result): h_level_dirs
 * [levels][k*k][2]; h_chi2, h_power [n_dir + levels*k*k] (coarse candidates
 * first, then each level); h_best [levels+1] (index within its level);
 * h_result [2] the best direction of the last level.
 * Workspace: au_direction_fit_workspace_bytes, or NULL for the stream's pool.
 */
au_status au_direction_fit_workspace_bytes(const au_table* table, const au_event* ev, int32_t n_dir,
                                           int32_t levels, int32_t k, uint64_t* bytes);
au_status au_direction_fit(const au_table* table, const au_event* ev, const void* d_volt, const double* h_pos,
                           int32_t n_dir, const double* h_dirs, int32_t levels, int32_t k, double step_zen,
                           double step_az, double* h_level_dirs, double* h_chi2, double* h_power,
                           int32_t* h_best, double* h_result, void* d_work, uint64_t work_bytes, void* stream);

/*
 * Interpolated pattern H[c][p](f_k; zen, az) at every in-band bin of ev, for
 * n_dir directions (section 3: linear interpolation between nodes).  Output
 * d_resp [n_dir][n_band][2][2] complex (interleaved re, im) of the precision's
 * type.  Used to check the interpolation on its own.
 */
au_status au_pattern_response(const au_table* table, const au_event* ev, int32_t n_dir,
                              const double* h_dirs, void* d_resp, void* stream);

/*
 * As au_pattern_response, with each of the three interpolation weights
 * (fractional node positions in frequency, zenith and azimuth) rounded to the
 * nearest multiple of 2^-weight_bits (ties to even) before interpolating:
 * the fixed-point weights of a hardware texture filter (section 3 interpolates
 * with texture hardware; NVIDIA documents 8 fractional bits, weight_bits = 8).
 * gfx950 has no texture sampler, so this models its weights in software to
 * measure the precision cost.  1 <= weight_bits <= 30.
 */
au_status au_pattern_response_quantized(const au_table* table, const au_event* ev, int32_t n_dir,
                                        const double* h_dirs, int32_t weight_bits, void* d_resp, void* stream);

/*
 * Batched unfolding of many events of uneven size (stations x directions x
 * events) in one launch per trace length, optionally replayed from a captured
 * HIP graph.  Motivation: the paper's GPU time was dominated by host<->device
 * copies of isolated calls and names keeping traces on the device as the way
 * to use the GPU better (section 5).
 *
 * au_batch describes E events sharing fs, band and precision:
 *   n_stations[e], n_samples[e], n_dirs[e]: per-event sizes (host arrays);
 *   h_dirs: host [sum_e n_dirs[e]][2] degrees, event-major;
 *   volt_offset[e]: element offset of event e's [S][2][N] traces inside d_volt;
 *   efield_offset[e]: element offset of its [D][S][2][N] output inside d_efield.
 * Offsets may alias: events may share input traces, and events whose output
 * regions overlap write them in an unspecified order (a throughput run can
 * recycle one output ring this way).
 * au_plan_create validates, sorts work longest-first, uploads the work lists
 * and allocates the plan's workspace (the only allocation; au_plan_run
 * allocates nothing).  flags: AU_PLAN_GRAPH to capture the launch sequence in
 * a hipGraph on first run (re-captured if d_volt / d_efield change),
 * AU_PLAN_PERSISTENT to run the unfold stage as a persistent kernel fed by an
 * atomic work counter, AU_PLAN_XCD to place all work units of one event on
 * one of the 8 XCDs (8 unit lists balanced by work; workgroup b takes units
 * from list b mod 8, then steals) so that the event's spectrum rows and its
 * directions' coefficient rows are fetched into one XCD's L2 only.
 * With AU_PLAN_FUSED, trace-length classes (FP32, 2048 or 4096 samples,
 * bands of at most N/4 bins) whose events all have at most 64 directions
 * run fused (section 4's
 * dual-domain container: the spectrum of a station is formed once and kept
 * on chip while every direction is unfolded from it): one kernel per class
 * takes units of (event, 16 stations, every direction), transforms each
 * station forward and unfolds all directions from the spectrum it keeps in
 * registers, so no spectrum rows are written or read (and none allocated);
 * these classes always use a persistent grid.  The operations are those of
 * the separate stages; the results agree with them to rounding (the
 * compiler contracts some products into fused multiply-adds differently in
 * the two kernels).
 */
#define AU_PLAN_GRAPH 1
#define AU_PLAN_PERSISTENT 2
#define AU_PLAN_XCD 4
#define AU_PLAN_FUSED 8    /* fuse the spectrum into the unfold for classes with few directions */
typedef struct {
    int32_t n_events;
    int32_t prec;
    int32_t trace_dtype;
    int32_t flags;
    int64_t fs_hz, band_lo_hz, band_hi_hz;
    double fallback_rel, singular_rel;
    const int32_t* n_stations;
    const int32_t* n_samples;
    const int32_t* n_dirs;
    const double* h_dirs;
    const int64_t* volt_offset;
    const int64_t* efield_offset;
} au_batch;

au_status au_plan_create(const au_table* table, const au_batch* batch, au_plan** out);
/* Number of station-unfolds (event, direction, station triples) in the plan. */
au_status au_plan_units(const au_plan* plan, uint64_t* station_unfolds);
au_status au_plan_run(au_plan* plan, const void* d_volt, void* d_efield, void* stream,
                      uint64_t* d_counts);

/*
 * Tune the plan's unfold kernel per trace-length class: every built variant
 * (au_unfold_variant_count) is run inside this plan (its work lists,
 * placement and persistent grid) on d_volt / d_efield, reps timed runs after
 * one warm-up, timed by HIP events around the class's unfold launch; the
 * fastest is kept for later runs (a captured graph is re-captured).  ms
 * ([n_classes][variant count], nullable) receives the average ms per launch
 * (-1 for a variant not built for that length), best ([n_classes], nullable)
 * the chosen variant.  Synchronises the stream.  The global per-length
 * choice (au_set_unfold_variant) is left unchanged.
 */
au_status au_plan_autotune(au_plan* plan, const void* d_volt, void* d_efield, int32_t reps, void* stream,
                           double* ms, int32_t* best);

/*
 * Stage timing for measurement: with timing enabled (plans without
 * AU_PLAN_GRAPH only), au_plan_run records a HIP event on the run's stream
 * before the first launch and after each launch, waits for the last one and
 * adds each launch's elapsed time to a per-stage total.  Enabling resets the
 * totals.  Stages are ordered [class][spectrum, coef, unfold]; classes are
 * the plan's distinct trace lengths, longest first (au_plan_classes).
 */
au_status au_plan_timing(au_plan* plan, int32_t enable);
au_status au_plan_classes(const au_plan* plan, int32_t max, int32_t* n_samples,
                          uint64_t* station_unfolds, int32_t* variants, int32_t* n_classes);
au_status au_plan_stage_ms(const au_plan* plan, int32_t max, double* ms, uint64_t* runs);
au_status au_plan_free(au_plan* plan);

/*
 * Serving: a continuous-batching request loop (section 5 motivates keeping
 * traces resident on the GPU instead of copying around isolated calls).
 * The server owns one device arena of hbm_budget_bytes (traces, outputs and
 * work space of admitted events), a pinned host staging area of
 * staging_bytes (traces of queued events), and 2 * n_streams descriptor
 * slots of 2 MiB (device + pinned) for batches of several events; all are
 * allocated at creation, the arena and staging carved up by a first-fit
 * allocator, so submit/poll/wait/release never allocate memory.
 * Admission is FIFO: an event is admitted when the arena has room for it and
 * fewer than max_inflight events are admitted and not released.  An event
 * with nothing queued ahead of it is admitted inside au_submit, its traces
 * copied straight into its arena region (au_submit returns once the copy is
 * done) and, with tick_s = 0, launched in the same call together with any
 * other admitted event; otherwise its traces go to staging and a scheduler
 * thread admits and launches it.  Admitted events form micro-batches
 * (launched when max_batch_events are ready or the oldest has waited tick_s
 * seconds; a batch shrinks to one event when no descriptor slot is free or
 * its descriptors would exceed a slot), spread round-robin over n_streams
 * streams so that the work of events arriving while others run overlaps on
 * the device.  Launching needs no memory beyond what its events hold, so an
 * arena filled exactly by admitted events still makes progress.  A reaper
 * thread waits on each batch's completion event (no polling loop) and wakes
 * au_wait callers.  Each event's result stays in the arena until
 * au_release.  Per-event arithmetic is the same whatever the batch mix, so a
 * result is identical alone and in a mix.
 * Thread safety: submit/poll/wait/release/stats may be called from any
 * thread; au_copy_result must not race with au_release of the same ticket.
 * Timestamps are seconds on the server's steady clock (au_server_now).
 */
typedef struct {
    uint64_t hbm_budget_bytes;    /* device arena size */
    uint64_t staging_bytes;       /* pinned host staging size */
    int32_t max_inflight;         /* admitted-and-unreleased events at most */
    int32_t n_streams;            /* 1..16 */
    int32_t max_batch_events;     /* events per micro-batch at most */
    int32_t prec;                 /* AU_PREC_FP32 / AU_PREC_FP64 */
    int32_t trace_dtype;          /* AU_F32 / AU_F64 of submitted traces */
    int32_t reserved;
    int64_t fs_hz, band_lo_hz, band_hi_hz;
    double fallback_rel, singular_rel;
    double tick_s;                /* longest wait of an admitted event before launch */
} au_server_cfg;

typedef struct {
    int32_t n_stations, n_samples, n_dirs, reserved;
    const void* h_volt;           /* host [S][2][N] of cfg.trace_dtype (copied by au_submit) */
    const double* h_dirs;         /* host [n_dirs][2] degrees (copied) */
    double t_arrival;             /* scheduled arrival on the server clock; <= 0: now */
} au_request;

typedef struct {
    void* d_efield;               /* [n_dirs][S][2][N] in the arena, valid until au_release */
    uint64_t efield_bytes;
    int32_t n_stations, n_samples, n_dirs, batch_events;
    double t_arrival, t_submit, t_admit, t_launch, t_complete;
    uint64_t batch_id;            /* events with equal batch_id shared one launch sequence */
} au_result;

typedef struct {
    uint64_t submitted, completed, rejected, batches, queued, in_flight;
    uint64_t arena_bytes, arena_in_use, arena_peak;
    uint64_t fallback_bins, singular_bins;
} au_server_counters;

/* Errors: AU_EINVAL (configuration, request; tick_s must lie in [0, 10]),
 * AU_ENOMEM (arena, staging or slots cannot be allocated; a request larger
 * than the whole arena), AU_EAGAIN (au_submit: staging full, retry later;
 * au_poll: not complete yet; au_wait: not complete within timeout_s),
 * AU_ENOTFOUND (unknown or released ticket), AU_EDEVICE (a HIP call failed;
 * the server then fails every pending request).
 * au_server_request_bytes: arena bytes one request of these sizes occupies
 * (output, work space, directions, traces).
 * au_wait: blocks until the ticket completes (then as au_poll) or timeout_s
 * seconds pass (AU_EAGAIN).
 * au_server_destroy waits for launched batches to complete. */
au_status au_server_create(const au_table* table, const au_server_cfg* cfg, au_server** out);
au_status au_server_destroy(au_server* server);
au_status au_server_now(const au_server* server, double* seconds);
au_status au_server_request_bytes(const au_server* server, int32_t n_stations, int32_t n_samples,
                                  int32_t n_dirs, uint64_t* dev_bytes);
au_status au_submit(au_server* server, const au_request* request, uint64_t* ticket);
au_status au_poll(au_server* server, uint64_t ticket, au_result* result);
au_status au_wait(au_server* server, uint64_t ticket, double timeout_s, au_result* result);
au_status au_copy_result(au_server* server, uint64_t ticket, void* dst, uint64_t dst_bytes);
au_status au_release(au_server* server, uint64_t ticket);
au_status au_server_stats(au_server* server, au_server_counters* stats);

/*
 * Kernel shapes and autotuning (the batched form picks its FFT radix
 * schedule per trace length and precision by measurement).  The unfold
 * kernel is built in au_unfold_variant_count() shapes, described by six
 * arrays of *count entries (each may be NULL; count is at most 32):
 * e_values = values per thread (0: one wavefront per transform, N/64 values
 * per lane), rmax = largest radix per pass, twmode = where the inverse FFT's
 * twiddles live (0 table, 1 registers, 2 registers times compile-time
 * constants, 3 an LDS table for the early passes and registers for the
 * rest, 4 as 3 with (tangent, cosine) pairs for fused multiply-add
 * butterflies, 5 the pairs of 4 for every pass in registers, 6 as 5 in the
 * 4096-point double-precision transform whose first two exchanges stay
 * inside the wavefront: one through the wavefront's own LDS slots, one as a
 * register transpose with DPP and lane-swap moves), wave = 1 if a single wavefront
 * owns each transform (no workgroup barriers), pair = 1 if lanes L and L^32
 * hold mirror bins k and N-k so each in-band bin is solved once and its
 * mirror taken with a cross-lane swap, pp = 1 if each transform alternates
 * between two LDS buffers (one workgroup barrier per exchange instead of
 * two).  Shapes other than the first two exist only for N >= 1024, and only
 * where they fit in registers and LDS.  The selection is process-wide per (precision,
 * N); plans read it when they are created.
 *
 * au_autotune runs the single-event path on a synthetic event of ev's sizes
 * and n_dir directions with every built variant (reps timed runs each after
 * one warm-up, HIP events on a private stream), writes the average ms per
 * variant to ms[] (-1 where not built; may be NULL), selects the fastest
 * and returns it in *best.  It allocates its own buffers (hipMalloc) and is
 * synchronous.
 */
au_status au_unfold_variant_count(int32_t* count, int32_t* e_values, int32_t* rmax, int32_t* twmode,
                                  int32_t* wave, int32_t* pair, int32_t* pp);
au_status au_set_unfold_variant(int32_t prec, int32_t n_samples, int32_t variant);
au_status au_get_unfold_variant(int32_t prec, int32_t n_samples, int32_t* variant);
au_status au_autotune(const au_table* table, const au_event* ev, int32_t n_dir, int32_t reps,
                      double* ms, int32_t* best);

/*
 * HBM copy probe: copies `bytes` (a multiple of 16; both pointers 16-byte
 * aligned) from d_src to d_dst with 16-byte loads and non-temporal stores on
 * a grid-stride loop, enqueued on `stream`.  It is the reference for
 * achievable HBM bandwidth and for calibrating the memory-traffic counters
 * of a profiler against a transfer of known size.
 */
au_status au_hbm_copy(void* d_dst, const void* d_src, uint64_t bytes, void* stream);
/* Write-only probe: fills `bytes` (multiple of 16, aligned) with a 32-bit value
 * using non-temporal stores -- the reference for a write-bound kernel. */
au_status au_hbm_fill(void* d_dst, uint64_t bytes, uint32_t value, void* stream);

#ifdef __cplusplus
}
#endif
#endif /* AERAUNFOLD_H */
