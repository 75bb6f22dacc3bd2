/*
 * oracle.c -- plain, slow FP64 CPU oracle for antenna-pattern unfolding.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path links, loads or
 * calls this file; only the test suite, the smoke check and the CPU-baseline
 * leg of the benchmark do.  It shares no code, header, table or helper with
 * the HIP library.  Build:  gcc -O2 -ffp-contract=off -fPIC -shared.
 *
 * What it computes, for one direction (theta, phi) and one station with two
 * channel voltage traces V_0, V_1 of N real samples:
 *
 *     E = IDFT_N( band(k) * H(f_k; theta, phi)^-1 * DFT_N(V) )
 *
 * - The radio reconstruction evaluates the antenna pattern for the current
 *   direction and reconstructs the E-field at each station from its two
 *   voltage channels (paper, section 2, the algorithm of Fig. 1).
 * - The pattern is the complex two-component vector effective length
 *   (theta and phi components), known at discrete frequency, zenith and
 *   azimuth nodes and linearly interpolated between them (section 3).
 *   Reading: trilinear interpolation on real and imaginary parts, azimuth
 *   periodic, zenith clamped to the grid.
 * - Reading of the unfolding: per frequency bin, V_c(f) = sum_p H_cp(f) E_p(f)
 *   with c the channel and p in {theta, phi}; it is solved by Cramer's rule.
 *   Bins whose |det| <= singular_rel * ||H||_F^2 are treated as singular:
 *   E(f) = 0 there, and they are counted.
 * - The antennas observe 30-80 MHz (section 1): bins outside the band are
 *   set to zero (ideal rectangular band, inclusive, integer test in Hz).
 * - Transforms (section 4 uses FFTs for both directions): forward with
 *   e^{-2 pi i k n / N} and no scaling, inverse with e^{+...} and 1/N.
 *   Both are a textbook iterative radix-2 Cooley-Tukey FFT; every twiddle
 *   is cos/sin of its own angle from libm, never a recurrence.
 *
 * Envelope (section 4: the envelope of a trace x is the magnitude of
 * x + i H(x), H the Hilbert transform; section 2: its maximum is the updated
 * timing of the station): H(x) = IDFT(-i sgn(k) DFT(x)), sgn(k) = +1 for
 * 0 < k < N/2, -1 for N/2 < k < N, 0 at k = 0 and N/2.  The paper's phase
 * convention is the opposite sign, which leaves the envelope unchanged.
 *
 * Reconstruction loop (section 2, Fig. 1): the first station times are the
 * maxima of the voltage traces; the direction follows from the times by
 * triangulation; the E-field is reconstructed for that direction; the
 * maximum of its envelope gives new times; repeat until converged.
 * Readings: a station's voltage maximum is the sample maximising
 * V_0^2 + V_1^2; the envelope used for timing is the total-field envelope
 * sqrt(env_theta^2 + env_phi^2); triangulation is a least-squares plane wave
 * t_s = t0 + p x_s + q y_s over ground positions (x east, y north), giving the
 * direction n = (-c p, -c q, ...) towards the source; the loop stops when a
 * set of station times repeats (a fixed point of the iteration) or after
 * max_iter directions.
 *
 * Direction fit (the reconstruction repeats the E-field step for candidate
 * directions; the paper states no objective).  Reading: for a candidate
 * direction d, every station is unfolded for d and timed at its total-field
 * envelope maximum t_s(d); the score is the timing inconsistency with a plane
 * wave from d, chi2(d) = min over t0 of sum_s (t_s(d) dt - t0 - tau_s(d))^2
 * with tau_s(d) = -(n(d) . x_s) / c in ns (the same plane-wave model as the
 * triangulation); the best candidate minimises chi2 (the first on ties).
 * Local refinement: a K x K grid around the best candidate at half the
 * previous spacing, zenith clamped to [0, 90], azimuth wrapped to [0, 360).
 *
 * Every pin of this file lives in tests/test_oracle_*.py (brute-force DFT,
 * Parseval, pure tones, exact node interpolation, multilinear
 * reproduction, azimuth wrap, exact rational 2x2 solve, band-pass and
 * round-trip reductions, dense linear map at N = 16).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef struct {
    int32_t n_freq, n_zen, n_az;
    int32_t pad_;
    int64_t f0_hz, df_hz;
    double zen0_deg, dzen_deg, az0_deg, daz_deg;
} orc_grid;

static const double ORC_PI = 3.14159265358979323846264338327950288;

/* ---------------------------------------------------------------------- */
/* FFT: iterative radix-2 decimation in time, in place.                    */
/* ---------------------------------------------------------------------- */

static int is_pow2(int64_t n) { return n >= 1 && (n & (n - 1)) == 0; }

/*
 * In-place complex DFT of length n (a power of two):
 *   out[k] = sum_j in[j] * exp(sign * 2 pi i j k / n), no scaling.
 * Returns 0, or -1 if n is not a power of two.
 */
int orc_fft(int64_t n, double* re, double* im, int sign)
{
    if (!is_pow2(n)) return -1;
    /* bit-reversal permutation */
    for (int64_t i = 1, j = 0; i < n; ++i) {
        int64_t bit = n >> 1;
        for (; j & bit; bit >>= 1) j ^= bit;
        j ^= bit;
        if (i < j) {
            double t = re[i]; re[i] = re[j]; re[j] = t;
            t = im[i]; im[i] = im[j]; im[j] = t;
        }
    }
    /* butterflies: sub-transforms of length len = 2m combine pairs m apart */
    for (int64_t len = 2; len <= n; len <<= 1) {
        int64_t m = len >> 1;
        for (int64_t j = 0; j < m; ++j) {
            double ang = (double)sign * 2.0 * ORC_PI * (double)j / (double)len;
            double wr = cos(ang), wi = sin(ang);
            for (int64_t s = j; s < n; s += len) {
                int64_t t = s + m;
                double xr = re[t] * wr - im[t] * wi;
                double xi = re[t] * wi + im[t] * wr;
                re[t] = re[s] - xr; im[t] = im[s] - xi;
                re[s] = re[s] + xr; im[s] = im[s] + xi;
            }
        }
    }
    return 0;
}

/* ---------------------------------------------------------------------- */
/* Band: bins k in [0, n/2] with lo <= k fs / n <= hi, exactly in Hz.      */
/* ---------------------------------------------------------------------- */

int orc_in_band(int64_t k, int64_t n, int64_t fs_hz, int64_t lo_hz, int64_t hi_hz)
{
    if (k < 0 || k > n / 2) return 0;
    return lo_hz * n <= k * fs_hz && k * fs_hz <= hi_hz * n;
}

/* ---------------------------------------------------------------------- */
/* Pattern interpolation.                                                  */
/* ---------------------------------------------------------------------- */

/* Cell index and weight along zenith: clamp to the grid. */
static void zen_cell(const orc_grid* g, double zen, int64_t* iz, double* tz)
{
    double v = (zen - g->zen0_deg) / g->dzen_deg;
    if (v < 0.0) v = 0.0;
    if (v > (double)(g->n_zen - 1)) v = (double)(g->n_zen - 1);
    double fl = floor(v);
    int64_t i = (int64_t)fl;
    if (i > g->n_zen - 2) i = g->n_zen - 2;
    *iz = i;
    *tz = v - (double)i;
}

/* Cell indices and weight along azimuth: periodic with period 360 deg. */
static void az_cell(const orc_grid* g, double az, int64_t* ia, int64_t* ja, double* ta)
{
    double w = fmod(az - g->az0_deg, 360.0);
    if (w < 0.0) w += 360.0;
    w = w / g->daz_deg;
    double fl = floor(w);
    int64_t i = ((int64_t)fl) % g->n_az;
    *ia = i;
    *ja = (i + 1) % g->n_az;
    *ta = w - fl;
}

/*
 * Frequency cell for FFT bin k of an n-point trace sampled at fs: the bin
 * frequency k fs / n sits at node position (k fs - f0 n) / (n df), split
 * exactly into integer part and remainder.  Returns -1 if the bin lies
 * outside the table's frequency range.
 */
static int freq_cell(const orc_grid* g, int64_t k, int64_t n, int64_t fs_hz, int64_t* ifr, double* tf)
{
    int64_t num = k * fs_hz - g->f0_hz * n;
    int64_t den = n * g->df_hz;
    if (num < 0 || num > (int64_t)(g->n_freq - 1) * den) return -1;
    int64_t i = num / den;
    int64_t r = num % den;
    double t = (double)r / (double)den;
    if (i > g->n_freq - 2) { i = g->n_freq - 2; t = 1.0; }
    *ifr = i;
    *tf = t;
    return 0;
}

static double lerp(double a, double b, double t) { return (1.0 - t) * a + t * b; }

/* table layout [2 ch][2 comp][nf][nz][na] complex (interleaved re, im) */
static const double* node(const orc_grid* g, const double* tab, int c, int p,
                          int64_t f, int64_t z, int64_t a)
{
    int64_t idx = ((((int64_t)(c * 2 + p) * g->n_freq + f) * g->n_zen + z) * g->n_az + a);
    return tab + 2 * idx;
}

/*
 * Trilinear interpolant of one (channel, component) at a cell: along
 * azimuth first, then zenith, then frequency, on re and im separately.
 */
static void trilinear(const orc_grid* g, const double* tab, int c, int p,
                      int64_t ifr, double tf, int64_t iz, double tz,
                      int64_t ia, int64_t ja, double ta, double out[2])
{
    for (int part = 0; part < 2; ++part) {
        double fz[2];
        for (int df = 0; df < 2; ++df) {
            double za[2];
            for (int dz = 0; dz < 2; ++dz) {
                double a0 = node(g, tab, c, p, ifr + df, iz + dz, ia)[part];
                double a1 = node(g, tab, c, p, ifr + df, iz + dz, ja)[part];
                za[dz] = lerp(a0, a1, ta);
            }
            fz[df] = lerp(za[0], za[1], tz);
        }
        out[part] = lerp(fz[0], fz[1], tf);
    }
}

/*
 * Pattern H[c][p] at FFT bin k (n samples at fs) for direction (zen, az) in
 * degrees.  h[8] receives (c, p) = (0,th), (0,ph), (1,th), (1,ph) as
 * interleaved re, im.  Returns 0, or -1 if the bin is outside the table.
 */
int orc_pattern_at_bin(const orc_grid* g, const double* tab, int64_t k, int64_t n,
                       int64_t fs_hz, double zen, double az, double* h)
{
    int64_t ifr, iz, ia, ja;
    double tf, tz, ta;
    if (freq_cell(g, k, n, fs_hz, &ifr, &tf)) return -1;
    zen_cell(g, zen, &iz, &tz);
    az_cell(g, az, &ia, &ja, &ta);
    for (int c = 0; c < 2; ++c)
        for (int p = 0; p < 2; ++p)
            trilinear(g, tab, c, p, ifr, tf, iz, tz, ia, ja, ta, h + 2 * (c * 2 + p));
    return 0;
}

/*
 * As orc_pattern_at_bin, with the three interpolation weights rounded to the
 * nearest multiple of 2^-weight_bits (ties to even): the fixed-point weights
 * of a texture filter (section 3 interpolates with texture hardware).
 */
int orc_pattern_at_bin_quantized(const orc_grid* g, const double* tab, int64_t k, int64_t n, int64_t fs_hz,
                                 double zen, double az, int weight_bits, double* h)
{
    int64_t ifr, iz, ia, ja;
    double tf, tz, ta;
    if (freq_cell(g, k, n, fs_hz, &ifr, &tf)) return -1;
    zen_cell(g, zen, &iz, &tz);
    az_cell(g, az, &ia, &ja, &ta);
    const double q = ldexp(1.0, weight_bits);
    tf = nearbyint(tf * q) / q;
    tz = nearbyint(tz * q) / q;
    ta = nearbyint(ta * q) / q;
    for (int c = 0; c < 2; ++c)
        for (int p = 0; p < 2; ++p)
            trilinear(g, tab, c, p, ifr, tf, iz, tz, ia, ja, ta, h + 2 * (c * 2 + p));
    return 0;
}

/* ---------------------------------------------------------------------- */
/* 2x2 complex solve by Cramer's rule.                                     */
/* ---------------------------------------------------------------------- */

static void cmul(double ar, double ai, double br, double bi, double* r, double* i)
{
    *r = ar * br - ai * bi;
    *i = ar * bi + ai * br;
}

static void cdiv(double ar, double ai, double br, double bi, double* r, double* i)
{
    double d = br * br + bi * bi;
    *r = (ar * br + ai * bi) / d;
    *i = (ai * br - ar * bi) / d;
}

/*
 * Solve H e = x for e (H as 8 doubles in (c,p) order, x and e as 4 doubles
 * (re, im) per entry).  Returns 1 and sets e = 0 when
 * |det| <= singular_rel * ||H||_F^2, else 0.
 */
int orc_solve2(const double* h, const double* x, double singular_rel, double* e)
{
    double ar = h[0], ai = h[1];   /* H[0][th] */
    double br = h[2], bi = h[3];   /* H[0][ph] */
    double cr = h[4], ci = h[5];   /* H[1][th] */
    double dr = h[6], di = h[7];   /* H[1][ph] */
    double p1r, p1i, p2r, p2i;
    cmul(ar, ai, dr, di, &p1r, &p1i);
    cmul(br, bi, cr, ci, &p2r, &p2i);
    double detr = p1r - p2r, deti = p1i - p2i;
    double fro2 = ar * ar + ai * ai + br * br + bi * bi + cr * cr + ci * ci + dr * dr + di * di;
    double adet = sqrt(detr * detr + deti * deti);
    if (adet <= singular_rel * fro2) {
        e[0] = e[1] = e[2] = e[3] = 0.0;
        return 1;
    }
    double x0r = x[0], x0i = x[1], x1r = x[2], x1i = x[3];
    /* E_th = (H[1][ph] x0 - H[0][ph] x1) / det ; E_ph = (H[0][th] x1 - H[1][th] x0) / det */
    double t1r, t1i, t2r, t2i, nr, ni;
    cmul(dr, di, x0r, x0i, &t1r, &t1i);
    cmul(br, bi, x1r, x1i, &t2r, &t2i);
    nr = t1r - t2r; ni = t1i - t2i;
    cdiv(nr, ni, detr, deti, &e[0], &e[1]);
    cmul(ar, ai, x1r, x1i, &t1r, &t1i);
    cmul(cr, ci, x0r, x0i, &t2r, &t2i);
    nr = t1r - t2r; ni = t1i - t2i;
    cdiv(nr, ni, detr, deti, &e[2], &e[3]);
    return 0;
}

/* ---------------------------------------------------------------------- */
/* Full unfolding of selected (direction, station) units.                  */
/* ---------------------------------------------------------------------- */

/*
 * volt:    [n_st][2][n] float64 voltage traces of one event.
 * dirs:    [n_dir][2] (zenith, azimuth) in degrees.
 * units:   [n_units][2] int64 (direction index, station index).
 * efield:  [n_units][2][n] float64 output (E_theta, E_phi).
 * singular_bins: per unit, number of in-band bins treated as singular (may be NULL).
 * max_imag: largest |Im| / max|Re| seen after the inverse transform (may be NULL).
 * Returns 0, -1 on bad sizes, -2 on a band outside the table, -3 on allocation failure.
 */
int orc_unfold_units(const orc_grid* g, const double* tab,
                     int64_t n_st, int64_t n, int64_t fs_hz, int64_t lo_hz, int64_t hi_hz,
                     double singular_rel, const double* volt,
                     int64_t n_dir, const double* dirs,
                     int64_t n_units, const int64_t* units,
                     double* efield, int64_t* singular_bins, double* max_imag)
{
    if (!is_pow2(n) || n < 2 || n_st < 1) return -1;
    for (int64_t k = 0; k <= n / 2; ++k)
        if (orc_in_band(k, n, fs_hz, lo_hz, hi_hz)) {
            int64_t ifr; double tf;
            if (freq_cell(g, k, n, fs_hz, &ifr, &tf)) return -2;
        }
    double* xr[2]; double* xi[2]; double* er[2]; double* ei[2];
    double* buf = (double*)malloc(sizeof(double) * (size_t)n * 8);
    if (!buf) return -3;
    for (int c = 0; c < 2; ++c) {
        xr[c] = buf + (size_t)n * (0 + c);
        xi[c] = buf + (size_t)n * (2 + c);
        er[c] = buf + (size_t)n * (4 + c);
        ei[c] = buf + (size_t)n * (6 + c);
    }
    double worst = 0.0;
    for (int64_t u = 0; u < n_units; ++u) {
        int64_t d = units[2 * u], s = units[2 * u + 1];
        if (d < 0 || d >= n_dir || s < 0 || s >= n_st) { free(buf); return -1; }
        double zen = dirs[2 * d], az = dirs[2 * d + 1];
        /* spectra of both channels */
        for (int c = 0; c < 2; ++c) {
            const double* v = volt + ((size_t)s * 2 + c) * (size_t)n;
            for (int64_t j = 0; j < n; ++j) { xr[c][j] = v[j]; xi[c][j] = 0.0; }
            orc_fft(n, xr[c], xi[c], -1);
        }
        /* per-bin unfolding, band mask, Hermitian completion */
        for (int p = 0; p < 2; ++p)
            for (int64_t j = 0; j < n; ++j) { er[p][j] = 0.0; ei[p][j] = 0.0; }
        int64_t nsing = 0;
        for (int64_t k = 0; k <= n / 2; ++k) {
            if (!orc_in_band(k, n, fs_hz, lo_hz, hi_hz)) continue;
            double h[8], x[4], e[4];
            orc_pattern_at_bin(g, tab, k, n, fs_hz, zen, az, h);
            x[0] = xr[0][k]; x[1] = xi[0][k]; x[2] = xr[1][k]; x[3] = xi[1][k];
            nsing += orc_solve2(h, x, singular_rel, e);
            for (int p = 0; p < 2; ++p) {
                er[p][k] = e[2 * p];
                ei[p][k] = e[2 * p + 1];
                if (k != 0 && 2 * k != n) {
                    er[p][n - k] = e[2 * p];
                    ei[p][n - k] = -e[2 * p + 1];
                }
            }
        }
        if (singular_bins) singular_bins[u] = nsing;
        /* inverse transforms, real part, 1/N */
        for (int p = 0; p < 2; ++p) {
            orc_fft(n, er[p], ei[p], +1);
            double* out = efield + ((size_t)u * 2 + p) * (size_t)n;
            double peak = 0.0, imax = 0.0;
            for (int64_t j = 0; j < n; ++j) {
                out[j] = er[p][j] / (double)n;
                double a = fabs(out[j]);
                if (a > peak) peak = a;
                double b = fabs(ei[p][j] / (double)n);
                if (b > imax) imax = b;
            }
            if (peak > 0.0 && imax / peak > worst) worst = imax / peak;
        }
    }
    if (max_imag) *max_imag = worst;
    free(buf);
    return 0;
}

/* ---------------------------------------------------------------------- */
/* Hilbert envelope and its peak.                                          */
/* ---------------------------------------------------------------------- */

/*
 * env[j] = sqrt(x[j]^2 + H(x)[j]^2) for a real trace x of length n (a power
 * of two).  Returns 0, -1 on a bad size, -3 on allocation failure.
 */
int orc_envelope(int64_t n, const double* x, double* env)
{
    if (!is_pow2(n) || n < 2) return -1;
    double* re = (double*)malloc(sizeof(double) * (size_t)n * 2);
    if (!re) return -3;
    double* im = re + n;
    for (int64_t j = 0; j < n; ++j) { re[j] = x[j]; im[j] = 0.0; }
    orc_fft(n, re, im, -1);
    for (int64_t k = 0; k < n; ++k) {
        double sg = 0.0;
        if (k > 0 && 2 * k < n) sg = 1.0;
        if (2 * k > n) sg = -1.0;
        /* -i sgn(k) (a + ib) = sgn(k) (b - ia) */
        const double a = re[k], b = im[k];
        re[k] = sg * b;
        im[k] = -sg * a;
    }
    orc_fft(n, re, im, +1);
    for (int64_t j = 0; j < n; ++j) {
        const double h = re[j] / (double)n;
        env[j] = sqrt(x[j] * x[j] + h * h);
    }
    free(re);
    return 0;
}

/*
 * Peak of the envelope of each of `n_tr` traces of length n stored back to
 * back: peak[t] = max_j env_t[j], arg[t] = the smallest j attaining it.
 */
int orc_envelope_peaks(int64_t n_tr, int64_t n, const double* traces, double* peak, int64_t* arg)
{
    double* env = (double*)malloc(sizeof(double) * (size_t)n);
    if (!env) return -3;
    for (int64_t t = 0; t < n_tr; ++t) {
        int rc = orc_envelope(n, traces + (size_t)t * (size_t)n, env);
        if (rc) { free(env); return rc; }
        double best = -1.0;
        int64_t bj = 0;
        for (int64_t j = 0; j < n; ++j)
            if (env[j] > best) { best = env[j]; bj = j; }
        peak[t] = best;
        arg[t] = bj;
    }
    free(env);
    return 0;
}

/* ---------------------------------------------------------------------- */
/* Reconstruction loop: timing -> triangulation -> unfold -> envelope.     */
/* ---------------------------------------------------------------------- */

static const double ORC_C_M_PER_NS = 0.299792458;

/*
 * Least-squares plane wave through station times t[s] (samples at fs) at
 * ground positions pos[s] = (x, y) metres: t_ns = t0 + p x + q y.  Writes
 * (zenith, azimuth) in degrees of the source direction.  Returns 0, or -1
 * if the normal equations are singular (fewer than 3 non-collinear stations).
 */
int orc_plane_fit(int64_t n_st, const double* pos, const int64_t* t, int64_t fs_hz, double* dir)
{
    double a[3][4] = {{0}};
    const double dt = 1e9 / (double)fs_hz;
    for (int64_t s = 0; s < n_st; ++s) {
        const double row[3] = {1.0, pos[2 * s], pos[2 * s + 1]};
        const double ts = (double)t[s] * dt;
        for (int i = 0; i < 3; ++i) {
            for (int j = 0; j < 3; ++j) a[i][j] += row[i] * row[j];
            a[i][3] += row[i] * ts;
        }
    }
    /* Gaussian elimination with partial pivoting on the 3x4 augmented matrix */
    for (int c = 0; c < 3; ++c) {
        int piv = c;
        for (int r = c + 1; r < 3; ++r)
            if (fabs(a[r][c]) > fabs(a[piv][c])) piv = r;
        if (fabs(a[piv][c]) < 1e-300) return -1;
        if (piv != c)
            for (int j = 0; j < 4; ++j) { double tmp = a[c][j]; a[c][j] = a[piv][j]; a[piv][j] = tmp; }
        for (int r = c + 1; r < 3; ++r) {
            const double f = a[r][c] / a[c][c];
            for (int j = c; j < 4; ++j) a[r][j] -= f * a[c][j];
        }
    }
    double x[3];
    for (int c = 2; c >= 0; --c) {
        double v = a[c][3];
        for (int j = c + 1; j < 3; ++j) v -= a[c][j] * x[j];
        x[c] = v / a[c][c];
    }
    if (fabs(a[2][2]) < 1e-12 * fabs(a[0][0])) return -1;
    const double nx = -ORC_C_M_PER_NS * x[1], ny = -ORC_C_M_PER_NS * x[2];
    double sn = sqrt(nx * nx + ny * ny);
    if (sn > 1.0) sn = 1.0;
    double az = atan2(ny, nx) * 180.0 / ORC_PI;
    if (az < 0.0) az += 360.0;
    dir[0] = asin(sn) * 180.0 / ORC_PI;
    dir[1] = az;
    return 0;
}

/*
 * volt [S][2][N], pos [S][2] metres.  dirs_out [max_iter][2] receives the
 * direction of every iteration, times_out [max_iter+1][S] the station times
 * (samples) of every pass: row 0 the voltage maxima, row i+1 the envelope
 * maxima after direction i (rows 0..*n_dirs are written).  *n_dirs is the
 * number of directions produced (the last one is the result; it is the
 * converged direction if *converged).  Returns 0 or a negative error (bad
 * sizes, singular geometry, allocation).
 */
int orc_reconstruct(const orc_grid* g, const double* tab, int64_t n_st, int64_t n, int64_t fs_hz,
                    int64_t lo_hz, int64_t hi_hz, double singular_rel, const double* volt,
                    const double* pos, int64_t max_iter, double* dirs_out, int64_t* times_out,
                    int64_t* n_dirs, int64_t* converged)
{
    if (n_st < 3 || max_iter < 1) return -1;
    int64_t* t = (int64_t*)malloc(sizeof(int64_t) * (size_t)n_st * 3);
    double* e = (double*)malloc(sizeof(double) * (size_t)n_st * 2 * (size_t)n);
    double* env0 = (double*)malloc(sizeof(double) * (size_t)n * 2);
    if (!t || !e || !env0) { free(t); free(e); free(env0); return -3; }
    int64_t* units = t + n_st;        /* [S][2] (direction 0, station) */
    double* env1 = env0 + n;
    for (int64_t s = 0; s < n_st; ++s) {
        const double* v0 = volt + (size_t)s * 2 * (size_t)n;
        const double* v1 = v0 + n;
        double best = -1.0;
        int64_t bj = 0;
        for (int64_t j = 0; j < n; ++j) {
            const double pw = v0[j] * v0[j] + v1[j] * v1[j];
            if (pw > best) { best = pw; bj = j; }
        }
        t[s] = bj;
        times_out[s] = bj;
        units[2 * s] = 0;
        units[2 * s + 1] = s;
    }
    int rc = 0;
    *n_dirs = 0;
    *converged = 0;
    for (int64_t it = 0; it < max_iter; ++it) {
        double* dir = dirs_out + 2 * it;
        if (orc_plane_fit(n_st, pos, t, fs_hz, dir)) { rc = -4; break; }
        *n_dirs = it + 1;
        rc = orc_unfold_units(g, tab, n_st, n, fs_hz, lo_hz, hi_hz, singular_rel, volt, 1, dir,
                              n_st, units, e, NULL, NULL);
        if (rc) break;
        int64_t changed = 0;
        for (int64_t s = 0; s < n_st; ++s) {
            const double* es = e + (size_t)s * 2 * (size_t)n;
            if ((rc = orc_envelope(n, es, env0)) || (rc = orc_envelope(n, es + n, env1))) break;
            double best = -1.0;
            int64_t bj = 0;
            for (int64_t j = 0; j < n; ++j) {
                const double tot = sqrt(env0[j] * env0[j] + env1[j] * env1[j]);
                if (tot > best) { best = tot; bj = j; }
            }
            changed += bj != t[s];
            t[s] = bj;
        }
        if (rc) break;
        for (int64_t s = 0; s < n_st; ++s) times_out[(it + 1) * n_st + s] = t[s];
        if (!changed) { *converged = 1; break; }
    }
    free(t);
    free(e);
    free(env0);
    return rc;
}

/* ---------------------------------------------------------------------- */
/* Direction fit: timing-consistency score over candidate directions.     */
/* ---------------------------------------------------------------------- */

/* chi2[d] for station times t [n_dir][n_st] (samples at fs), dirs [n_dir][2]
 * degrees, pos [n_st][2] metres; also power[d] = sum_s peak[d][s]^2 when
 * peak (nullable) is given.  Two plain passes: the best t0 is the mean of
 * the residuals, then the sum of squared deviations from it. */
void orc_direction_objective(int64_t n_st, const double* pos, int64_t n_dir, const double* dirs,
                             const int64_t* t, int64_t fs_hz, const double* peak, double* chi2, double* power)
{
    const double dt = 1e9 / (double)fs_hz;
    for (int64_t d = 0; d < n_dir; ++d) {
        const double zr = dirs[2 * d] * ORC_PI / 180.0, ar = dirs[2 * d + 1] * ORC_PI / 180.0;
        const double nx = sin(zr) * cos(ar), ny = sin(zr) * sin(ar);
        double mean = 0.0;
        for (int64_t s = 0; s < n_st; ++s) {
            const double tau = -(nx * pos[2 * s] + ny * pos[2 * s + 1]) / ORC_C_M_PER_NS;
            mean += (double)t[d * n_st + s] * dt - tau;
        }
        mean /= (double)n_st;
        double acc = 0.0, pw = 0.0;
        for (int64_t s = 0; s < n_st; ++s) {
            const double tau = -(nx * pos[2 * s] + ny * pos[2 * s + 1]) / ORC_C_M_PER_NS;
            const double r = (double)t[d * n_st + s] * dt - tau - mean;
            acc += r * r;
            if (peak) pw += peak[d * n_st + s] * peak[d * n_st + s];
        }
        chi2[d] = acc;
        if (power) power[d] = pw;
    }
}

/* K x K directions around (zc, ac): zenith zc + (i - (K-1)/2) hz clamped to
 * [0, 90] (row i), azimuth ac + (j - (K-1)/2) ha wrapped to [0, 360)
 * (column j); dirs [K*K][2] row-major. */
void orc_local_grid(double zc, double ac, double hz, double ha, int64_t k, double* dirs)
{
    const double m = 0.5 * (double)(k - 1);
    for (int64_t i = 0; i < k; ++i) {
        for (int64_t j = 0; j < k; ++j) {
            double z = zc + ((double)i - m) * hz;
            if (z < 0.0) z = 0.0;
            if (z > 90.0) z = 90.0;
            double a = ac + ((double)j - m) * ha;
            a = a - 360.0 * floor(a / 360.0);
            if (a >= 360.0) a -= 360.0;
            dirs[2 * (i * k + j)] = z;
            dirs[2 * (i * k + j) + 1] = a;
        }
    }
}

/* The fit: score the n_dir candidates, then `levels` refinements, each a
 * k x k grid around the best so far at spacing (step_z, step_a) / 2^level.
 * Outputs: level_dirs [levels][k*k][2]; chi2 and power [n_dir + levels*k*k]
 * (candidates in order, coarse first); best [levels + 1] (index within its
 * level); result [2] the best direction of the last level.  Returns 0 or a
 * negative error. */
int orc_direction_fit(const orc_grid* g, const double* tab, int64_t n_st, int64_t n, int64_t fs_hz,
                      int64_t lo_hz, int64_t hi_hz, double singular_rel, const double* volt, const double* pos,
                      int64_t n_dir, const double* dirs, int64_t levels, int64_t k, double step_z,
                      double step_a, double* level_dirs, double* chi2, double* power, int64_t* best,
                      double* result)
{
    if (n_st < 3 || n_dir < 1 || levels < 0 || k < 1) return -1;
    const int64_t dmax = n_dir > k * k ? n_dir : k * k;
    int64_t* units = (int64_t*)malloc(sizeof(int64_t) * 2 * (size_t)(dmax * n_st));
    int64_t* t = (int64_t*)malloc(sizeof(int64_t) * (size_t)(dmax * n_st));
    double* pk = (double*)malloc(sizeof(double) * (size_t)(dmax * n_st));
    double* e = (double*)malloc(sizeof(double) * 2 * (size_t)n * (size_t)(dmax * n_st));
    double* env = (double*)malloc(sizeof(double) * 2 * (size_t)n);
    if (!units || !t || !pk || !e || !env) {
        free(units); free(t); free(pk); free(e); free(env);
        return -3;
    }
    int rc = 0;
    const double* cand = dirs;
    int64_t nc = n_dir, off = 0;
    for (int64_t lv = 0; lv <= levels && rc == 0; ++lv) {
        if (lv > 0) {
            double* nd = level_dirs + 2 * (lv - 1) * k * k;
            const double sc = ldexp(1.0, (int)-lv);
            orc_local_grid(result[0], result[1], step_z * sc, step_a * sc, k, nd);
            cand = nd;
            nc = k * k;
        }
        for (int64_t d = 0; d < nc; ++d)
            for (int64_t s = 0; s < n_st; ++s) {
                units[2 * (d * n_st + s)] = d;
                units[2 * (d * n_st + s) + 1] = s;
            }
        rc = orc_unfold_units(g, tab, n_st, n, fs_hz, lo_hz, hi_hz, singular_rel, volt, nc, cand, nc * n_st,
                              units, e, NULL, NULL);
        for (int64_t u = 0; rc == 0 && u < nc * n_st; ++u) {
            const double* eu = e + (size_t)u * 2 * (size_t)n;
            if ((rc = orc_envelope(n, eu, env)) || (rc = orc_envelope(n, eu + n, env + n))) break;
            double bv = -1.0;
            int64_t bj = 0;
            for (int64_t j = 0; j < n; ++j) {
                const double tot = sqrt(env[j] * env[j] + env[n + j] * env[n + j]);
                if (tot > bv) { bv = tot; bj = j; }
            }
            t[u] = bj;
            pk[u] = bv;
        }
        if (rc) break;
        orc_direction_objective(n_st, pos, nc, cand, t, fs_hz, pk, chi2 + off, power + off);
        int64_t b = 0;
        for (int64_t d = 1; d < nc; ++d)
            if (chi2[off + d] < chi2[off + b]) b = d;
        best[lv] = b;
        result[0] = cand[2 * b];
        result[1] = cand[2 * b + 1];
        off += nc;
    }
    free(units); free(t); free(pk); free(e); free(env);
    return rc;
}
