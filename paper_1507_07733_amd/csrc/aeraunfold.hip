// aeraunfold.hip -- kernels, launch dispatch and the C ABI of the unfolding
// library (declarations and contracts in include/aeraunfold.h).
//
// Path per event (arXiv:1507.07733, section 2, the E-field step of the
// reconstruction; section 3 pattern interpolation; section 4 FFTs; band of
// section 1):
//   k_spectrum  once per station       V[2][N] -> X_0, X_1 at in-band bins
//   k_coef      once per direction     H(f_k) interpolated, inverted -> coef
//   k_unfold    per direction x station coef * X -> packed iFFT -> E_theta, E_phi
// k_unfold writes the only large data stream (2 N values per station and
// direction), so the whole path is bound by HBM write bandwidth when the
// FFT keeps up.
#include "aeraunfold.h"
#include "au_internal.h"
#include "au_kernels.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <map>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

using namespace au;

// ---------------------------------------------------------------------------
// errors
// ---------------------------------------------------------------------------

static thread_local std::string g_err;

static au_status fail(au_status s, const std::string& msg)
{
    g_err = msg;
    return s;
}

au_status au::set_error(au_status s, const std::string& msg) { return fail(s, msg); }
const std::string& au::error_string() { return g_err; }

#define HIP_TRY(expr)                                                                        \
    do {                                                                                     \
        hipError_t e_ = (expr);                                                              \
        if (e_ != hipSuccess)                                                                \
            return fail(AU_EDEVICE, std::string(#expr) + ": " + hipGetErrorString(e_));     \
    } while (0)

extern "C" const char* au_last_error(void) { return g_err.c_str(); }
extern "C" const char* au_version(void) { return "aeraunfold 0.1 gfx950"; }

// ---------------------------------------------------------------------------
// device helpers: pattern-grid cells (section 3: linear interpolation
// between frequency / zenith / azimuth nodes)
// ---------------------------------------------------------------------------

// Zenith cell and weight; positions outside the grid are clamped to it.
// Azimuth cell, its periodic neighbour and weight.
__device__ __forceinline__ void angle_cells(const GridDev& g, double zen, double az, int& iz,
                                            double& tz, int& ia, int& ja, double& ta)
{
    double v = (zen - g.zen0) / g.dzen;
    v = v < 0.0 ? 0.0 : v;
    v = v > (double)(g.n_zen - 1) ? (double)(g.n_zen - 1) : v;
    int i = (int)floor(v);
    if (i > g.n_zen - 2) i = g.n_zen - 2;
    iz = i;
    tz = v - (double)i;
    double w = fmod(az - g.az0, 360.0);
    if (w < 0.0) w += 360.0;
    w = w / g.daz;
    const double fl = floor(w);
    const int a = ((int)fl) % g.n_az;
    ia = a;
    ja = (a + 1 == g.n_az) ? 0 : a + 1;
    ta = w - fl;
}

// Frequency cell of FFT bin k (N samples at fs): node position
// (k fs - f0 N) / (N df), split exactly into integer part and remainder.
__device__ __forceinline__ void freq_cell(const GridDev& g, int64_t k, int n, int64_t fs, int& ifr,
                                          double& tf)
{
    const int64_t num = k * fs - g.f0_hz * (int64_t)n;
    const int64_t den = (int64_t)n * g.df_hz;
    // The truncated quotient num / den without a 64-bit integer division:
    // |num| < 2^53, so num and den are exact in double and the estimate is
    // within one of the quotient; one correction step makes it exact (the
    // remainder takes the sign of num, as the integer division's does).
    int64_t i = (int64_t)((double)num * (1.0 / (double)den));
    int64_t r = num - i * den;
    if (num >= 0) {
        if (r < 0) {
            --i;
            r += den;
        } else if (r >= den) {
            ++i;
            r -= den;
        }
    } else {
        if (r > 0) {
            ++i;
            r -= den;
        } else if (r <= -den) {
            --i;
            r += den;
        }
    }
    double t = (double)r / (double)den;
    if (i > g.n_freq - 2) {
        i = g.n_freq - 2;
        t = 1.0;
    }
    ifr = (int)i;
    tf = t;
}

template <typename T>
__device__ __forceinline__ C2<T> clerp(C2<T> a, C2<T> b, T t)
{
    const T s = (T)1 - t;
    return {s * a.re + t * b.re, s * a.im + t * b.im};
}

// Entry cp of the four (channel, component) entries at frequency node f,
// interpolated along azimuth, then zenith (a direction's angular slice at
// that node).  Table layout [f][z][a][4] complex.  One entry per call, so
// that a workgroup spreads a slice over (node, entry) pairs: four
// independent loads per thread.
template <typename Tt, typename T>
__device__ __forceinline__ C2<T> slice1(const C2<Tt>* __restrict__ nodes, const GridDev& g, int f, int cp, int iz,
                                        T tz, int ia, int ja, T ta)
{
    C2<T> za[2];
#pragma unroll
    for (int dz = 0; dz < 2; ++dz) {
        const int64_t row = ((int64_t)f * g.n_zen + (iz + dz)) * g.n_az;
        const C2<Tt> p0 = nodes[(row + ia) * 4 + cp];
        const C2<Tt> p1 = nodes[(row + ja) * 4 + cp];
        za[dz] = clerp(C2<T>{(T)p0.re, (T)p0.im}, C2<T>{(T)p1.re, (T)p1.im}, ta);
    }
    return clerp(za[0], za[1], tz);
}

// Frequency nodes a direction's angular slice holds in LDS at a time (the
// 30-80 MHz band spans 52 nodes at 1 MHz, 102 at 0.5 MHz); wider bands are
// taken in windows of this many nodes.
constexpr int kMaxSliceNodes = 256;


// Power-of-two exponent e such that the largest real or imaginary part of
// h, times 2^-e, lies in [0.5, 1), and hs = 2^-e h.  Scaling by a power of two
// is exact, so every threshold decision and every rounding of the inverse
// below is the one the unscaled H would give, while |det|^2 and
// (rel ||H||_F^2)^2 stay inside the format's range whatever the table's
// units (a table of order 1e-12 or 1e12 squares to 1e-48 / 1e48, outside
// FP32).  Returns false for an all-zero or non-finite H.
template <typename T>
__device__ __forceinline__ bool pow2_normalise(const C2<T> h[4], C2<T> hs[4], int& e)
{
    T mx = 0;
#pragma unroll
    for (int i = 0; i < 4; ++i) mx = fmax(mx, fmax(fabs(h[i].re), fabs(h[i].im)));
    if (!(mx > (T)0) || !isfinite(mx)) return false;
    (void)frexp(mx, &e);
#pragma unroll
    for (int i = 0; i < 4; ++i) hs[i] = C2<T>{ldexp(h[i].re, -e), ldexp(h[i].im, -e)};
    return true;
}

// Coefficients of the bin from the normalised hs = 2^-e H (pow2_normalise):
// C = (1/N) H^-1 = (1/(N det)) [h3 -h1; -h2 h0] with H = [h0 h1; h2 h3]
// indexed [channel][component]; as H^-1 = 2^-e hs^-1, the scale goes into
// the numerator inv_n_scaled = 2^-e / N.  Written in the packed form of MBin
// (p_j = C_0j + i C_1j, q_j = C_0j - i C_1j).  Singular (|det| <=
// singular_rel ||H||_F^2, the same test on hs) gives zero coefficients and
// returns 1.
template <typename T>
__device__ __forceinline__ int invert2_scaled(const C2<T> h[4], T inv_n_scaled, double singular_rel, MBin<T>& m)
{
    const C2<T> det = csub(cmul(h[0], h[3]), cmul(h[1], h[2]));
    T fro2 = 0;
#pragma unroll
    for (int i = 0; i < 4; ++i) fro2 += h[i].re * h[i].re + h[i].im * h[i].im;
    const T ad2 = det.re * det.re + det.im * det.im;
    const T thr = (T)singular_rel * fro2;
    if (!(ad2 > thr * thr)) {
        m.p0 = m.p1 = m.q0 = m.q1 = C2<T>{0, 0};
        return 1;
    }
    const T sc = inv_n_scaled / ad2;
    const C2<T> inv{det.re * sc, -det.im * sc};
    const C2<T> c00 = cmul(h[3], inv);
    const C2<T> c01 = cmul(C2<T>{-h[1].re, -h[1].im}, inv);
    const C2<T> c10 = cmul(C2<T>{-h[2].re, -h[2].im}, inv);
    const C2<T> c11 = cmul(h[0], inv);
    // c + i c' = (c.re - c'.im, c.im + c'.re); c - i c' = (c.re + c'.im, c.im - c'.re)
    m.p0 = C2<T>{c00.re - c10.im, c00.im + c10.re};
    m.p1 = C2<T>{c01.re - c11.im, c01.im + c11.re};
    m.q0 = C2<T>{c00.re + c10.im, c00.im - c10.re};
    m.q1 = C2<T>{c01.re + c11.im, c01.im - c11.re};
    return 0;
}

// Coefficients of the bin from H as interpolated (any scale).  Returns 1 if singular.
template <typename T>
__device__ __forceinline__ int invert2(const C2<T> h[4], T inv_n, double singular_rel, MBin<T>& m)
{
    C2<T> hs[4];
    int e;
    if (!pow2_normalise(h, hs, e)) {
        m.p0 = m.p1 = m.q0 = m.q1 = C2<T>{0, 0};
        return 1;
    }
    return invert2_scaled(hs, ldexp(inv_n, -e), singular_rel, m);
}

// The packed spectrum of one bin from its packed coefficients: zp = Z[k] and
// zq = conj Z[N - k] (see MBin); at k = 0 the packed value is (E_theta.re,
// E_phi.re) = ((zp + zq).re / 2, (zp - zq).im / 2).
// a0 b0 + a1 b1 as one chain of fused multiply-adds per component.
template <typename T>
__device__ __forceinline__ C2<T> cdot2(C2<T> a0, C2<T> b0, C2<T> a1, C2<T> b1)
{
    return C2<T>{fma(a0.re, b0.re, fma(-a0.im, b0.im, fma(a1.re, b1.re, -a1.im * b1.im))),
                 fma(a0.re, b0.im, fma(a0.im, b0.re, fma(a1.re, b1.im, a1.im * b1.re)))};
}

template <typename T>
__device__ __forceinline__ void packed_bin(const MBin<T>& m, const XBin<T>& xb, C2<T>& zp, C2<T>& zq)
{
    zp = cdot2(m.p0, xb.x0, m.p1, xb.x1);
    zq = cdot2(m.q0, xb.x0, m.q1, xb.x1);
}
template <typename T>
__device__ __forceinline__ C2<T> packed_dc(const C2<T>& zp, const C2<T>& zq)
{
    return C2<T>{(T)0.5 * (zp.re + zq.re), (T)0.5 * (zp.im - zq.im)};
}

// ---------------------------------------------------------------------------
// kernels
// ---------------------------------------------------------------------------

// Spectra of one station per FFT group: z = V_0 + i V_1, Z = FFT(z), and at
// each in-band bin X_0 = (Z[k] + conj Z[N-k]) / 2, X_1 = (Z[k] - conj Z[N-k]) / 2i.
// Units: (event, station); units == nullptr means event ev0, unit = station.
template <typename Tin, typename T, int N, int E>
__global__ __launch_bounds__(kBlock) void k_spectrum(const Tin* __restrict__ volt, EvDesc ev0,
                                                     const EvDesc* __restrict__ evs,
                                                     const int2* __restrict__ units, int n_units,
                                                     XBin<T>* __restrict__ X,
                                                     const C2<T>* __restrict__ tw)
{
    constexpr int TT = N / E;
    constexpr int G = groups_per_block<T, N, E>();
    extern __shared__ __align__(16) unsigned char smem[];
    const int g = G == 1 ? 0 : (int)(threadIdx.x / TT), t = threadIdx.x % TT;
    C2<T>* lds = reinterpret_cast<C2<T>*>(smem) + g * lds_elems<N>();
    const int u = blockIdx.x * G + g;
    const bool active = u < n_units;
    int e = 0, s = active ? u : 0;
    if (units != nullptr && active) {
        const int2 w = units[u];
        e = w.x;
        s = w.y;
    }
    const EvDesc ev = evs ? evs[e] : ev0;
    const Tin* v = volt + ev.volt_off + (int64_t)s * 2 * N;
    C2<T> x[E];
#pragma unroll
    for (int i = 0; i < E; ++i) {
        const int n = t + TT * i;
        x[i] = active ? C2<T>{(T)v[n], (T)v[N + n]} : C2<T>{0, 0};
    }
    fft<T, N, E, -1>(x, lds, tw, t);
#pragma unroll
    for (int i = 0; i < E; ++i) lds[lpad<T>(t + TT * i)] = x[i];
    __syncthreads();
    if (active) {
        XBin<T>* out = X + ev.x_off + (int64_t)s * ev.nb;
        for (int j = t; j < ev.nb; j += TT) {
            const int k = ev.k_lo + j;
            const C2<T> a = lds[lpad<T>(k)];
            const C2<T> b = lds[lpad<T>((N - k) & (N - 1))];
            XBin<T> r;
            r.x0 = C2<T>{(T)0.5 * (a.re + b.re), (T)0.5 * (a.im - b.im)};
            r.x1 = C2<T>{(T)0.5 * (a.im + b.im), (T)0.5 * (b.re - a.re)};
            out[j] = r;
        }
    }
}

// Bins per thread the streaming spectrum kernel stores: it serves bands of at
// most N/4 bins (30-80 MHz at 200 MHz sampling is 0.25 N bins); wider bands
// take k_spectrum.
constexpr int kSpecStreamBins = 2;

// The same spectra by a persistent grid (FP32, 8 values per thread, radix 8):
// each workgroup takes the stations blockIdx.x, blockIdx.x + gridDim.x, ...
// and issues the trace loads of its next station before transforming the
// current one, so that their latency hides behind the transform.  Nothing in
// the station loop waits for a load issued after the previous station's
// stores (vector-memory completions count in issue order): the early passes'
// twiddles (fused multiply-add form, TW_LF) sit in an LDS table and the last
// pass's in registers, both set
// once, and every thread issues a fixed number of spectrum stores, the lanes
// past the band storing out of range of the row (dropped).
template <typename Tin, int N>
__global__ __launch_bounds__(N / 8) void k_spectrum_stream(const Tin* __restrict__ volt, EvDesc ev0,
                                                           const EvDesc* __restrict__ evs,
                                                           const int2* __restrict__ units, int n_units,
                                                           XBin<float>* __restrict__ X,
                                                           const C2<float>* __restrict__ tw)
{
    using T = float;
    constexpr int E = 8, RMAX = 8, TT = N / E;
    static_assert(kSpecStreamBins * TT <= N, "gathered bins stay inside the transform");
    extern __shared__ __align__(16) unsigned char smem[];
    C2<T>* lds = reinterpret_cast<C2<T>*>(smem);
    C2<T>* ltw = lds + lds_elems<N>();
    const int t = threadIdx.x;
    C2<T> w[tw_count<N, E, RMAX, TW_LF>()];
    load_twiddles<T, N, E, RMAX, TW_LF, +1>(w, tw, t);  // TW_LF entries serve both directions
    fill_lds_twiddles<T, N, E, RMAX, +1, TW_LF>(ltw, tw, t, TT);
    vmem_wait_all();
    lds_barrier();
    // the host launches at most n_units workgroups; a station's trace pair,
    // spectrum row, row length and first bin:
    struct Row {
        const Tin* v;
        XBin<T>* out;
        int nb, k_lo;
    };
    auto locate = [&](int uu) {
        // uu is uniform; stated so, the unit is read with a scalar load: a
        // vector load here would wait (in issue order) for the previous
        // station's stores
        uu = __builtin_amdgcn_readfirstlane(uu);
        int e = 0, s = uu;
        if (units != nullptr) {
            const int2 su = units[uu];
            e = su.x;
            s = su.y;
        }
        const int64_t volt_off = evs ? evs[e].volt_off : ev0.volt_off;
        const int64_t x_off = evs ? evs[e].x_off : ev0.x_off;
        const int nb = evs ? evs[e].nb : ev0.nb;
        const int k_lo = evs ? evs[e].k_lo : ev0.k_lo;
        return Row{volt + volt_off + (int64_t)s * 2 * N, X + x_off + (int64_t)s * nb, nb, k_lo};
    };
    int u = blockIdx.x;
    Row row = locate(u);
    Tin a[E], b[E];
#pragma unroll
    for (int i = 0; i < E; ++i) {
        a[i] = row.v[t + TT * i];
        b[i] = row.v[N + t + TT * i];
    }
    for (;;) {
        C2<T> x[E];
#pragma unroll
        for (int i = 0; i < E; ++i) x[i] = C2<T>{(T)a[i], (T)b[i]};
        const int un = u + (int)gridDim.x;
        Row next = row;
        if (un < n_units) {
            next = locate(un);
#pragma unroll
            for (int i = 0; i < E; ++i) {
                a[i] = next.v[t + TT * i];
                b[i] = next.v[N + t + TT * i];
            }
        }
        fft<T, N, E, -1, TW_LF, RMAX>(x, lds, tw, t, w, ltw);
#pragma unroll
        for (int i = 0; i < E; ++i) lds[lpad<T>(t + TT * i)] = x[i];
        lds_barrier();
        const unsigned nb = (unsigned)row.nb;
        const __amdgpu_buffer_rsrc_t out = buffer_range(row.out, nb * (unsigned)sizeof(XBin<T>));
#pragma unroll
        for (int q = 0; q < kSpecStreamBins; ++q) {
            const unsigned j = (unsigned)(t + TT * q);
            const int k = j < nb ? row.k_lo + (int)j : 0;
            const C2<T> za = lds[lpad<T>(k)];
            const C2<T> zb = lds[lpad<T>((N - k) & (N - 1))];
            XBin<T> r;
            r.x0 = C2<T>{(T)0.5 * (za.re + zb.re), (T)0.5 * (za.im - zb.im)};
            r.x1 = C2<T>{(T)0.5 * (za.im + zb.im), (T)0.5 * (zb.re - za.re)};
            buffer_store16(r, out, (j < nb ? j : nb) * (unsigned)sizeof(XBin<T>));
        }
        if (un >= n_units) break;
        // every gather done before the next transform writes the buffer
        lds_barrier();
        u = un;
        row = next;
    }
}

// Coefficients of every in-band bin of one (event, direction) per block.
// FP32 (T = float): interpolation, determinant and inverse in float; where
// |det| < fallback_rel ||H||_F^2 in float, the determinant and inverse are
// redone in double from the same float H.  Singular bins give zero coefs.
// RESP: write the interpolated H instead (au_pattern_response).
// The packed coefficients of one bin from its interpolated H (1/N folded
// in): FP64 by the direct inverse; FP32 by the inverse on 2^-e H (exact
// scaling, see pow2_normalise) with the FP64 determinant fallback when
// |det| < fallback_rel ||H||_F^2.  Counts fallback and singular bins.
template <typename T>
__device__ __forceinline__ MBin<T> coef_from_h(const C2<T> (&h)[4], int n, T inv_n, double fallback_rel,
                                               double singular_rel, unsigned int& n_fb, unsigned int& n_sg)
{
    // the counts go through locals added once at the end: increments of the
    // two references on different branches became a select of their
    // addresses, i.e. the counters in scratch memory with a wait for every
    // outstanding memory operation at each bin
    MBin<T> m;
    unsigned int fb = 0, sg = 0;
    if constexpr (sizeof(T) == 4) {
        C2<float> hs[4];
        int e;
        if (!pow2_normalise(h, hs, e)) {
            m.p0 = m.p1 = m.q0 = m.q1 = C2<T>{0, 0};
            sg = 1;
        } else {
            const C2<float> det = csub(cmul(hs[0], hs[3]), cmul(hs[1], hs[2]));
            float fro2 = 0.f;
#pragma unroll
            for (int i = 0; i < 4; ++i) fro2 += hs[i].re * hs[i].re + hs[i].im * hs[i].im;
            const float ad2 = det.re * det.re + det.im * det.im;
            const float thr = (float)fallback_rel * fro2;
            if (ad2 < thr * thr) {
                C2<double> hd[4];
#pragma unroll
                for (int i = 0; i < 4; ++i) hd[i] = C2<double>{(double)hs[i].re, (double)hs[i].im};
                MBin<double> md;
                sg = (unsigned int)invert2_scaled<double>(hd, ldexp(1.0 / (double)n, -e), singular_rel, md);
                fb = 1;
                m.p0 = C2<T>{(T)md.p0.re, (T)md.p0.im};
                m.p1 = C2<T>{(T)md.p1.re, (T)md.p1.im};
                m.q0 = C2<T>{(T)md.q0.re, (T)md.q0.im};
                m.q1 = C2<T>{(T)md.q1.re, (T)md.q1.im};
            } else {
                sg = (unsigned int)invert2_scaled<T>(hs, ldexp(inv_n, -e), singular_rel, m);
            }
        }
    } else {
        sg = (unsigned int)invert2<T>(h, inv_n, singular_rel, m);
    }
    n_fb += fb;
    n_sg += sg;
    return m;
}

// The work of workgroup bx of k_coef.  dirs and skip may be written earlier
// in the same kernel (by another thread of the workgroup, before a barrier).
template <typename Tt, typename T, bool RESP>
__device__ __forceinline__ void coef_block(int bx, const C2<Tt>* __restrict__ nodes, const GridDev& gd,
                                           const EvDesc& ev0, const EvDesc* __restrict__ evs,
                                           const int2* __restrict__ units, const double* dirs, double zen1,
                                           double az1, int64_t fs, double fallback_rel, double singular_rel,
                                           MBin<T>* __restrict__ M, unsigned long long* __restrict__ counts,
                                           double wq, const int* skip, int skip_stride)
{
    __shared__ unsigned int cnt[2];
    if (threadIdx.x < 2) cnt[threadIdx.x] = 0;
    __syncthreads();
    int e = 0, d = bx;
    if (units != nullptr) {
        const int2 w = units[bx];
        e = w.x;
        d = w.y;
    }
    // a converged reconstruction loop: its envelope launch is skipped too
    if (skip != nullptr && skip[(int64_t)e * skip_stride]) return;
    const EvDesc ev = evs ? evs[e] : ev0;
    double zen = zen1, az = az1;
    if (dirs != nullptr) {
        zen = dirs[2 * (ev.dir_off + d)];
        az = dirs[2 * (ev.dir_off + d) + 1];
    }
    int iz, ia, ja;
    double tz, ta;
    angle_cells(gd, zen, az, iz, tz, ia, ja, ta);
    if constexpr (RESP) {
        if (wq > 0.0) {  // interpolation weights rounded to multiples of 1 / wq
            tz = rint(tz * wq) / wq;
            ta = rint(ta * wq) / wq;
        }
    }
    const T inv_n = (T)(1.0 / (double)ev.N);
    unsigned int n_fb = 0, n_sg = 0;
    MBin<T>* out = M + ev.m_off + (int64_t)d * ev.nb;
    // The direction's angular slice (bilinear in azimuth and zenith) at every
    // frequency node the band's bins fall between, once, in LDS; each bin then
    // only interpolates in frequency between two slice nodes.  The same
    // operations in the same order as interpolating every bin from the table.
    // A band spanning more than kMaxSliceNodes nodes is taken in windows of
    // that many nodes, consecutive windows sharing one node; a bin belongs to
    // the window that holds both of its nodes.
    __shared__ C2<T> sl[kMaxSliceNodes][4];
    int f_lo = 0, n_nodes = 0;
    if (ev.nb > 0) {
        int f_hi;
        double tdummy;
        freq_cell(gd, (int64_t)ev.k_lo, ev.N, fs, f_lo, tdummy);
        freq_cell(gd, (int64_t)(ev.k_lo + ev.nb - 1), ev.N, fs, f_hi, tdummy);
        n_nodes = f_hi - f_lo + 2;
    }
    constexpr int kRecWords = (int)(sizeof(MBin<T>) / 16);
    __shared__ uint4 stage[kBlock * kRecWords];
    const bool one_window = n_nodes <= kMaxSliceNodes;  // uniform
    for (int w0 = 0; w0 < n_nodes - 1; w0 += kMaxSliceNodes - 1) {
        const int wn = min(kMaxSliceNodes, n_nodes - w0);  // uniform over the workgroup
        if (w0 > 0) __syncthreads();                         // the previous window's reads are done
        for (int it = threadIdx.x; it < 4 * wn; it += blockDim.x)
            sl[it >> 2][it & 3] = slice1<Tt, T>(nodes, gd, f_lo + w0 + (it >> 2), it & 3, iz, (T)tz, ia, ja, (T)ta);
        __syncthreads();
        for (int j0 = 0; j0 < ev.nb; j0 += blockDim.x) {  // uniform trip count
            const int j = j0 + (int)threadIdx.x;
            MBin<T> m;
            bool have = false;
            if (j < ev.nb) {
                int ifr;
                double tf;
                freq_cell(gd, (int64_t)(ev.k_lo + j), ev.N, fs, ifr, tf);
                const int li = ifr - f_lo - w0;
                if (li >= 0 && li <= wn - 2) {  // else in another window
                    if constexpr (RESP) {
                        if (wq > 0.0) tf = rint(tf * wq) / wq;
                    }
                    C2<T> h[4];
#pragma unroll
                    for (int cp = 0; cp < 4; ++cp) h[cp] = clerp(sl[li][cp], sl[li + 1][cp], (T)tf);
                    if constexpr (RESP) {
                        m.p0 = h[0];
                        m.p1 = h[1];
                        m.q0 = h[2];
                        m.q1 = h[3];
                    } else {
                        m = coef_from_h<T>(h, ev.N, inv_n, fallback_rel, singular_rel, n_fb, n_sg);
                    }
                    have = true;
                }
            }
            if (one_window) {
                // every bin of the band is in this window: the block's records
                // go out through LDS as consecutive 16-byte words (a wave's
                // store covers 1 KiB of the row instead of 16 bytes of each of
                // 64 records)
                reinterpret_cast<MBin<T>*>(stage)[threadIdx.x] = m;
                __syncthreads();
                const int words = min((int)blockDim.x, ev.nb - j0) * kRecWords;
                uint4* dst = reinterpret_cast<uint4*>(out + j0);
                for (int c = threadIdx.x; c < words; c += blockDim.x) dst[c] = stage[c];
                __syncthreads();
            } else if (have) {
                out[j] = m;
            }
        }
    }
    if (!RESP && counts != nullptr) {
        if (n_fb) atomicAdd(&cnt[0], n_fb);
        if (n_sg) atomicAdd(&cnt[1], n_sg);
        __syncthreads();
        if (threadIdx.x < 2 && cnt[threadIdx.x])
            atomicAdd(&counts[threadIdx.x], (unsigned long long)cnt[threadIdx.x]);
    }
}

template <typename Tt, typename T, bool RESP>
__global__ __launch_bounds__(kBlock) void k_coef(const C2<Tt>* __restrict__ nodes, GridDev gd,
                                                 EvDesc ev0, const EvDesc* __restrict__ evs,
                                                 const int2* __restrict__ units,
                                                 const double* __restrict__ dirs, double zen1,
                                                 double az1, int64_t fs, double fallback_rel,
                                                 double singular_rel, MBin<T>* __restrict__ M,
                                                 unsigned long long* __restrict__ counts, double wq,
                                                 const int* __restrict__ skip = nullptr, int skip_stride = 0)
{
    coef_block<Tt, T, RESP>(blockIdx.x, nodes, gd, ev0, evs, units, dirs, zen1, az1, fs, fallback_rel, singular_rel,
                            M, counts, wq, skip, skip_stride);
}

// E-field traces of one (event, direction, station range) per block; each
// FFT group takes one station at a time.  Per station:
//   1. every in-band bin k is handled once: the packed spectrum
//      Z[k] = E_th + i E_ph, Z[N-k] = conj E_th + i conj E_ph comes straight
//      from the packed coefficients and (X_0, X_1) (see MBin) and is written
//      to LDS (DC keeps real parts only);
//   2. each thread reads its column of Z (zero outside the band);
//   3. inverse FFT; thread t ends with z[t + (N/E) i], whose real and
//      imaginary parts are E_theta and E_phi -- stored with non-temporal,
//      coalesced writes.
// With `counter` non-null the grid is persistent and blocks take units from
// the atomic counter until the list is exhausted (every block leaves through
// the same check); without, block b takes units b, b + grid, ...  Either way
// the per-thread twiddles are loaded once per block.
// Lane -> FFT thread index.  With PAIR, every wavefront plays FFT threads t
// (lanes 0-31) and TT - t (lanes 32-63, the partner of lane L is lane L ^ 32),
// so the mirror bin N - k of any bin k a lane holds lives in the partner
// lane (same register slot reflected), except for the self-mirrored threads
// 0 and TT/2, which lanes 0 and 32 of the group's first wave play.
template <int TT, bool PAIR>
__device__ __forceinline__ int fft_thread(int r)
{
    if constexpr (!PAIR) {
        return r;
    } else {
        const int wv = r >> 6, lane = r & 63;
        if (lane < 32) return 32 * wv + lane;
        const int u = 32 * wv + lane - 32;
        return u == 0 ? TT / 2 : TT - u;
    }
}

// An empty use of a value held in registers: the compiler must have it
// (and so wait for the load that produces it) at this point.
template <typename T>
__device__ __forceinline__ void touch(const C2<T>& v)
{
    asm volatile("" ::"v"(v.re), "v"(v.im));
}



// One in-band bin of the packed spectrum: Z[k] = E_theta + i E_phi and
// Z[N-k] = conj E_theta + i conj E_phi (only the real parts at k = 0).
// (XW: in the digit-reversed slots of the 4096-point in-wave transform)
template <typename T, int N, bool XW = false>
__device__ __forceinline__ int stage_slot(unsigned k)
{
    if constexpr (XW)
        return xw_slot(xw_pos((int)k));
    else
        return lpad<T>((int)k);
}

template <typename T, int N, bool XW = false>
__device__ __forceinline__ void stage_bin(C2<T>* __restrict__ lds, unsigned k, const MBin<T>& m, const XBin<T>& xb)
{
    C2<T> zp, zq;
    packed_bin(m, xb, zp, zq);
    if (k == 0) {
        lds[0] = packed_dc(zp, zq);
    } else {
        lds[stage_slot<T, N, XW>(k)] = zp;
        lds[stage_slot<T, N, XW>(N - k)] = C2<T>{zq.re, -zq.im};
    }
}

// Zero the spare zero slot of LDS buffer b of the block (G groups of one or
// two buffers, buffer after buffer); no transform writes it, and the gather
// reads it for out-of-band bins.
template <typename T, int N>
__device__ __forceinline__ void zero_slot_clear(unsigned char* smem, int b)
{
    reinterpret_cast<C2<T>*>(smem)[b * lds_elems<N>() + lds_zero_slot<N>()] = C2<T>{0, 0};
}

#ifndef AU_UNFOLD_PF
#define AU_UNFOLD_PF 2
#endif

// Minimum waves per SIMD the register allocator must leave room for: the
// FP32 shapes with 8 values per thread and two LDS buffers or paired lanes
// fit in 128 VGPRs (four waves per SIMD, the same as the plain 8-value shape)
// without spilling; unconstrained they take 129-130 and drop to three.  The
// FP64 8-value shape with hybrid twiddles and one buffer fits in 128 too
// (unconstrained 142: three waves, one 8-wave workgroup per CU; at four, two).
template <typename T, int E, int TWMODE, bool PAIR, bool PP>
constexpr int unfold_min_waves()
{
    if (sizeof(T) == 4 && E == 8 && (PAIR || PP)) return 4;
    if (sizeof(T) == 8 && E == 8 && tw_lds_early(TWMODE) && !PAIR && !PP) return 4;
    return 1;
}

template <typename T, int N, int E, int RMAX, int TWMODE, bool WAVE, bool PAIR, bool PP>
__global__ __launch_bounds__((N / E) > kBlock ? (N / E) : kBlock)
__attribute__((amdgpu_waves_per_eu(unfold_min_waves<T, E, TWMODE, PAIR, PP>()))) void k_unfold(EvDesc ev0, const EvDesc* __restrict__ evs,
                                                   const int4* __restrict__ units, int n_units,
                                                   int spw, const XBin<T>* __restrict__ X,
                                                   const MBin<T>* __restrict__ M,
                                                   T* __restrict__ efield,
                                                   const C2<T>* __restrict__ tw,
                                                   unsigned int* __restrict__ counter,
                                                   const int* __restrict__ xcd_off)
{
    constexpr int TT = N / E;
    constexpr int G = groups_per_block<T, N, E, PP ? 2 : 1>();
    // bins per thread prefetched for the next station: the FP32 shapes whose
    // early twiddles live in LDS have the registers for it; in FP64 the
    // two-buffer shape, at two waves per SIMD (one workgroup per CU, which
    // its LDS allows anyway)
    constexpr int PF = ((tw_lds_early(TWMODE) || TWMODE == TW_LFR || TWMODE == TW_LFW) && E <= 8 && !PAIR && !WAVE &&
                        (sizeof(T) == 4 || PP)) ? AU_UNFOLD_PF : 0;
    // the 4096-point transform with in-wavefront exchanges: the staging
    // writes the digit-reversed order it reads, the first buffer holds the
    // staging and the second its one exchange
    constexpr bool XW = TWMODE == TW_LFW;
    static_assert(!XW || (N == 4096 && E == 8 && RMAX == 8 && PP && !PAIR && !WAVE && G == 1 && PF > 0),
                  "in-wave exchanges: the 4096-point shape only");
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ int sh_u;
    __shared__ int sh_list;
    static_assert(!PAIR || ((N / E) % 64 == 0 && E % 2 == 0), "paired lanes need whole wavefronts");
    // g is stated as 0 with one group per block, so that the compiler treats
    // the station and everything derived from it as uniform
    const int g = G == 1 ? 0 : (int)(threadIdx.x / TT), t = fft_thread<TT, PAIR>(threadIdx.x % TT);
    // PP: two buffers per group; the staging exchange uses lds, the passes
    // alternate lds2, lds, ...
    C2<T>* lds = reinterpret_cast<C2<T>*>(smem) + g * (PP ? 2 : 1) * lds_elems<N>();
    C2<T>* lds2 = lds + lds_elems<N>();
    C2<T>* ltw = reinterpret_cast<C2<T>*>(smem) + G * (PP ? 2 : 1) * lds_elems<N>();
    C2<T> w[tw_count<N, E, RMAX, TWMODE>()];
    load_twiddles<T, N, E, RMAX, TWMODE, +1>(w, tw, t);
    if constexpr (tw_lds_early(TWMODE)) fill_lds_twiddles<T, N, E, RMAX, +1, TWMODE>(ltw, tw, threadIdx.x, blockDim.x);
    if constexpr (PF > 0) {  // (ordered by the barrier below)
        if (threadIdx.x < (PP ? 2 : 1) * G) zero_slot_clear<T, N>(smem, threadIdx.x);
    }
    // Wait for the twiddle loads here, once.  Left to the compiler, the wait
    // lands at their first use inside the station loop, where vector-memory
    // completions are counted in issue order: every station would then wait
    // for all stores of the station before it.
    vmem_wait_all();
    if constexpr (tw_lds_early(TWMODE) || PF > 0) lds_barrier();
    // XCD-aware placement (xcd_off != nullptr): the unit array holds 8 lists,
    // list x = [xcd_off[x], xcd_off[x+1]), built so that all units of one
    // event -- which share its spectrum rows, and per direction a coefficient
    // row -- sit in one list.  Workgroups are dispatched round-robin over the
    // 8 XCDs, so block b runs on XCD b mod 8 and takes its units from that
    // list (persistent: from that list's counter, then from the other lists
    // once it is empty), and those rows are fetched into one XCD's L2 only.
    if (threadIdx.x == 0) sh_list = blockIdx.x & 7;
    // XW: the band whose out-of-band slots of the staging buffer hold zeros
    unsigned zb_klo = ~0u, zb_nb = ~0u;
    for (int iter = 0;; ++iter) {
        int u;
        if (counter != nullptr) {
            if (threadIdx.x == 0) {
                int got = n_units;
                if (xcd_off != nullptr) {
                    for (int k = 0; k < 8; ++k) {
                        const int x = (sh_list + k) & 7;
                        const unsigned cnt = (unsigned)(xcd_off[x + 1] - xcd_off[x]);
                        if (cnt == 0) continue;
                        const unsigned i = atomicAdd(&counter[x], 1u);
                        if (i < cnt) {
                            got = xcd_off[x] + (int)i;
                            sh_list = x;
                            break;
                        }
                    }
                } else {
                    got = (int)atomicAdd(counter, 1u);
                }
                sh_u = got;
            }
            lds_barrier();
            u = sh_u;
            lds_barrier();
        } else {
            // without a counter, block b takes units b, b + grid, ... (of list
            // b mod 8 with XCD lists, the grid then a multiple of 8)
            if (xcd_off != nullptr) {
                const int x = blockIdx.x & 7;
                const int64_t i = (int64_t)(blockIdx.x >> 3) + (int64_t)iter * (gridDim.x >> 3);
                u = (i < xcd_off[x + 1] - xcd_off[x]) ? xcd_off[x] + (int)i : n_units;
            } else {
                const int64_t v = (int64_t)blockIdx.x + (int64_t)iter * gridDim.x;
                u = v < n_units ? (int)v : n_units;
            }
        }
        if (u >= n_units) break;
        int e = 0, d, s0, s1;
        if (units != nullptr) {
            const int4 wu = units[u];
            e = wu.x;
            d = wu.y;
            s0 = wu.z;
            s1 = wu.w;
        } else {
            const int chunks = (ev0.S + spw - 1) / spw;
            d = u / chunks;
            s0 = (u - d * chunks) * spw;
            s1 = min(ev0.S, s0 + spw);
        }
        const EvDesc ev = evs ? evs[e] : ev0;
        const MBin<T>* __restrict__ Md = M + ev.m_off + (int64_t)d * ev.nb;
        const unsigned nb = (unsigned)ev.nb, k_lo = (unsigned)ev.k_lo;
        if constexpr (XW) {
            // The staging writes in-band slots (and the pad slot) only and
            // nothing else writes this buffer, so zeros written once per
            // band stay: the gathers read every slot unconditionally.
            // (Every gather of the previous station is done: its exchange
            // barrier has passed.)
            if (k_lo != zb_klo || nb != zb_nb) {  // uniform
#pragma unroll
                for (int i = 0; i < E; ++i) lds[xw_slot(t + TT * i)] = C2<T>{0, 0};
                lds_barrier();
                zb_klo = k_lo;
                zb_nb = nb;
            }
        }
        MBin<T> pm[PF > 0 ? PF : 1];
        XBin<T> px[PF > 0 ? PF : 1];
        // loads of PF bins of station s (clamped: a valid station, bin nb-1 for
        // bins past the band, the twiddle table when the band is empty)
        auto prefetch_bins = [&](const MBin<T>* md, const XBin<T>* xe, int sv, unsigned nbv, const C2<T>* safe,
                                 int tv) {
#pragma unroll
            for (int q = 0; q < PF; ++q) {
                const unsigned j = min(tv + TT * q, nbv > 0 ? (int)nbv - 1 : 0);
                const MBin<T>* pmq = nbv > 0 ? md + j : reinterpret_cast<const MBin<T>*>(safe);
                pm[q] = *pmq;
                if constexpr (G == 1 && sizeof(XBin<T>) == 16) {
                    // uniform station: the row as a buffer range (one record
                    // of the twiddle table when the band is empty)
                    const __amdgpu_buffer_rsrc_t xr =
                        nbv > 0 ? buffer_range(xe + (int64_t)sv * nbv, nbv * (unsigned)sizeof(XBin<T>))
                                : buffer_range(safe, (unsigned)sizeof(XBin<T>));
                    px[q] = buffer_load16<XBin<T>>(xr, j * (unsigned)sizeof(XBin<T>));
                } else {
                    const XBin<T>* pxq =
                        nbv > 0 ? xe + (int64_t)sv * nbv + j : reinterpret_cast<const XBin<T>*>(safe);
                    px[q] = *pxq;
                }
            }
        };
        if constexpr (PF > 0) {
            prefetch_bins(Md, X + ev.x_off, min(s0 + g, s1 - 1), nb, tw, t);
            // Once per unit, take these loads in here (an empty use of every
            // loaded register): then the only loads outstanding at the top of
            // the station loop are the prefetch issued ahead of the previous
            // station's stores, and the wait for them leaves those stores in
            // flight.
#pragma unroll
            for (int q = 0; q < PF; ++q) {
                touch(pm[q].p0);
                touch(pm[q].p1);
                touch(pm[q].q0);
                touch(pm[q].q1);
                touch(px[q].x0);
                touch(px[q].x1);
            }
        }
        for (int base = s0; base < s1; base += G) {
            const int s = base + g;
            const bool active = s < s1;
            const XBin<T>* __restrict__ Xs = X + ev.x_off + (int64_t)s * ev.nb;
            C2<T> x[E];
            if constexpr (PAIR) {
                // registers i < E/2 hold bins k = t + TT i < N/2: solve them here;
                // registers i >= E/2 hold the mirrors of the partner's (or, for
                // t = 0 and TT/2, the lane's own) lower registers, Z[N - b] =
                // conj zq(b).
                C2<T> zqs[E / 2];
#pragma unroll
                for (int i = 0; i < E / 2; ++i) {
                    const unsigned k = t + TT * i;
                    const unsigned j = k - k_lo;
                    C2<T> zp{0, 0}, zq{0, 0};
                    if (active && j < nb) {
                        packed_bin(Md[j], Xs[j], zp, zq);
                        if (k == 0) zp = packed_dc(zp, zq);
                    }
                    zqs[i] = zq;
                    x[i] = zp;
                }
                const bool self0 = (t == 0), selfh = (t == TT / 2);
#pragma unroll
                for (int i = E / 2; i < E; ++i) {
                    const int jp = E - 1 - i;
                    C2<T> zq{__shfl_xor(zqs[jp].re, 32), __shfl_xor(zqs[jp].im, 32)};
                    if (selfh) zq = zqs[jp];
                    if (self0) zq = (i > E / 2) ? zqs[E - i] : C2<T>{0, 0};
                    x[i] = C2<T>{zq.re, -zq.im};
                }
                __builtin_amdgcn_s_setprio(0);
            } else {
                if constexpr (PF > 0) {
                    // Bins past the prefetched ones (a band wider than PF TT
                    // bins) are loaded here; the loop is skipped uniformly
                    // otherwise.
                    if (nb > (unsigned)(PF * TT) && (G == 1 || active))
                        for (unsigned j = t + TT * PF; j < nb; j += TT) stage_bin<T, N, XW>(lds, k_lo + j, Md[j], Xs[j]);
                    // The first PF bins of this thread were loaded ahead (at
                    // the unit's start, or before the previous station's
                    // stores).  Branch-free: every lane computes them, and a
                    // lane with nothing to write writes the spare pad slot
                    // (never read), so that the only wait for these loads is
                    // the one before their use.
#pragma unroll
                    for (int q = 0; q < PF; ++q) {
                        const unsigned j = t + TT * q;
                        const unsigned k = k_lo + j;
                        const bool ok = (G == 1 || active) && j < nb;
                        C2<T> zp, zq;
                        packed_bin(pm[q], px[q], zp, zq);
                        lds[ok ? stage_slot<T, N, XW>(k) : lds_pad_slot<N>()] = zp;
                        lds[(ok && k != 0) ? stage_slot<T, N, XW>(N - k) : lds_pad_slot<N>()] = C2<T>{zq.re, -zq.im};
                        // a band that includes DC (a uniform test, skipped
                        // otherwise): bin 0 keeps real parts only
                        if (q == 0 && k_lo == 0u && ok && k == 0) lds[0] = packed_dc(zp, zq);
                    }
                } else if (active) {
                    for (unsigned j = t; j < nb; j += TT) stage_bin<T, N>(lds, k_lo + j, Md[j], Xs[j]);
                }
                __builtin_amdgcn_s_setprio(0);
                lds_sync<WAVE>();
#pragma unroll
                for (int i = 0; i < E; ++i) {
                    if constexpr (XW) {
                        // position t + TT i of the digit-reversed order; out
                        // of band it holds the zero written for the band
                        x[i] = lds[xw_slot((int)(t + TT * i))];
                    } else {
                        const unsigned k = t + TT * i;
                        const unsigned kk = (k <= N / 2) ? k : N - k;
                        const bool inb = active && (kk - k_lo) < nb;
                        // with the prefetch the registers are short: a zero
                        // slot in place of a per-bin select (the compiler
                        // keeps the eight addresses for the unit)
                        if constexpr (PF > 0)
                            x[i] = lds[inb ? lpad<T>(k) : lds_zero_slot<N>()];
                        else
                            x[i] = inb ? lds[lpad<T>(k)] : C2<T>{0, 0};
                    }
                }
                if constexpr (!PP) lds_sync<WAVE>();
            }
            if constexpr (XW) {
                // staging in lds, both exchanges in lds2: the next station's
                // staging writes lds after this station's exchange barrier,
                // which every thread passes after its gathers from lds
                fft4096_xw<T, +1>(x, lds2, w, t);
            } else if constexpr (PP) {
                fft_pp<T, N, E, +1, TWMODE, RMAX, WAVE>(x, lds2, lds, tw, t, w, ltw);
                // exchanges this station: the staging one (lds, unless PAIR)
                // plus one per pass boundary, alternating from lds2; make the
                // next station's first write go to the buffer not gathered last
                constexpr int ex = num_passes<N, (RMAX < E ? RMAX : E)>() - 1;
                if constexpr ((ex % 2 == 1) == PAIR) {
                    C2<T>* tmp = lds;
                    lds = lds2;
                    lds2 = tmp;
                }
            } else {
                fft<T, N, E, +1, TWMODE, RMAX, WAVE>(x, lds, tw, t, w, ltw);
            }
            // From here to the next station's staging exchange (prefetch,
            // stores, staging) the wave runs at a raised issue priority: its
            // memory instructions and the short staging then go ahead of the
            // other workgroup's transform on the same SIMDs, which keeps the
            // store stream fed and shortens the barrier wait (+2-3 % at
            // N = 4096).  Not in FP64, whose one workgroup per CU has no
            // other workgroup to go ahead of (-2 % with the raise there).
            if constexpr (sizeof(T) == 4) __builtin_amdgcn_s_setprio(2);
            // Prefetch the next station's bins before this station's stores:
            // vector-memory completions are counted in issue order, so loads
            // issued after the stores would wait for every store to land.
            // Branch-free, clamped to a valid station and bin.
            if constexpr (PF > 0) prefetch_bins(Md, X + ev.x_off, min(s + G, s1 - 1), nb, tw, t);
            if constexpr (G == 1) {
                // one group per block: its station is always active and the
                // trace base uniform
                const __amdgpu_buffer_rsrc_t r = buffer_range(
                    efield + ev.efield_off + ((int64_t)d * ev.S + s) * 2 * N, 2 * N * (unsigned)sizeof(T));
                const unsigned toff = (unsigned)t * (unsigned)sizeof(T);
#pragma unroll
                for (int i = 0; i < E; ++i) {
                    buffer_store_nt(x[i].re, r, toff, (int)(TT * i * sizeof(T)));
                    buffer_store_nt(x[i].im, r, toff, (int)((N + TT * i) * sizeof(T)));
                }
            } else if (active) {
                T* out = efield + ev.efield_off + ((int64_t)d * ev.S + s) * 2 * N;
#pragma unroll
                for (int i = 0; i < E; ++i) {
                    __builtin_nontemporal_store(x[i].re, out + t + TT * i);
                    __builtin_nontemporal_store(x[i].im, out + N + t + TT * i);
                }
            }
        }
    }
}

// Envelope peaks (the timing step after the unfolding: the station time is
// the maximum of the Hilbert envelope of its E-field trace).  Per (direction,
// station) the in-band solution (E_th, E_ph) is packed twice:
//   Z[k]   = E_th + i E_ph,            Z[N-k]   = conj E_th + i conj E_ph
//   Zh[k]  = -i E_th + E_ph = -i Z[k],  Zh[N-k]  = i conj E_th - conj E_ph = i Z[N-k]
// (Zh is the packed spectrum of the Hilbert transforms H(e_th) + i H(e_ph),
// with H = IDFT(-i sgn(k) DFT)), both are inverse-transformed, and
// env = sqrt(e^2 + H(e)^2) is reduced to its maximum and the first sample
// attaining it, per component (decided on env^2, in the compute precision;
// the peak is the root of the largest square).  Optionally the traces are
// stored too.  A
// non-null skip flag that reads nonzero turns the launch into a no-op.
// Two complex floats: one 16-byte record of a coefficient row.
template <typename T>
struct alignas(16) C2x2 {
    C2<T> a, b;
};

// One float or double at byte offset voff + soff of a buffer range.
template <typename V>
__device__ __forceinline__ V buffer_load_scalar(__amdgpu_buffer_rsrc_t r, unsigned voff, int soff)
{
    if constexpr (sizeof(V) == 4) {
        return __builtin_bit_cast(V, __builtin_amdgcn_raw_buffer_load_b32(r, (int)voff, soff, 0));
    } else {
        return __builtin_bit_cast(V, __builtin_amdgcn_raw_buffer_load_b64(r, (int)voff, soff, 0));
    }
}

// ---------------------------------------------------------------------------
// Spectrum and unfold fused, for events with few directions (FP32)
// ---------------------------------------------------------------------------

// Events with at most this many directions take the fused kernel in batched
// plans (their work units then cover every direction of a station range).
constexpr int kFusedMaxDirs = 64;
// Stations per work unit of the fused kernel.
constexpr int kFusedStations = 8;

// One work unit (event, stations [s0, s1)) with ALL of the event's directions
// per workgroup (persistent grid, units taken as in k_unfold).  Per station:
//   1. its two channel traces (loaded ahead, after the previous station's
//      last staging and before its last stores) go through the forward
//      transform Z = F-(z), z = V_0 + i V_1, with the twiddles the inverse
//      transforms use (TW_LF entries serve both directions), and the
//      in-band split X_0 = (Z[k] + conj Z[N-k]) / 2, X_1 = (Z[k] -
//      conj Z[N-k]) / 2i: the operations of the streaming spectrum kernel
//      (up to the compiler's choice of which products it fuses into FMAs);
//   2. each thread keeps X of its bins k_lo + t + TT q (q < 2) in registers
//      (the same bins the unfold stages);
//   3. per direction: the packed coefficients of those bins (loaded ahead,
//      before the previous direction's stores) times X, staged in LDS, the
//      inverse transform, and the stores -- the operations of k_unfold.
// The spectra never reach HBM and each station is transformed forward once.
// Needs one transform per workgroup (N >= 2048) and bands of at most 2 TT
// bins (30-80 MHz at 200 MHz is N/4 bins).
template <typename Tin, int N>
__global__ __launch_bounds__(N / 8) __attribute__((amdgpu_waves_per_eu(4))) void k_unfold_fused(
    const Tin* __restrict__ volt, const EvDesc* __restrict__ evs, const int4* __restrict__ units, int n_units,
    const MBin<float>* __restrict__ M, float* __restrict__ efield, const C2<float>* __restrict__ tw,
    unsigned int* __restrict__ counter, const int* __restrict__ xcd_off)
{
    using T = float;
    constexpr int E = 8, RMAX = 8, TT = N / E, PF = 2;
    static_assert(TT >= 256 && PF * TT <= N, "one transform per workgroup");
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ int sh_u;
    __shared__ int sh_list;
    const int t = threadIdx.x;
    // la: staging and the inverse transform's second exchange; lb: the other
    C2<T>* la = reinterpret_cast<C2<T>*>(smem);
    C2<T>* lb = la + lds_elems<N>();
    C2<T>* ltw = lb + lds_elems<N>();
    C2<T> w[tw_count<N, E, RMAX, TW_LF>()];
    load_twiddles<T, N, E, RMAX, TW_LF, +1>(w, tw, t);
    fill_lds_twiddles<T, N, E, RMAX, +1, TW_LF>(ltw, tw, t, TT);
    if (t == 0) zero_slot_clear<T, N>(smem, 0);
    vmem_wait_all();
    lds_barrier();
    if (t == 0) sh_list = blockIdx.x & 7;
    // the next unit: from this XCD's list, then from the others (as k_unfold)
    auto next_unit = [&]() {
        int got = n_units;
        if (xcd_off != nullptr) {
            for (int k = 0; k < 8; ++k) {
                const int x = (sh_list + k) & 7;
                const unsigned cnt = (unsigned)(xcd_off[x + 1] - xcd_off[x]);
                if (cnt == 0) continue;
                const unsigned i = atomicAdd(&counter[x], 1u);
                if (i < cnt) {
                    got = xcd_off[x] + (int)i;
                    sh_list = x;
                    break;
                }
            }
        } else {
            got = (int)atomicAdd(counter, 1u);
        }
        return got;
    };
    Tin a[E], b[E];
    const unsigned toff_in = (unsigned)t * (unsigned)sizeof(Tin);
    // the two channel traces of one station (2 N samples from `base`)
    auto load_traces = [&](const Tin* base) {
        const __amdgpu_buffer_rsrc_t r = buffer_range(base, 2 * N * (unsigned)sizeof(Tin));
#pragma unroll
        for (int i = 0; i < E; ++i) {
            a[i] = buffer_load_scalar<Tin>(r, toff_in, (int)(TT * i * sizeof(Tin)));
            b[i] = buffer_load_scalar<Tin>(r, toff_in, (int)((N + TT * i) * sizeof(Tin)));
        }
    };
    // Units are reserved one ahead: the first station of the next unit is
    // loaded like any next station (before the last stores of the current
    // unit), so a unit start waits for no stores and small units (fewer
    // events in flight per XCD, coefficient rows kept in L2) cost nothing.
    if (t == 0) sh_u = next_unit();
    lds_barrier();
    // the unit index is uniform: stated so, the unit and its event are read by
    // scalar loads
    int u = __builtin_amdgcn_readfirstlane(sh_u);
    if (u < n_units) {
        const int4 w0 = units[u];
        load_traces(volt + evs[w0.x].volt_off + (int64_t)w0.z * 2 * N);
    }
    while (u < n_units) {
        lds_barrier();  // every wave has read sh_u
        if (t == 0) sh_u = next_unit();
        lds_barrier();
        const int un = __builtin_amdgcn_readfirstlane(sh_u);
        const int4 wu = units[u];  // (event, -, first station, end station)
        const EvDesc ev = evs[wu.x];
        const int s0 = wu.z, s1 = wu.w, D = ev.D;
        const unsigned nb = (unsigned)ev.nb, k_lo = (unsigned)ev.k_lo;
        const MBin<T>* __restrict__ Me = M + ev.m_off;
        const Tin* __restrict__ Ve = volt + ev.volt_off;
        // the first station of the next unit (null: none)
        const Tin* Vn = nullptr;
        if (un < n_units) {
            const int4 wn = units[un];
            Vn = volt + evs[wn.x].volt_off + (int64_t)wn.z * 2 * N;
        }
        // byte offsets of this thread's bins in a coefficient row, clamped to a
        // valid bin past the band (to the first record of the twiddle table
        // when the band is empty)
        unsigned jq[PF];
#pragma unroll
        for (int q = 0; q < PF; ++q)
            jq[q] = min((unsigned)(t + TT * q), nb > 0 ? nb - 1 : 0u) * (unsigned)sizeof(MBin<T>);
        // rows and traces as buffer ranges with scalar bases (uniform
        // direction and station): 32-bit lane offsets, no 64-bit addresses
        auto load_coef = [&](int d, MBin<T> (&pm)[PF]) {
            const __amdgpu_buffer_rsrc_t r = nb > 0 ? buffer_range(Me + (int64_t)d * nb, nb * (unsigned)sizeof(MBin<T>))
                                                    : buffer_range(tw, (unsigned)sizeof(MBin<T>));
#pragma unroll
            for (int q = 0; q < PF; ++q) {
                const C2x2<T> lo = buffer_load16<C2x2<T>>(r, jq[q]);
                const C2x2<T> hi = buffer_load16<C2x2<T>>(r, jq[q] + 16u);
                pm[q].p0 = lo.a;
                pm[q].p1 = lo.b;
                pm[q].q0 = hi.a;
                pm[q].q1 = hi.b;
            }
        };
        MBin<T> pm[PF];
        for (int s = s0; s < s1; ++s) {
            // 1. forward transform of the station, conj(F+(conj z)), through the
            // buffers in the inverse transforms' order (lb, la, lb: the same LDS
            // addresses); lb was gathered last, so every thread first passes a barrier
            C2<T> x[E];
#pragma unroll
            for (int i = 0; i < E; ++i) x[i] = C2<T>{(T)a[i], (T)b[i]};
            lds_barrier();
            fft_pp<T, N, E, -1, TW_LF, RMAX, false>(x, lb, la, tw, t, w, ltw);
            // the first direction's coefficients (issued after the previous
            // station's last stores, a transform and the split ago)
            load_coef(0, pm);
            // 2. the in-band split of this thread's bins, through la (natural
            // order; gathered last before the transform's final exchange)
#pragma unroll
            for (int i = 0; i < E; ++i) la[lpad<T>(t + TT * i)] = x[i];
            lds_barrier();
            XBin<T> px[PF];
#pragma unroll
            for (int q = 0; q < PF; ++q) {
                const unsigned j = (unsigned)(t + TT * q);
                const unsigned k = k_lo + j;
                const C2<T> za = la[j < nb ? lpad<T>(k) : lds_pad_slot<N>()];
                const C2<T> zb = la[j < nb ? lpad<T>((N - k) & (N - 1)) : lds_pad_slot<N>()];
                px[q].x0 = C2<T>{(T)0.5 * (za.re + zb.re), (T)0.5 * (za.im - zb.im)};
                px[q].x1 = C2<T>{(T)0.5 * (za.im + zb.im), (T)0.5 * (zb.re - za.re)};
            }
            lds_barrier();  // every split read done before the staging writes la
            // 3. every direction of the event; the last one is peeled off, so
            // that the next station's traces, loaded only there, are not held
            // in registers across the others
            auto direction = [&](int d, bool last) {
                // staging into la, as k_unfold (branch-free; lanes with nothing
                // to write write the pad slot)
#pragma unroll
                for (int q = 0; q < PF; ++q) {
                    const unsigned j = t + TT * q;
                    const unsigned k = k_lo + j;
                    const bool ok = j < nb;
                    C2<T> zp, zq;
                    packed_bin(pm[q], px[q], zp, zq);
                    la[ok ? lpad<T>(k) : lds_pad_slot<N>()] = zp;
                    la[(ok && k != 0) ? lpad<T>(N - k) : lds_pad_slot<N>()] = C2<T>{zq.re, -zq.im};
                    if (q == 0 && k_lo == 0u && ok && k == 0) la[0] = packed_dc(zp, zq);
                }
                __builtin_amdgcn_s_setprio(0);
                // the last direction: the next station's traces (this station's
                // X and coefficients are dead now), ahead of the stores; after
                // the unit's last station, the next unit's first
                if (last) {
                    const Tin* nx = s + 1 < s1 ? Ve + (int64_t)(s + 1) * 2 * N : Vn;
                    if (nx != nullptr) load_traces(nx);
                }
                lds_barrier();
#pragma unroll
                for (int i = 0; i < E; ++i) {
                    const unsigned k = t + TT * i;
                    const unsigned kk = (k <= N / 2) ? k : N - k;
                    const bool inb = (kk - k_lo) < nb;
                    x[i] = la[inb ? lpad<T>(k) : lds_zero_slot<N>()];
                }
                fft_pp<T, N, E, +1, TW_LF, RMAX, false>(x, lb, la, tw, t, w, ltw);
                __builtin_amdgcn_s_setprio(2);
                // the next direction's coefficients, ahead of the stores
                if (!last) load_coef(d + 1, pm);
                const __amdgpu_buffer_rsrc_t r =
                    buffer_range(efield + ev.efield_off + ((int64_t)d * ev.S + s) * 2 * N, 2 * N * (unsigned)sizeof(T));
                const unsigned toff = (unsigned)t * (unsigned)sizeof(T);
#pragma unroll
                for (int i = 0; i < E; ++i) {
                    buffer_store_nt(x[i].re, r, toff, (int)(TT * i * sizeof(T)));
                    buffer_store_nt(x[i].im, r, toff, (int)((N + TT * i) * sizeof(T)));
                }
            };
            for (int d = 0; d + 1 < D; ++d) direction(d, false);
            direction(D - 1, true);
        }
        __builtin_amdgcn_s_setprio(0);
        u = un;
    }
}

// ---------------------------------------------------------------------------
// One event, one direction, in one launch (the latency path)
// ---------------------------------------------------------------------------

// The single-direction call (au_unfold_event) for 2048 and 4096 samples:
// one workgroup per station runs the operations of the three launches of
// the general path -- the forward transform and in-band split of its two
// channel traces (as the fused kernel), the direction's coefficients of the
// bins it stages (the angular slice at the band's frequency nodes in LDS,
// then per bin the frequency interpolation and the inverse, as k_coef:
// every workgroup computes the same direction's coefficients, a few hundred
// bins), and the staging, inverse transform and stores of k_unfold -- so a
// small event pays one launch instead of three.  Workgroup 0 counts the
// fallback and singular bins (once per direction, as k_coef).  Needs bands
// of at most 2 N/8 bins and at most kMaxSliceNodes frequency nodes.
template <typename Tt, typename T, int N>
__global__ __launch_bounds__(N / 8) void k_event_fused(const C2<Tt>* __restrict__ nodes, GridDev gd, EvDesc ev,
                                                       const T* __restrict__ volt, double zen, double az, int64_t fs,
                                                       double fallback_rel, double singular_rel,
                                                       T* __restrict__ efield, const C2<T>* __restrict__ tw,
                                                       unsigned long long* __restrict__ counts)
{
    constexpr int E = 8, RMAX = 8, TT = N / E, PF = 2;
    static_assert(TT >= 256, "one transform per workgroup");
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ C2<T> sl[kMaxSliceNodes][4];
    __shared__ unsigned int cnt[2];
    const int t = threadIdx.x, s = blockIdx.x;
    C2<T>* la = reinterpret_cast<C2<T>*>(smem);
    C2<T>* lb = la + lds_elems<N>();
    C2<T>* ltw = lb + lds_elems<N>();
    C2<T> w[tw_count<N, E, RMAX, TW_LF>()];
    load_twiddles<T, N, E, RMAX, TW_LF, +1>(w, tw, t);
    fill_lds_twiddles<T, N, E, RMAX, +1, TW_LF>(ltw, tw, t, TT);
    if (t == 0) zero_slot_clear<T, N>(smem, 0);
    if (t < 2) cnt[t] = 0;
    // the direction's angular slice at the frequency nodes the band spans
    int iz, ia, ja;
    double tz, ta;
    angle_cells(gd, zen, az, iz, tz, ia, ja, ta);
    const unsigned nb = (unsigned)ev.nb, k_lo = (unsigned)ev.k_lo;
    int f_lo = 0, n_nodes = 0;
    if (nb > 0) {
        int f_hi;
        double tdummy;
        freq_cell(gd, (int64_t)k_lo, N, fs, f_lo, tdummy);
        freq_cell(gd, (int64_t)(k_lo + nb - 1), N, fs, f_hi, tdummy);
        n_nodes = f_hi - f_lo + 2;
    }
    for (int it = t; it < 4 * n_nodes; it += TT)
        sl[it >> 2][it & 3] = slice1<Tt, T>(nodes, gd, f_lo + (it >> 2), it & 3, iz, (T)tz, ia, ja, (T)ta);
    // the station's traces: forward transform conj(F+(conj z)), z = V_0 + i V_1
    const T* __restrict__ V = volt + ev.volt_off + (int64_t)s * 2 * N;
    C2<T> x[E];
#pragma unroll
    for (int i = 0; i < E; ++i) x[i] = C2<T>{V[t + TT * i], V[N + t + TT * i]};
    vmem_wait_all();
    lds_barrier();  // twiddle table, zero slot, slice and counters written
    fft_pp<T, N, E, -1, TW_LF, RMAX, false>(x, lb, la, tw, t, w, ltw);
    // in-band split of this thread's bins through la (gathered last before
    // the transform's final exchange): X_0 = (Z[k] + conj Z[N-k]) / 2,
    // X_1 = (Z[k] - conj Z[N-k]) / 2i
#pragma unroll
    for (int i = 0; i < E; ++i) la[lpad<T>(t + TT * i)] = x[i];
    lds_barrier();
    XBin<T> px[PF];
#pragma unroll
    for (int q = 0; q < PF; ++q) {
        const unsigned j = (unsigned)(t + TT * q);
        const unsigned k = k_lo + j;
        const C2<T> za = la[j < nb ? lpad<T>(k) : lds_pad_slot<N>()];
        const C2<T> zb = la[j < nb ? lpad<T>((N - k) & (N - 1)) : lds_pad_slot<N>()];
        px[q].x0 = C2<T>{(T)0.5 * (za.re + zb.re), (T)0.5 * (za.im - zb.im)};
        px[q].x1 = C2<T>{(T)0.5 * (za.im + zb.im), (T)0.5 * (zb.re - za.re)};
    }
    lds_barrier();  // every split read done before the staging writes la
    // the coefficients of this thread's bins, the packed solve, the staging
    const T inv_n = (T)(1.0 / (double)N);
    unsigned int n_fb = 0, n_sg = 0;
#pragma unroll
    for (int q = 0; q < PF; ++q) {
        const unsigned j = t + TT * q;
        const unsigned k = k_lo + j;
        const bool ok = j < nb;
        MBin<T> m{};
        if (ok) {
            int ifr;
            double tf;
            freq_cell(gd, (int64_t)k, N, fs, ifr, tf);
            const int li = ifr - f_lo;
            C2<T> h[4];
#pragma unroll
            for (int cp = 0; cp < 4; ++cp) h[cp] = clerp(sl[li][cp], sl[li + 1][cp], (T)tf);
            m = coef_from_h<T>(h, N, inv_n, fallback_rel, singular_rel, n_fb, n_sg);
        }
        C2<T> zp, zq;
        packed_bin(m, px[q], zp, zq);
        la[ok ? lpad<T>(k) : lds_pad_slot<N>()] = zp;
        la[(ok && k != 0) ? lpad<T>(N - k) : lds_pad_slot<N>()] = C2<T>{zq.re, -zq.im};
        if (q == 0 && k_lo == 0u && ok && k == 0) la[0] = packed_dc(zp, zq);
    }
    if (s == 0 && counts != nullptr) {
        if (n_fb) atomicAdd(&cnt[0], n_fb);
        if (n_sg) atomicAdd(&cnt[1], n_sg);
    }
    lds_barrier();
#pragma unroll
    for (int i = 0; i < E; ++i) {
        const unsigned k = t + TT * i;
        const unsigned kk = (k <= N / 2) ? k : N - k;
        x[i] = la[(kk - k_lo) < nb ? lpad<T>(k) : lds_zero_slot<N>()];
    }
    fft_pp<T, N, E, +1, TW_LF, RMAX, false>(x, lb, la, tw, t, w, ltw);
    const __amdgpu_buffer_rsrc_t r = buffer_range(efield + ev.efield_off + (int64_t)s * 2 * N, 2 * N * (unsigned)sizeof(T));
    const unsigned toff = (unsigned)t * (unsigned)sizeof(T);
#pragma unroll
    for (int i = 0; i < E; ++i) {
        buffer_store_nt(x[i].re, r, toff, (int)(TT * i * sizeof(T)));
        buffer_store_nt(x[i].im, r, toff, (int)((N + TT * i) * sizeof(T)));
    }
    if (s == 0 && counts != nullptr && t < 2 && cnt[t]) atomicAdd(&counts[t], (unsigned long long)cnt[t]);
}

// Shape of the envelope kernel.  FP32, and FP64 at 8 values per thread: the
// two transforms run in lockstep (fft2) through two LDS buffers, with the
// early passes' twiddles from the LDS table and the rest in registers, as
// (tangent, cosine) pairs for the fused multiply-add butterflies (TW_LF) at
// 8 values per thread.  FP64 at 16 values per thread (N < 1024):
// the registers do not hold two transforms, so they run one after the other
// through one buffer with table twiddles.
template <typename T, int E>
constexpr bool env_dual() { return sizeof(T) == 4 || E <= 8; }
template <typename T, int E>
constexpr int env_twmode() { return env_dual<T, E>() && E <= 8 ? TW_LF : TW_TABLE; }
template <typename T, int N, int E>
constexpr int env_ltw() { return tw_lds_early(env_twmode<T, E>()) ? ltw_count<N, E, E, env_twmode<T, E>()>() : 0; }
template <typename T, int E>
constexpr int env_bufs() { return env_dual<T, E>() ? 2 : 1; }

template <typename T, int N, int E>
__global__ __launch_bounds__((N / E) > kBlock ? (N / E) : kBlock) void k_unfold_env(
    EvDesc ev0, int spw, const XBin<T>* __restrict__ X, const MBin<T>* __restrict__ M, T* __restrict__ efield,
    T* __restrict__ peak, int* __restrict__ arg, const C2<T>* __restrict__ tw, const int* __restrict__ skip,
    const EvDesc* __restrict__ evs, const int4* __restrict__ units, int skip_stride, int total_only)
{
    constexpr int TT = N / E;
    constexpr int G = groups_per_block<T, N, E, env_bufs<T, E>()>();
    constexpr int NW = (TT + 63) / 64;  // waves per group
    constexpr int TWM = env_twmode<T, E>();
    constexpr bool DUAL = env_dual<T, E>();
    // FP64 at 4096 samples: the two transforms in fft4096_xw2's form; the
    // first buffer holds the staged Z (digit-reversed, zeros out of band)
    // and later the Hilbert transform's workgroup exchange, the second the
    // wavefront-local transposes, the trace's exchange and the reduction
    constexpr bool XWE = sizeof(T) == 8 && N == 4096 && E == 8 && G == 1 && DUAL && TWM == TW_LF;
    // one event (ev0; workgroup = direction x chunk of spw stations), or many
    // (units[b] = (event, direction, s0, s1) with descriptors evs[]; then
    // ev.efield_off is the element offset of the event's [D][S][3] peak and
    // sample block and no traces are stored)
    int e = 0, d, s0, s1;
    if (units != nullptr) {
        const int4 u = units[blockIdx.x];
        e = u.x;
        d = u.y;
        s0 = u.z;
        s1 = u.w;
    } else {
        const int chunks = (ev0.S + spw - 1) / spw;
        d = blockIdx.x / chunks;
        s0 = (blockIdx.x - d * chunks) * spw;
        s1 = min(ev0.S, s0 + spw);
    }
    if (skip != nullptr && skip[(int64_t)e * skip_stride]) return;  // set by a converged reconstruction loop
    const EvDesc ev = units != nullptr ? evs[e] : ev0;
    const int64_t pk_off = units != nullptr ? ev.efield_off : 0;
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ T red_v[G][NW][3];
    __shared__ int red_i[G][NW][3];
    // g stated as 0 with one group per block: per-station values stay uniform
    const int g = G == 1 ? 0 : (int)(threadIdx.x / TT), t = threadIdx.x % TT;
    C2<T>* la = reinterpret_cast<C2<T>*>(smem) + g * env_bufs<T, E>() * lds_elems<N>();
    C2<T>* lb = DUAL ? la + lds_elems<N>() : la;
    C2<T>* ltw = reinterpret_cast<C2<T>*>(smem) + G * env_bufs<T, E>() * lds_elems<N>();
    C2<T> w[tw_count<N, E, E, TWM>()];
    load_twiddles<T, N, E, E, TWM, +1>(w, tw, t);
    if constexpr (tw_lds_early(TWM)) {
        fill_lds_twiddles<T, N, E, E, +1, TWM>(ltw, tw, threadIdx.x, blockDim.x);
        if constexpr (XWE) {
            // the staging buffer's zeros (the staging writes in-band slots only)
#pragma unroll
            for (int i = 0; i < E; ++i) la[xw_slot(t + TT * i)] = C2<T>{0, 0};
        }
        lds_barrier();
    }
    const unsigned nb = (unsigned)ev.nb, k_lo = (unsigned)ev.k_lo;
    const MBin<T>* __restrict__ Md = M + ev.m_off + (int64_t)d * ev.nb;
    // Bins per thread loaded one station ahead (FP64, one transform pair per
    // workgroup, which has the registers at two waves per SIMD): their loads
    // then overlap the current station's transforms instead of opening the
    // next station's staging.  Clamped like k_unfold's: a valid station, bin
    // nb-1 for bins past the band, the twiddle table when the band is empty.
    // Not in the in-wavefront form, which needs those registers (with them it
    // spills and runs 9 % slower).
    constexpr int PF = (!XWE && sizeof(T) == 8 && E == 8 && G == 1 && DUAL) ? 2 : 0;
    MBin<T> pm[PF > 0 ? PF : 1];
    XBin<T> px[PF > 0 ? PF : 1];
    auto prefetch = [&](int sv) {
        const XBin<T>* __restrict__ xs = X + ev.x_off + (int64_t)sv * ev.nb;
#pragma unroll
        for (int q = 0; q < PF; ++q) {
            const unsigned j = min((unsigned)(t + TT * q), nb > 0 ? nb - 1 : 0u);
            pm[q] = nb > 0 ? Md[j] : *reinterpret_cast<const MBin<T>*>(tw);
            px[q] = nb > 0 ? xs[j] : *reinterpret_cast<const XBin<T>*>(tw);
        }
    };
    if constexpr (PF > 0) prefetch(min(s0, s1 - 1));
    // Z[k] = zp, Z[N-k] = conj zq; the Hilbert spectrum Zh[k] = -i Z[k],
    // Zh[N-k] = i Z[N-k]; a lane with nothing to write (ok false) writes the
    // spare pad slot, which no gather reads
    auto stage = [&](int h, unsigned j, const C2<T>& zp, const C2<T>& zq, bool ok) {
        const unsigned k = k_lo + j;
        if constexpr (XWE) {
            // Z only: the gathers derive Zh
            if (ok && k == 0) {
                la[0] = packed_dc(zp, zq);
            } else {
                la[ok ? stage_slot<T, N, true>(k) : lds_pad_slot<N>()] = zp;
                la[ok ? stage_slot<T, N, true>(N - k) : lds_pad_slot<N>()] = C2<T>{zq.re, -zq.im};
            }
            return;
        }
        if (ok && k == 0) {
            if (DUAL || h == 0) la[0] = packed_dc(zp, zq);
            if (DUAL || h == 1) lb[0] = C2<T>{0, 0};
        } else {
            const int a = ok ? lpad<T>(k) : lds_pad_slot<N>(), b = ok ? lpad<T>(N - k) : lds_pad_slot<N>();
            if (DUAL || h == 0) {
                la[a] = zp;
                la[b] = C2<T>{zq.re, -zq.im};
            }
            if (DUAL || h == 1) {
                lb[a] = C2<T>{zp.im, -zp.re};
                lb[b] = C2<T>{zq.im, zq.re};
            }
        }
    };
    for (int base = s0; base < s1; base += G) {
        const int s = base + g;
        const bool active = s < s1;
        const XBin<T>* __restrict__ Xs = X + ev.x_off + (int64_t)s * ev.nb;
        // the packed spectra: Z into la and Zh into lb at once (DUAL), or Z
        // then Zh through the one buffer
        C2<T> x[E], xh[E];
        // the staging (coefficient and spectrum loads, LDS writes) at a raised
        // issue priority, ahead of other workgroups' transforms on the same
        // SIMDs, as in k_unfold (+1.2-1.5 % on the 2048-direction scans)
        __builtin_amdgcn_s_setprio(2);
#pragma unroll
        for (int h = 0; h < (DUAL ? 1 : 2); ++h) {
            if constexpr (PF > 0) {
                // bins past the prefetched ones (a band wider than PF TT bins)
                if (active && nb > (unsigned)(PF * TT))
                    for (unsigned j = t + TT * PF; j < nb; j += TT) {
                        C2<T> zp, zq;
                        packed_bin(Md[j], Xs[j], zp, zq);
                        stage(h, j, zp, zq, true);
                    }
#pragma unroll
                for (int q = 0; q < PF; ++q) {
                    const unsigned j = t + TT * q;
                    C2<T> zp, zq;
                    packed_bin(pm[q], px[q], zp, zq);
                    stage(h, j, zp, zq, active && j < nb);
                }
                // the next station's bins, ahead of this station's transforms
                prefetch(min(s + G, s1 - 1));
            } else if (active) {
                for (unsigned j = t; j < nb; j += TT) {
                    C2<T> zp, zq;
                    packed_bin(Md[j], Xs[j], zp, zq);
                    stage(h, j, zp, zq, true);
                }
            }
            lds_barrier();
            if constexpr (XWE) {
                // position t + TT i holds element 512 i + c, c < 512: below
                // N/2 for i < 4, where Zh = -i Z, above for i >= 4, Zh = i Z;
                // Zh = 0 at DC (thread 0, register 0)
#pragma unroll
                for (int i = 0; i < E; ++i) {
                    x[i] = la[xw_slot(t + TT * i)];
                    xh[i] = i < E / 2 ? C2<T>{x[i].im, -x[i].re} : C2<T>{-x[i].im, x[i].re};
                }
                if (t == 0) xh[0] = C2<T>{0, 0};
                continue;  // no barrier: the transposes write the other buffer
            }
#pragma unroll
            for (int i = 0; i < E; ++i) {
                const unsigned k = t + TT * i;
                const unsigned kk = (k <= N / 2) ? k : N - k;
                const bool inb = active && (kk - k_lo) < nb;
                if (DUAL || h == 0) x[i] = inb ? la[lpad<T>(k)] : C2<T>{0, 0};
                if (DUAL || h == 1) xh[i] = inb ? lb[lpad<T>(k)] : C2<T>{0, 0};
            }
            lds_barrier();
        }
        __builtin_amdgcn_s_setprio(0);
        if constexpr (XWE) {
            fft4096_xw2<T, +1, TWM>(x, xh, lb, la, w, t, ltw);
        } else if constexpr (DUAL) {
            fft2<T, N, E, +1, TWM, E>(x, xh, la, lb, tw, t, w, ltw);
        } else {
            fft<T, N, E, +1>(x, la, tw, t);
            fft<T, N, E, +1>(xh, la, tw, t);
        }
        // per-thread maxima over its samples n = t + TT i (increasing in i) of
        // the squared theta, phi and total-field envelopes: the square root is
        // monotone, so it is taken once, of the largest square (a correctly
        // rounded root per sample is some fifteen instructions)
        T bv[3] = {(T)-1, (T)-1, (T)-1};
        int bi[3] = {0, 0, 0};
        // with total_only (a uniform flag: the batched loop and the direction
        // fit read only the total field; the one-event loop also returns the
        // theta and phi peaks) the component maxima are neither tracked nor
        // stored
        const int c_lo = (TT >= 256 && total_only) ? 2 : 0;
        if (c_lo == 2) {
#pragma unroll
            for (int i = 0; i < E; ++i) {
                const T p0 = x[i].re * x[i].re + xh[i].re * xh[i].re;
                const T p1 = x[i].im * x[i].im + xh[i].im * xh[i].im;
                const T p = p0 + p1;  // as in the three-component form
                if (p > bv[2]) {
                    bv[2] = p;
                    bi[2] = t + TT * i;
                }
            }
        } else {
#pragma unroll
            for (int i = 0; i < E; ++i) {
                const T p0 = x[i].re * x[i].re + xh[i].re * xh[i].re;
                const T p1 = x[i].im * x[i].im + xh[i].im * xh[i].im;
                const T e[3] = {p0, p1, p0 + p1};
#pragma unroll
                for (int c = 0; c < 3; ++c)
                    if (e[c] > bv[c]) {
                        bv[c] = e[c];
                        bi[c] = t + TT * i;
                    }
            }
        }
        // larger value wins; equal values: smaller sample index.
        if constexpr (TT >= 256) {
            // Three waves reduce one component each: every thread leaves its
            // three candidates in the first buffer (the transforms' last
            // gathers are behind a barrier, so it is free), then wave c scans
            // component c (TT / 64 candidates per lane and a butterfly)
            // while the other waves go on -- a fraction of the VALU work of a
            // three-component butterfly in every wave.
            T* cv = reinterpret_cast<T*>(XWE ? lb : la);
            int* ci = reinterpret_cast<int*>(cv + 3 * TT);
            static_assert(3 * TT * (sizeof(T) + sizeof(int)) <= lds_elems<N>() * sizeof(C2<T>), "scratch");
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                if (c < c_lo) continue;
                cv[c * TT + t] = bv[c];
                ci[c * TT + t] = bi[c];
            }
            lds_barrier();
            if constexpr (XWE) {
                // every read of the Hilbert exchange in the first buffer is
                // behind that barrier: its zeros back before the closing one
#pragma unroll
                for (int i = 0; i < E; ++i) la[xw_slot(t + TT * i)] = C2<T>{0, 0};
            }
            const int wv = t >> 6, lane = t & 63;
            const int cc = c_lo + wv;  // the component this wave reduces
            if (cc < 3 && active) {  // whole waves: no barrier inside
                // the reducing waves run ahead of the others' issue (which
                // only reach the station's closing barrier): +6 % FP32
                __builtin_amdgcn_s_setprio(2);
                T v = cv[cc * TT + lane];
                int ix = ci[cc * TT + lane];
#pragma unroll
                for (int k = lane + 64; k < TT; k += 64) {
                    const T ov = cv[cc * TT + k];
                    const int oi = ci[cc * TT + k];
                    if (ov > v || (ov == v && oi < ix)) {
                        v = ov;
                        ix = oi;
                    }
                }
                for (int off = 32; off >= 1; off >>= 1) {
                    const T ov = __shfl_xor(v, off);
                    const int oi = __shfl_xor(ix, off);
                    if (ov > v || (ov == v && oi < ix)) {
                        v = ov;
                        ix = oi;
                    }
                }
                if (lane == 0) {
                    const int64_t o = pk_off + ((int64_t)d * ev.S + s) * 3 + cc;
                    peak[o] = sqrt(v);
                    arg[o] = ix;
                }
                __builtin_amdgcn_s_setprio(0);
            }
        } else {
            // A group of TT < 64 threads shares its wave with other groups, so the
            // butterfly stays within the group's TT lanes.
            constexpr int kShfl = TT < 64 ? TT / 2 : 32;
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                for (int off = kShfl; off >= 1; off >>= 1) {
                    const T ov = __shfl_xor(bv[c], off);
                    const int oi = __shfl_xor(bi[c], off);
                    if (ov > bv[c] || (ov == bv[c] && oi < bi[c])) {
                        bv[c] = ov;
                        bi[c] = oi;
                    }
                }
            }
            const int wv = t >> 6;
            if ((t & 63) == 0) {
#pragma unroll
                for (int c = 0; c < 3; ++c) {
                    red_v[g][wv][c] = bv[c];
                    red_i[g][wv][c] = bi[c];
                }
            }
            lds_barrier();
            // components c = t, t + TT, ... (a group of N = 16 or 32 has fewer than 3 threads)
            for (int c = t; active && c < 3; c += TT) {
                T v = red_v[g][0][c];
                int ix = red_i[g][0][c];
                for (int w2 = 1; w2 < NW; ++w2) {
                    const T ov = red_v[g][w2][c];
                    const int oi = red_i[g][w2][c];
                    if (ov > v || (ov == v && oi < ix)) {
                        v = ov;
                        ix = oi;
                    }
                }
                const int64_t o = pk_off + ((int64_t)d * ev.S + s) * 3 + c;
                peak[o] = sqrt(v);
                arg[o] = ix;
            }
        }
        if (active && efield != nullptr && units == nullptr) {
            T* out = efield + ((int64_t)d * ev.S + s) * 2 * N;
#pragma unroll
            for (int i = 0; i < E; ++i) {
                __builtin_nontemporal_store(x[i].re, out + t + TT * i);
                __builtin_nontemporal_store(x[i].im, out + N + t + TT * i);
            }
        }
        lds_barrier();
    }
}

__global__ void k_zero_u32(unsigned int* p, int n)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0u;
}

// ---------------------------------------------------------------------------
// launch dispatch over N (compile-time FFT sizes)
// ---------------------------------------------------------------------------

#define AU_FOR_EACH_N(X) X(16) X(32) X(64) X(128) X(256) X(512) X(1024) X(2048) X(4096)

// Values per thread of the forward (station) FFTs.
constexpr int kE = 16;

template <typename T, int N>
struct Shape {
    static constexpr int E = kE;
    static constexpr int TT = N / E;
    static constexpr int G = groups_per_block<T, N, E>();
    static constexpr int BLOCK = G * TT;
    static constexpr size_t LDS = (size_t)G * lds_elems<N>() * sizeof(C2<T>);
};

// Shapes the unfold kernel is built in.  E: values per thread (0 = one
// wavefront per transform, E = N/64); RMAX: largest radix per pass (the
// radix schedule); twmode: where the inverse transform's twiddles live (see
// TW_* in au_device.h); wave: the transform is owned by one wavefront and
// its passes need no workgroup barrier.  The autotuner times them per
// (trace length, precision).
struct UnfoldVariant {
    int E;
    int rmax;
    int twmode;
    bool wave;
    bool pair;  // mirror-paired lanes: bins solved once, mirrors by a cross-lane swap
    bool pp;    // two LDS buffers per transform: one barrier per exchange
};
constexpr UnfoldVariant kUnfoldVariants[] = {
    {16, 16, TW_REG, false, false, false}, {16, 16, TW_TABLE, false, false, false},
    {8, 8, TW_REG, false, false, false},   {8, 8, TW_TABLE, false, false, false},
    {32, 32, TW_REG, false, false, false}, {32, 32, TW_TABLE, false, false, false},
    {0, 16, TW_SPLIT, true, false, false}, {0, 8, TW_SPLIT, true, false, false},
    {8, 8, TW_REG, false, true, false},    {16, 16, TW_REG, false, true, false},
    {8, 8, TW_REG, false, false, true},    {16, 16, TW_REG, false, false, true},
    {8, 8, TW_HYB, false, false, true},    {8, 8, TW_HYB, false, false, false},
    {8, 8, TW_LF, false, false, true},     {8, 8, TW_LF, false, false, false},
    {8, 8, TW_LFR, false, false, true},    {8, 8, TW_LFW, false, false, true},
};
constexpr int kNumVariants = 18;

// LDS one workgroup may allocate on gfx950 (the whole 160 KiB of a CU).
constexpr int kMaxLdsPerBlock = 163840;

constexpr int variant_e(int n, int v) { return kUnfoldVariants[v].E == 0 ? n / 64 : kUnfoldVariants[v].E; }

// Every variant for the long traces, the E=16 pair for the rest.  Shapes that
// do not fit the register file are not built: more than 16 complex doubles
// per thread, 32 complex doubles in the block form, and wavefront-owned
// transforms above 16 values per lane (N > 1024).
constexpr bool variant_built(int n, int v, int tsize)
{
    if (v < 0 || v >= kNumVariants) return false;
    if (v >= 2 && n < 1024) return false;
    const int e = variant_e(n, v);
    if (e < 8 || e > (tsize == 8 ? 16 : 32)) return false;
    if (kUnfoldVariants[v].wave && e > 16) return false;
    if (kUnfoldVariants[v].rmax > e) return false;
    if (kUnfoldVariants[v].pair && ((n / e) % 64 != 0 || e % 2 != 0)) return false;
    if (kUnfoldVariants[v].pp && 2 * (n + 16) * 2 * tsize > kMaxLdsPerBlock) return false;  // 2 x lds_elems
    // every pass's twiddle pairs in registers: FP64 (one workgroup per CU,
    // registers to spare); FP32 shapes need them for four waves per SIMD
    if (kUnfoldVariants[v].twmode == TW_LFR && tsize != 8) return false;
    // the in-wavefront exchanges exist for the 4096-point transform only, in
    // FP64 (the FP32 shape would spill at four waves per SIMD)
    if (kUnfoldVariants[v].twmode == TW_LFW && (n != 4096 || tsize != 8)) return false;
    return true;
}

template <typename T, int N, int V>
struct UShape {
    static constexpr int E0 = variant_e(N, V);
    static constexpr int E = E0 < N ? E0 : N;
    static constexpr int RMAX = kUnfoldVariants[V].rmax < E ? kUnfoldVariants[V].rmax : E;
    static constexpr int TWMODE = kUnfoldVariants[V].twmode;
    static constexpr bool WAVE = kUnfoldVariants[V].wave;
    static constexpr bool PAIR = kUnfoldVariants[V].pair;
    static constexpr bool PP = kUnfoldVariants[V].pp;
    static constexpr int BUFS = PP ? 2 : 1;
    static constexpr int TT = N / E;
    static constexpr int G = groups_per_block<T, N, E, BUFS>();
    static constexpr int BLOCK = G * TT;
    static constexpr size_t LDS =
        ((size_t)G * BUFS * lds_elems<N>() + (tw_lds_early(TWMODE) ? ltw_count<N, E, RMAX, TWMODE>() : 0)) *
        sizeof(C2<T>);
};

static int ilog2(int n)
{
    int l = 0;
    while ((1 << l) < n) ++l;
    return l;
}

// Selected variant per [precision][log2 N]; the defaults are the shapes
// that measured fastest on MI355X (from 1024 samples up, E=8 with two LDS
// buffers and the next station's bins prefetched: for float the fused
// multiply-add butterflies with the early passes' twiddle pairs in LDS, for
// double at 4096 samples the same butterflies with every pass's pairs in
// registers and two of the three exchanges inside the wavefront, at 2048
// the hybrid table, at 1024 register twiddles; below, E=16 with register
// twiddles for float and table twiddles for double).
static std::mutex g_var_mu;
static int g_variant[2][13] = {{1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 10, 12, 17},
                               {0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 12, 14, 14}};

static int unfold_variant(int prec, int n)
{
    std::lock_guard<std::mutex> lk(g_var_mu);
    return g_variant[prec == AU_PREC_FP32 ? 1 : 0][ilog2(n)];
}

// Workgroups of k_spectrum_stream the device holds at once (0 if unknown).
template <typename Tin, int N>
static int spectrum_stream_blocks()
{
    static const int blocks = [] {
        constexpr size_t lds = (lds_elems<N>() + ltw_count<N, 8, 8, TW_LF>()) * sizeof(C2<float>);
        int dev = 0, cus = 0, occ = 0;
        if (hipGetDevice(&dev) != hipSuccess ||
            hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
            hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, k_spectrum_stream<Tin, N>, N / 8, lds) != hipSuccess)
            return 0;
        return cus * occ;
    }();
    return blocks;
}

// max_nb: the largest band (bins) of the launch's events.
template <typename Tin, typename T, int N>
static hipError_t launch_spectrum_n(hipStream_t st, const Tin* volt, const EvDesc& ev0,
                                    const EvDesc* evs, const int2* units, int n_units, int max_nb,
                                    XBin<T>* X, const C2<T>* tw)
{
    using S = Shape<T, N>;
    if (n_units <= 0) return hipSuccess;
    if constexpr (sizeof(T) == 4 && N >= 1024) {
        const int blocks = spectrum_stream_blocks<Tin, N>();
        if (max_nb <= kSpecStreamBins * (N / 8) && blocks > 0) {
            constexpr size_t lds = (lds_elems<N>() + ltw_count<N, 8, 8, TW_LF>()) * sizeof(C2<float>);
            hipLaunchKernelGGL((k_spectrum_stream<Tin, N>), dim3(std::min(n_units, blocks)), dim3(N / 8), lds,
                               st, volt, ev0, evs, units, n_units, X, tw);
            return hipGetLastError();
        }
    }
    const int grid = (n_units + S::G - 1) / S::G;
    hipLaunchKernelGGL((k_spectrum<Tin, T, N, S::E>), dim3(grid), dim3(S::BLOCK), S::LDS, st, volt,
                       ev0, evs, units, n_units, X, tw);
    return hipGetLastError();
}

// Persistent grid of the fused kernel: as many workgroups as the device holds.
template <typename Tin, int N>
static int fused_blocks()
{
    static const int blocks = [] {
        constexpr size_t lds = (2 * lds_elems<N>() + ltw_count<N, 8, 8, TW_LF>()) * sizeof(C2<float>);
        int dev = 0, cus = 0, occ = 0;
        if (hipGetDevice(&dev) != hipSuccess ||
            hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
            hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, k_unfold_fused<Tin, N>, N / 8, lds) != hipSuccess)
            return 0;
        return cus * occ;
    }();
    return blocks;
}

// Whether a class of N-sample events with up to max_dirs directions and
// bands of up to max_nb bins takes the fused kernel.
static bool fused_eligible(int prec, int n, int max_dirs, int max_nb)
{
    return prec == AU_PREC_FP32 && (n == 2048 || n == 4096) && max_dirs <= kFusedMaxDirs && max_nb <= 2 * (n / 8);
}

template <typename Tin>
static hipError_t launch_fused(int n, hipStream_t st, const Tin* volt, const EvDesc* evs, const int4* units,
                               int n_units, const MBin<float>* M, float* efield, const C2<float>* tw,
                               unsigned int* counter, const int* xcd_off)
{
    if (n_units <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_zero_u32, dim3(1), dim3(64), 0, st, counter, 8);
    switch (n) {
#define F_(NN)                                                                                                  \
    case NN: {                                                                                                  \
        constexpr size_t lds = (2 * lds_elems<NN>() + ltw_count<NN, 8, 8, TW_LF>()) * sizeof(C2<float>);       \
        const int blocks = fused_blocks<Tin, NN>();                                                             \
        if (blocks <= 0) return hipErrorInvalidValue;                                                           \
        hipLaunchKernelGGL((k_unfold_fused<Tin, NN>), dim3(std::min(n_units, blocks)), dim3(NN / 8), lds, st,  \
                           volt, evs, units, n_units, M, efield, tw, counter, xcd_off);                         \
        return hipGetLastError();                                                                               \
    }
        F_(2048) F_(4096)
#undef F_
    }
    return hipErrorInvalidValue;
}

template <typename T, int N, int V>
static int occupancy_nv();

// Workgroups of unfold variant V the device holds at once (cached; 256 if
// the occupancy query fails).
template <typename T, int N, int V>
static int resident_blocks()
{
    static const int blocks = [] {
        int dev = 0, cus = 0;
        const int occ = occupancy_nv<T, N, V>();
        if (hipGetDevice(&dev) != hipSuccess ||
            hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || occ <= 0 ||
            cus <= 0)
            return 256;
        return cus * occ;
    }();
    return blocks;
}

template <typename T, int N, int V>
static hipError_t launch_unfold_nv(hipStream_t st, const EvDesc& ev0, const EvDesc* evs,
                                   const int4* units, int n_units, int spw, const XBin<T>* X,
                                   const MBin<T>* M, T* efield, const C2<T>* tw,
                                   unsigned int* counter, int persistent_blocks, const int* xcd_off,
                                   int xcd_max_list)
{
    if constexpr (!variant_built(N, V, (int)sizeof(T))) {
        return hipErrorInvalidValue;
    } else {
        using S = UShape<T, N, V>;
        if (n_units <= 0) return hipSuccess;
        int grid;
        if (counter != nullptr) {
            hipLaunchKernelGGL(k_zero_u32, dim3(1), dim3(64), 0, st, counter, 8);
            grid = std::min(n_units, persistent_blocks);
        } else {
            // no more blocks than the device holds at once: each loops over
            // its share of the units, so the per-block set-up (twiddles, the
            // LDS table) is paid once per block and the next unit's start
            // overlaps the previous unit's stores
            const int cap = resident_blocks<T, N, V>();
            grid = xcd_off != nullptr ? 8 * std::max(1, std::min(xcd_max_list, cap / 8)) : std::min(n_units, cap);
        }
        hipLaunchKernelGGL((k_unfold<T, N, S::E, S::RMAX, S::TWMODE, S::WAVE, S::PAIR, S::PP>), dim3(grid), dim3(S::BLOCK), S::LDS, st,
                           ev0, evs, units, n_units, spw, X, M, efield, tw, counter, xcd_off);
        return hipGetLastError();
    }
}

template <typename T, int N>
static hipError_t launch_unfold_n(int v, hipStream_t st, const EvDesc& ev0, const EvDesc* evs,
                                  const int4* units, int n_units, int spw, const XBin<T>* X,
                                  const MBin<T>* M, T* efield, const C2<T>* tw,
                                  unsigned int* counter, int persistent_blocks, const int* xcd_off,
                                  int xcd_max_list)
{
    switch (v) {
#define V_(VV) \
    case VV: return launch_unfold_nv<T, N, VV>(st, ev0, evs, units, n_units, spw, X, M, efield, tw, counter, persistent_blocks, xcd_off, xcd_max_list);
        V_(0) V_(1) V_(2) V_(3) V_(4) V_(5) V_(6) V_(7) V_(8) V_(9) V_(10) V_(11) V_(12) V_(13) V_(14) V_(15)
        V_(16) V_(17)
#undef V_
    }
    return hipErrorInvalidValue;
}

template <typename T, int N, int V>
static int occupancy_nv()
{
    if constexpr (!variant_built(N, V, (int)sizeof(T))) {
        return 0;
    } else {
        using S = UShape<T, N, V>;
        int occ = 0;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, k_unfold<T, N, S::E, S::RMAX, S::TWMODE, S::WAVE, S::PAIR, S::PP>, S::BLOCK,
                                                         S::LDS) != hipSuccess)
            return 0;
        return occ;
    }
}

template <typename Tin, typename T>
static hipError_t launch_spectrum(int n, hipStream_t st, const Tin* volt, const EvDesc& ev0,
                                  const EvDesc* evs, const int2* units, int n_units, int max_nb,
                                  XBin<T>* X, const C2<T>* tw)
{
    switch (n) {
#define X_(NN) \
    case NN: return launch_spectrum_n<Tin, T, NN>(st, volt, ev0, evs, units, n_units, max_nb, X, tw);
        AU_FOR_EACH_N(X_)
#undef X_
    }
    return hipErrorInvalidValue;
}

template <typename T>
static hipError_t launch_unfold(int n, int v, hipStream_t st, const EvDesc& ev0, const EvDesc* evs,
                                const int4* units, int n_units, int spw, const XBin<T>* X,
                                const MBin<T>* M, T* efield, const C2<T>* tw, unsigned int* counter,
                                int persistent_blocks, const int* xcd_off = nullptr, int xcd_max_list = 0)
{
    switch (n) {
#define X_(NN)                                                                                  \
    case NN:                                                                                    \
        return launch_unfold_n<T, NN>(v, st, ev0, evs, units, n_units, spw, X, M, efield, tw,   \
                                      counter, persistent_blocks, xcd_off, xcd_max_list);
        AU_FOR_EACH_N(X_)
#undef X_
    }
    return hipErrorInvalidValue;
}

template <typename T>
static int persistent_blocks_for(int n, int v, int device)
{
    int cus = 256;
    (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device);
    int per_cu = 0;
    switch (n) {
#define X_(NN)                                                                                  \
    case NN:                                                                                    \
        switch (v) {                                                                            \
            case 0: per_cu = occupancy_nv<T, NN, 0>(); break;                                   \
            case 1: per_cu = occupancy_nv<T, NN, 1>(); break;                                   \
            case 2: per_cu = occupancy_nv<T, NN, 2>(); break;                                   \
            case 3: per_cu = occupancy_nv<T, NN, 3>(); break;                                   \
            case 4: per_cu = occupancy_nv<T, NN, 4>(); break;                                   \
            case 5: per_cu = occupancy_nv<T, NN, 5>(); break;                                   \
            case 6: per_cu = occupancy_nv<T, NN, 6>(); break;                                   \
            case 7: per_cu = occupancy_nv<T, NN, 7>(); break;                                   \
            case 8: per_cu = occupancy_nv<T, NN, 8>(); break;                                   \
            case 9: per_cu = occupancy_nv<T, NN, 9>(); break;                                   \
            case 10: per_cu = occupancy_nv<T, NN, 10>(); break;                                 \
            case 11: per_cu = occupancy_nv<T, NN, 11>(); break;                                 \
            case 12: per_cu = occupancy_nv<T, NN, 12>(); break;                                 \
            case 13: per_cu = occupancy_nv<T, NN, 13>(); break;                                 \
            case 14: per_cu = occupancy_nv<T, NN, 14>(); break;                                 \
            case 15: per_cu = occupancy_nv<T, NN, 15>(); break;                                 \
            case 16: per_cu = occupancy_nv<T, NN, 16>(); break;                                 \
            case 17: per_cu = occupancy_nv<T, NN, 17>(); break;                                 \
        }                                                                                       \
        break;
        AU_FOR_EACH_N(X_)
#undef X_
    }
    return cus * std::max(per_cu, 1);
}

// ---------------------------------------------------------------------------
// twiddle tables, one pair (float, double) per device
// ---------------------------------------------------------------------------

static std::mutex g_mu;
constexpr int kMaxDev = 64;
static C2<float>* g_tw32[kMaxDev];
static C2<double>* g_tw64[kMaxDev];

// exp(+2 pi i q / n) in long double, reduced to the first octant so that
// quarter turns are exact and the libm argument stays small.
static void unit_root(int q, int n, long double& c, long double& s)
{
    q = ((q % n) + n) % n;
    const int quarter = n / 4;
    const int quad = q / quarter, r = q % quarter;
    const long double two_pi = 6.283185307179586476925286766559005768L;
    long double cr, sr;
    if (2 * r <= quarter) {
        const long double a = two_pi * (long double)r / (long double)n;
        cr = cosl(a);
        sr = sinl(a);
    } else {
        const long double a = two_pi * (long double)(quarter - r) / (long double)n;
        cr = sinl(a);
        sr = cosl(a);
    }
    switch (quad) {
        case 0: c = cr; s = sr; break;
        case 1: c = -sr; s = cr; break;
        case 2: c = -cr; s = -sr; break;
        default: c = sr; s = -cr; break;
    }
}

static au_status ensure_twiddles(int dev)
{
    if (dev < 0 || dev >= kMaxDev) return fail(AU_EDEVICE, "device index out of range");
    std::lock_guard<std::mutex> lk(g_mu);
    if (g_tw32[dev] != nullptr) return AU_OK;
    // kTwN roots exp(-2 pi i q / kTwN), then the (tangent, cosine) table of
    // the fused multiply-add butterflies (see lf_tab)
    constexpr int n_tw = kTwN + 4 * kLfQ;
    std::vector<C2<float>> h32(n_tw);
    std::vector<C2<double>> h64(n_tw);
    for (int q = 0; q < kTwN; ++q) {
        long double c, s;
        unit_root(q, kTwN, c, s);
        h64[q] = C2<double>{(double)c, (double)-s};
        h32[q] = C2<float>{(float)c, (float)-s};
    }
    for (int q = 0; q < kLfQ; ++q) {
        const int angle[4] = {q, 2 * q, 4 * q, q + kTwN / 8};  // a, 2a, 4a, a + pi/4 in units of 2 pi / kTwN
        for (int e = 0; e < 4; ++e) {
            long double c, s;
            unit_root(angle[e], kTwN, c, s);
            // +-90 deg: a tiny cosine keeps the tangent finite; its size is far
            // below each precision's rounding (2^-40 against 2^-24 for float,
            // 2^-90 against 2^-53 for double) and its tangent far below the range
            const long double c32 = c == 0.0L ? 0x1p-40L : c, c64 = c == 0.0L ? 0x1p-90L : c;
            h64[kTwN + 4 * q + e] = C2<double>{(double)(s / c64), (double)c64};
            h32[kTwN + 4 * q + e] = C2<float>{(float)(s / c32), (float)c32};
        }
    }
    void *p32 = nullptr, *p64 = nullptr;
    HIP_TRY(hipMalloc(&p32, sizeof(C2<float>) * n_tw));
    HIP_TRY(hipMalloc(&p64, sizeof(C2<double>) * n_tw));
    HIP_TRY(hipMemcpy(p32, h32.data(), sizeof(C2<float>) * n_tw, hipMemcpyHostToDevice));
    HIP_TRY(hipMemcpy(p64, h64.data(), sizeof(C2<double>) * n_tw, hipMemcpyHostToDevice));
    g_tw32[dev] = (C2<float>*)p32;
    g_tw64[dev] = (C2<double>*)p64;
    return AU_OK;
}

template <typename T>
static const C2<T>* twiddles(int dev);
template <>
const C2<float>* twiddles<float>(int dev) { return g_tw32[dev]; }
template <>
const C2<double>* twiddles<double>(int dev) { return g_tw64[dev]; }

// ---------------------------------------------------------------------------
// pattern table
// ---------------------------------------------------------------------------

static bool finite_pos(double x) { return std::isfinite(x) && x > 0.0; }

extern "C" au_status au_load_pattern_table(const au_grid* grid, int32_t dtype, const void* h_vel,
                                           au_table** out)
{
    if (!grid || !h_vel || !out) return fail(AU_EINVAL, "null argument");
    if (dtype != AU_F32 && dtype != AU_F64) return fail(AU_EINVAL, "table dtype must be AU_F32 or AU_F64");
    const au_grid& G = *grid;
    if (G.n_freq < 2 || G.n_zen < 2 || G.n_az < 2)
        return fail(AU_EINVAL, "grid needs at least 2 nodes per axis");
    if (G.df_hz <= 0 || G.f0_hz < 0 || !finite_pos(G.dzen_deg) || !finite_pos(G.daz_deg) ||
        !std::isfinite(G.zen0_deg) || !std::isfinite(G.az0_deg))
        return fail(AU_EINVAL, "grid steps must be positive and finite");
    const int nf = G.n_freq, nz = G.n_zen, na = G.n_az;
    const size_t esz = dtype == AU_F64 ? 16 : 8;
    const size_t col = (size_t)nz * na;
    int na_eff = na;
    if (std::fabs(na * G.daz_deg - 360.0) <= 1e-9 * 360.0) {
        na_eff = na;
    } else if (std::fabs((na - 1) * G.daz_deg - 360.0) <= 1e-9 * 360.0) {
        // duplicated 360-degree column: accepted only if equal to column 0
        const unsigned char* b = (const unsigned char*)h_vel;
        for (size_t cpf = 0; cpf < (size_t)4 * nf * nz; ++cpf) {
            const unsigned char* row = b + cpf * na * esz;
            if (std::memcmp(row, row + (size_t)(na - 1) * esz, esz) != 0)
                return fail(AU_EINVAL, "last azimuth column duplicates 360 deg but differs from column 0");
        }
        na_eff = na - 1;
    } else {
        return fail(AU_EINVAL, "azimuth grid must cover 360 degrees periodically (n_az * daz == 360)");
    }
    if (na_eff < 2) return fail(AU_EINVAL, "azimuth grid too small");
    (void)col;
    const size_t n_nodes = (size_t)nf * nz * na_eff;
    std::vector<unsigned char> host(n_nodes * 4 * esz);
    const unsigned char* src = (const unsigned char*)h_vel;
    for (int cp = 0; cp < 4; ++cp)
        for (int f = 0; f < nf; ++f)
            for (int z = 0; z < nz; ++z)
                for (int a = 0; a < na_eff; ++a) {
                    const size_t si = (((size_t)cp * nf + f) * nz + z) * na + a;
                    const size_t di = (((size_t)f * nz + z) * na_eff + a) * 4 + cp;
                    std::memcpy(&host[di * esz], src + si * esz, esz);
                }
    for (size_t i = 0; i < host.size() / (esz / 2); ++i) {
        const double v = esz == 16 ? ((const double*)host.data())[i] : ((const float*)host.data())[i];
        if (!std::isfinite(v)) return fail(AU_EINVAL, "pattern table holds a non-finite value");
    }
    int dev = 0;
    HIP_TRY(hipGetDevice(&dev));
    au_status st = ensure_twiddles(dev);
    if (st != AU_OK) return st;
    au_table* t = new au_table();
    t->device = dev;
    t->dtype = dtype;
    t->g = GridDev{nf, nz, na_eff, 0, G.f0_hz, G.df_hz, G.zen0_deg, G.dzen_deg, G.az0_deg, G.daz_deg};
    t->bytes = host.size();
    hipError_t e = hipMalloc(&t->d_nodes, t->bytes);
    if (e != hipSuccess) {
        delete t;
        return fail(AU_ENOMEM, std::string("hipMalloc(table): ") + hipGetErrorString(e));
    }
    e = hipMemcpy(t->d_nodes, host.data(), t->bytes, hipMemcpyHostToDevice);
    if (e != hipSuccess) {
        (void)hipFree(t->d_nodes);
        delete t;
        return fail(AU_EDEVICE, std::string("hipMemcpy(table): ") + hipGetErrorString(e));
    }
    *out = t;
    return AU_OK;
}

extern "C" au_status au_free_pattern_table(au_table* t)
{
    if (!t) return AU_OK;
    if (t->d_nodes) HIP_TRY(hipFree(t->d_nodes));
    delete t;
    return AU_OK;
}

// ---------------------------------------------------------------------------
// event validation and the band
// ---------------------------------------------------------------------------

static au_status band_of(int64_t n, int64_t fs, int64_t lo, int64_t hi, int* k_lo, int* nb)
{
    const int64_t klo = (lo * n + fs - 1) / fs;  // smallest k with k fs >= lo n
    const int64_t khi = (hi * n) / fs;           // largest k with k fs <= hi n
    *k_lo = (int)klo;
    *nb = khi >= klo ? (int)(khi - klo + 1) : 0;
    return AU_OK;
}

au_status au::check_common(const au_table* tb, int64_t fs, int64_t lo, int64_t hi, int prec,
                              int tin, double fb, double sg)
{
    if (!tb) return fail(AU_EINVAL, "null table");
    if (fs <= 0 || fs > (int64_t)1000000000000000LL) return fail(AU_EINVAL, "fs_hz out of range");
    if (lo < 0 || hi < lo || 2 * hi >= fs) return fail(AU_EINVAL, "band must satisfy 0 <= lo <= hi < fs/2");
    if (prec != AU_PREC_FP32 && prec != AU_PREC_FP64) return fail(AU_EINVAL, "prec must be AU_PREC_FP32 or AU_PREC_FP64");
    if (tin != AU_F32 && tin != AU_F64) return fail(AU_EINVAL, "trace_dtype must be AU_F32 or AU_F64");
    if (prec == AU_PREC_FP64 && tb->dtype != AU_F64)
        return fail(AU_EINVAL, "FP64 precision needs a complex128 pattern table");
    if (!(fb >= 0.0) || !std::isfinite(fb) || !(sg >= 0.0) || !std::isfinite(sg))
        return fail(AU_EINVAL, "fallback_rel and singular_rel must be finite and >= 0");
    return AU_OK;
}

au_status au::check_n(const au_table* tb, int s, int n, int64_t fs, int64_t lo, int64_t hi,
                         EvParams* p)
{
    if (n < 16 || n > 4096 || (n & (n - 1)) != 0)
        return fail(AU_EINVAL, "n_samples must be a power of two in [16, 4096]");
    if (s < 1) return fail(AU_EINVAL, "n_stations must be >= 1");
    int k_lo, nb;
    band_of(n, fs, lo, hi, &k_lo, &nb);
    if (nb > 0) {
        const GridDev& g = tb->g;
        // The device splits the node position (k fs - f0 N) / (N df) of every
        // in-band bin exactly through a double estimate, which needs the
        // numerator and denominator below 2^53 (exact in double); checked in
        // 128-bit arithmetic so that no product here overflows either.
        const __int128 lim = (__int128)1 << 53;
        const __int128 den = (__int128)n * g.df_hz;
        const __int128 num_lo = (__int128)k_lo * fs - (__int128)g.f0_hz * n;
        const __int128 num_hi = (__int128)(k_lo + nb - 1) * fs - (__int128)g.f0_hz * n;
        if (den >= lim || num_lo <= -lim || num_hi >= lim || num_lo >= lim || num_hi <= -lim)
            return fail(AU_EINVAL, "frequency arithmetic out of range: |k fs - f0 N| and N df must stay below 2^53");
        if (num_lo < 0 || num_hi > (__int128)(g.n_freq - 1) * den)
            return fail(AU_EINVAL, "band lies outside the pattern table's frequency range");
    }
    p->S = s;
    p->N = n;
    p->k_lo = k_lo;
    p->nb = nb;
    return AU_OK;
}

static au_status check_event(const au_table* tb, const au_event* ev, EvParams* p)
{
    if (!ev) return fail(AU_EINVAL, "null event");
    au_status st = check_common(tb, ev->fs_hz, ev->band_lo_hz, ev->band_hi_hz, ev->prec,
                                ev->trace_dtype, ev->fallback_rel, ev->singular_rel);
    if (st != AU_OK) return st;
    return check_n(tb, ev->n_stations, ev->n_samples, ev->fs_hz, ev->band_lo_hz, ev->band_hi_hz, p);
}

bool au::dirs_finite(const double* h, int64_t n)
{
    for (int64_t i = 0; i < 2 * n; ++i)
        if (!std::isfinite(h[i]) || std::fabs(h[i]) > 1e6) return false;
    return true;
}

struct WsLayout {
    size_t x, m, dirs, total;
};

static WsLayout ws_layout(const EvParams& p, int prec, int n_dir)
{
    const size_t xb = prec == AU_PREC_FP64 ? sizeof(XBin<double>) : sizeof(XBin<float>);
    const size_t mb = prec == AU_PREC_FP64 ? sizeof(MBin<double>) : sizeof(MBin<float>);
    WsLayout w;
    w.x = align256((size_t)p.S * p.nb * xb + 1);
    w.m = align256((size_t)n_dir * p.nb * mb + 1);
    w.dirs = align256((size_t)n_dir * 2 * sizeof(double) + 1);
    w.total = w.x + w.m + w.dirs;
    return w;
}

extern "C" au_status au_band_bins(const au_event* ev, int32_t* k_lo, int32_t* n_band)
{
    if (!ev || !k_lo || !n_band) return fail(AU_EINVAL, "null argument");
    if (ev->fs_hz <= 0 || ev->band_lo_hz < 0 || ev->band_hi_hz < ev->band_lo_hz)
        return fail(AU_EINVAL, "bad band");
    int a, b;
    band_of(ev->n_samples, ev->fs_hz, ev->band_lo_hz, ev->band_hi_hz, &a, &b);
    *k_lo = a;
    *n_band = b;
    return AU_OK;
}

extern "C" au_status au_workspace_bytes(const au_table* tb, const au_event* ev, int32_t n_dir,
                                        uint64_t* bytes)
{
    if (!bytes) return fail(AU_EINVAL, "null argument");
    EvParams p;
    au_status st = check_event(tb, ev, &p);
    if (st != AU_OK) return st;
    if (n_dir < 1) return fail(AU_EINVAL, "n_dir must be >= 1");
    *bytes = ws_layout(p, ev->prec, n_dir).total;
    return AU_OK;
}

// ---------------------------------------------------------------------------
// single-event path: spectra, coefficients, unfold as three launches
// ---------------------------------------------------------------------------

template <typename Tt, typename T>
static void launch_coef(hipStream_t st, const au_table* tb, const EvDesc& ev0, const EvDesc* evs,
                        const int2* units, int n_units, const double* dirs, double zen, double az,
                        int64_t fs, double fb, double sg, MBin<T>* M, unsigned long long* counts,
                        const int* skip = nullptr, int skip_stride = 0)
{
    hipLaunchKernelGGL((k_coef<Tt, T, false>), dim3(n_units), dim3(kBlock), 0, st,
                       (const C2<Tt>*)tb->d_nodes, tb->g, ev0, evs, units, dirs, zen, az, fs, fb, sg,
                       M, counts, 0.0, skip, skip_stride);
}

// Stations per work unit of a direction scan (one event, n_dir directions;
// units (direction, station range) spread over a grid of up to `blocks`
// that each loop over their share): from 16, halved while there are fewer
// units than blocks (a small scan -- one event of ten stations and one
// direction -- then runs a station per workgroup instead of all ten in one),
// doubled while every block still gets at least four units.  A unit's first
// station waits for the stores of the block's previous unit (its bins are
// loaded after them), so fewer, longer units leave fewer such waits: the
// FP64 scan of 124 stations x 2048 directions runs 3 % faster with one unit
// per direction than with 16-station units.
static int scan_stations_per_unit(int S, int64_t n_dir, int blocks)
{
    const int64_t b = std::max(blocks, 1);
    int spw = kStationsPerUnit;
    while (spw > 1 && n_dir * (int64_t)((S + spw - 1) / spw) < b) spw /= 2;
    while (spw < S && n_dir * (int64_t)((S + 2 * spw - 1) / (2 * spw)) >= 4 * b) spw *= 2;
    return spw;
}

// Workgroups of unfold variant v the device holds at once, cached per
// (precision, trace length, variant).
static int scan_blocks(int prec, int n, int variant, int device)
{
    static std::atomic<int> cache[2][13][kNumVariants];
    const int pi = prec == AU_PREC_FP64 ? 1 : 0, li = ilog2(n);
    if (li < 0 || li > 12 || variant < 0 || variant >= kNumVariants) return 256;
    int b = cache[pi][li][variant].load(std::memory_order_relaxed);
    if (b == 0) {
        b = au::persistent_blocks(prec, n, variant, device);
        cache[pi][li][variant].store(b, std::memory_order_relaxed);
    }
    return b;
}

// The frequency node below bin k (freq_cell's quotient, exact on the host).
static int64_t host_freq_node(const GridDev& g, int64_t k, int n, int64_t fs)
{
    const int64_t q = (k * fs - g.f0_hz * (int64_t)n) / ((int64_t)n * g.df_hz);
    return std::min<int64_t>(q, g.n_freq - 2);
}

// The single-direction call in one launch (k_event_fused), where it applies:
// 2048 or 4096 samples, traces and table in the compute precision, a band of
// at most 2 N/8 bins spanning at most kMaxSliceNodes frequency nodes.
// Returns false (nothing enqueued) where it does not apply.
template <typename T>
static bool event_fused(const au_table* tb, const au_event* ev, const EvParams& p, const void* d_volt, double zen,
                        double az, void* d_efield, hipStream_t st, uint64_t* d_counts, au_status* rc)
{
    constexpr int tcode = sizeof(T) == 8 ? AU_F64 : AU_F32;
    if ((p.N != 2048 && p.N != 4096) || ev->trace_dtype != tcode || tb->dtype != tcode || p.S < 1)
        return false;
    if (p.nb > 2 * (p.N / 8)) return false;
    if (p.nb > 0) {
        const int64_t f_lo = host_freq_node(tb->g, p.k_lo, p.N, ev->fs_hz);
        const int64_t f_hi = host_freq_node(tb->g, (int64_t)p.k_lo + p.nb - 1, p.N, ev->fs_hz);
        if (f_lo < 0 || f_hi - f_lo + 2 > kMaxSliceNodes) return false;
    }
    const C2<T>* tw = twiddles<T>(tb->device);
    if (tw == nullptr) {
        *rc = fail(AU_EDEVICE, "twiddle tables missing on this device");
        return true;
    }
    EvDesc ev0{};
    ev0.S = p.S;
    ev0.N = p.N;
    ev0.D = 1;
    ev0.k_lo = p.k_lo;
    ev0.nb = p.nb;
#define EVF_(NN)                                                                                                 \
    hipLaunchKernelGGL((k_event_fused<T, T, NN>), dim3(p.S), dim3(NN / 8),                                       \
                       (2 * lds_elems<NN>() + ltw_count<NN, 8, 8, TW_LF>()) * sizeof(C2<T>), st,                  \
                       (const C2<T>*)tb->d_nodes, tb->g, ev0, (const T*)d_volt, zen, az, ev->fs_hz,               \
                       ev->fallback_rel, ev->singular_rel, (T*)d_efield, tw, (unsigned long long*)d_counts)
    if (p.N == 2048)
        EVF_(2048);
    else
        EVF_(4096);
#undef EVF_
    const hipError_t e = hipGetLastError();
    *rc = e == hipSuccess ? AU_OK : fail(AU_EDEVICE, std::string("k_event_fused: ") + hipGetErrorString(e));
    return true;
}

// Directions come from h_dirs (copied into the workspace's direction slot
// first), from d_dirs (already in that slot, device memory), or, with both
// null, the one direction (zen, az).
template <typename T>
static au_status run_event(const au_table* tb, const au_event* ev, const EvParams& p,
                           const void* d_volt, int n_dir, const double* h_dirs, double zen,
                           double az, void* d_efield, void* d_work, hipStream_t st,
                           uint64_t* d_counts, int variant = -1, bool d_dirs = false)
{
    if (variant < 0) variant = unfold_variant(ev->prec, p.N);
    const WsLayout w = ws_layout(p, ev->prec, n_dir);
    unsigned char* base = (unsigned char*)d_work;
    XBin<T>* X = (XBin<T>*)base;
    MBin<T>* M = (MBin<T>*)(base + w.x);
    double* dirs = (double*)(base + w.x + w.m);
    if (h_dirs != nullptr)
        HIP_TRY(hipMemcpyAsync(dirs, h_dirs, sizeof(double) * 2 * n_dir, hipMemcpyHostToDevice, st));
    if (d_dirs) h_dirs = dirs;  // only its non-nullness is used below
    EvDesc ev0{};
    ev0.S = p.S;
    ev0.N = p.N;
    ev0.D = n_dir;
    ev0.k_lo = p.k_lo;
    ev0.nb = p.nb;
    const C2<T>* tw = twiddles<T>(tb->device);
    if (tw == nullptr) return fail(AU_EDEVICE, "twiddle tables missing on this device");
    hipError_t e;
    if (ev->trace_dtype == AU_F64)
        e = launch_spectrum<double, T>(p.N, st, (const double*)d_volt, ev0, nullptr, nullptr, p.S, ev0.nb, X, tw);
    else
        e = launch_spectrum<float, T>(p.N, st, (const float*)d_volt, ev0, nullptr, nullptr, p.S, ev0.nb, X, tw);
    if (e != hipSuccess) return fail(AU_EDEVICE, std::string("k_spectrum: ") + hipGetErrorString(e));
    unsigned long long* cnt = (unsigned long long*)d_counts;
    if (tb->dtype == AU_F64)
        launch_coef<double, T>(st, tb, ev0, nullptr, nullptr, n_dir, h_dirs ? dirs : nullptr, zen,
                               az, ev->fs_hz, ev->fallback_rel, ev->singular_rel, M,
                               cnt);
    else
        launch_coef<float, T>(st, tb, ev0, nullptr, nullptr, n_dir, h_dirs ? dirs : nullptr, zen, az,
                              ev->fs_hz, ev->fallback_rel, ev->singular_rel, M, cnt);
    e = hipGetLastError();
    if (e != hipSuccess) return fail(AU_EDEVICE, std::string("k_coef: ") + hipGetErrorString(e));
    const int spw = scan_stations_per_unit(p.S, n_dir, scan_blocks(ev->prec, p.N, variant, tb->device));
    const int chunks = (p.S + spw - 1) / spw;
    const int64_t n_units = (int64_t)n_dir * chunks;
    if (n_units > (int64_t)0x7fffffff) return fail(AU_EINVAL, "too many work units");
    e = launch_unfold<T>(p.N, variant, st, ev0, nullptr, nullptr, (int)n_units, spw, X, M, (T*)d_efield, tw,
                         nullptr, 0);
    if (e != hipSuccess) return fail(AU_EDEVICE, std::string("k_unfold: ") + hipGetErrorString(e));
    return AU_OK;
}

static au_status unfold_common(const au_table* tb, const au_event* ev, const void* d_volt,
                               int32_t n_dir, const double* h_dirs, double zen, double az,
                               void* d_efield, void* d_work, uint64_t work_bytes, void* stream,
                               uint64_t* d_counts)
{
    EvParams p;
    au_status s = check_event(tb, ev, &p);
    if (s != AU_OK) return s;
    if (!d_volt || !d_efield) return fail(AU_EINVAL, "null trace or output pointer");
    if (n_dir < 1) return fail(AU_EINVAL, "n_dir must be >= 1");
    if (h_dirs != nullptr && !dirs_finite(h_dirs, n_dir))
        return fail(AU_EINVAL, "directions must be finite");
    if (h_dirs == nullptr && (!std::isfinite(zen) || !std::isfinite(az) || std::fabs(az) > 1e6))
        return fail(AU_EINVAL, "direction must be finite");
    int dev = 0;
    HIP_TRY(hipGetDevice(&dev));
    if (dev != tb->device) return fail(AU_EINVAL, "table lives on another device");
    const WsLayout w = ws_layout(p, ev->prec, n_dir);
    hipStream_t st = (hipStream_t)stream;
    void* work = d_work;
    bool pooled = false;
    if (work != nullptr && work_bytes < w.total) return fail(AU_ENOMEM, "workspace smaller than au_workspace_bytes");
    // one direction given by value: one launch (k_event_fused) where it applies
    if (h_dirs == nullptr && n_dir == 1) {
        au_status rc = AU_OK;
        const bool done = ev->prec == AU_PREC_FP64
                              ? event_fused<double>(tb, ev, p, d_volt, zen, az, d_efield, st, d_counts, &rc)
                              : event_fused<float>(tb, ev, p, d_volt, zen, az, d_efield, st, d_counts, &rc);
        if (done) return rc;
    }
    if (work == nullptr) {
        hipError_t e = hipMallocAsync(&work, w.total, st);
        if (e != hipSuccess) return fail(AU_ENOMEM, std::string("hipMallocAsync: ") + hipGetErrorString(e));
        pooled = true;
    } else if (work_bytes < w.total) {
        return fail(AU_ENOMEM, "workspace smaller than au_workspace_bytes");
    }
    if (ev->prec == AU_PREC_FP64)
        s = run_event<double>(tb, ev, p, d_volt, n_dir, h_dirs, zen, az, d_efield, work, st, d_counts);
    else
        s = run_event<float>(tb, ev, p, d_volt, n_dir, h_dirs, zen, az, d_efield, work, st, d_counts);
    if (pooled) {
        hipError_t e = hipFreeAsync(work, st);
        if (s == AU_OK && e != hipSuccess)
            return fail(AU_EDEVICE, std::string("hipFreeAsync: ") + hipGetErrorString(e));
    }
    return s;
}

void au::workspace_layout(const EvParams& p, int prec, int n_dir, size_t* x_bytes, size_t* m_bytes,
                          size_t* dir_bytes)
{
    const WsLayout w = ws_layout(p, prec, n_dir);
    *x_bytes = w.x;
    *m_bytes = w.m;
    *dir_bytes = w.dirs;
}

au_status au::enqueue_event(const au_table* tb, const au_event* ev, const EvParams& p, const void* d_volt,
                            int n_dir, void* d_efield, void* d_work, hipStream_t st, uint64_t* d_counts)
{
    if (ev->prec == AU_PREC_FP64)
        return run_event<double>(tb, ev, p, d_volt, n_dir, nullptr, 0.0, 0.0, d_efield, d_work, st, d_counts, -1,
                                 true);
    return run_event<float>(tb, ev, p, d_volt, n_dir, nullptr, 0.0, 0.0, d_efield, d_work, st, d_counts, -1, true);
}

extern "C" au_status au_unfold_event(const au_table* tb, const au_event* ev, const void* d_volt,
                                     double zen_deg, double az_deg, void* d_efield, void* d_work,
                                     uint64_t work_bytes, void* stream, uint64_t* d_counts)
{
    return unfold_common(tb, ev, d_volt, 1, nullptr, zen_deg, az_deg, d_efield, d_work, work_bytes,
                         stream, d_counts);
}

extern "C" au_status au_unfold_direction_scan(const au_table* tb, const au_event* ev,
                                              const void* d_volt, int32_t n_dir,
                                              const double* h_dirs, void* d_efield, void* d_work,
                                              uint64_t work_bytes, void* stream, uint64_t* d_counts)
{
    if (!h_dirs) return fail(AU_EINVAL, "null direction list");
    return unfold_common(tb, ev, d_volt, n_dir, h_dirs, 0.0, 0.0, d_efield, d_work, work_bytes,
                         stream, d_counts);
}

// ---------------------------------------------------------------------------
// direction scan without allocation: the spectra and coefficients live in a
// file-scope device array
// ---------------------------------------------------------------------------

// Work space of au_unfold_direction_scan_noalloc: the event's in-band spectra
// and one chunk of directions' coefficients.  Each device holds its own copy
// from module load until the process ends.  In host code the array's name
// is a host-side stand-in; its device address comes from
// hipGetSymbolAddress, taken once per device (scratch_address).
constexpr size_t kScratchBytes = (size_t)32 << 20;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];
static std::mutex g_scratch_mu;
static unsigned char* g_scratch[kMaxDev];

static au_status scratch_address(int dev, unsigned char** out)
{
    if (dev < 0 || dev >= kMaxDev) return fail(AU_EDEVICE, "device index out of range");
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (g_scratch[dev] == nullptr) {
        void* ptr = nullptr;
        const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));  // the current device's copy
        if (e != hipSuccess || ptr == nullptr)
            return fail(AU_EDEVICE, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
        g_scratch[dev] = (unsigned char*)ptr;
    }
    *out = g_scratch[dev];
    return AU_OK;
}

// Spectra once, then the directions in chunks whose coefficients fit the
// rest of the scratch array: per chunk one coefficient and one unfold launch
// (the same kernels and per-unit arithmetic as the workspace path).
template <typename T>
static au_status run_scan_scratch(const au_table* tb, const au_event* ev, const EvParams& p, const void* d_volt,
                                  int n_dir, const double* d_dirs, void* d_efield, unsigned char* base,
                                  size_t x_bytes, int chunk, hipStream_t st, uint64_t* d_counts)
{
    const int variant = unfold_variant(ev->prec, p.N);
    XBin<T>* X = (XBin<T>*)base;
    MBin<T>* M = (MBin<T>*)(base + x_bytes);
    EvDesc ev0{};
    ev0.S = p.S;
    ev0.N = p.N;
    ev0.k_lo = p.k_lo;
    ev0.nb = p.nb;
    const C2<T>* tw = twiddles<T>(tb->device);
    if (tw == nullptr) return fail(AU_EDEVICE, "twiddle tables missing on this device");
    hipError_t e;
    if (ev->trace_dtype == AU_F64)
        e = launch_spectrum<double, T>(p.N, st, (const double*)d_volt, ev0, nullptr, nullptr, p.S, ev0.nb, X, tw);
    else
        e = launch_spectrum<float, T>(p.N, st, (const float*)d_volt, ev0, nullptr, nullptr, p.S, ev0.nb, X, tw);
    if (e != hipSuccess) return fail(AU_EDEVICE, std::string("k_spectrum: ") + hipGetErrorString(e));
    unsigned long long* cnt = (unsigned long long*)d_counts;
    const int blocks = scan_blocks(ev->prec, p.N, variant, tb->device);
    for (int d0 = 0; d0 < n_dir; d0 += chunk) {
        const int nd = std::min(chunk, n_dir - d0);
        const int spw = scan_stations_per_unit(p.S, nd, blocks);
        const int chunks = (p.S + spw - 1) / spw;
        ev0.D = nd;
        if (tb->dtype == AU_F64)
            launch_coef<double, T>(st, tb, ev0, nullptr, nullptr, nd, d_dirs + 2 * (size_t)d0, 0.0, 0.0, ev->fs_hz,
                                   ev->fallback_rel, ev->singular_rel, M, cnt);
        else
            launch_coef<float, T>(st, tb, ev0, nullptr, nullptr, nd, d_dirs + 2 * (size_t)d0, 0.0, 0.0, ev->fs_hz,
                                  ev->fallback_rel, ev->singular_rel, M, cnt);
        e = hipGetLastError();
        if (e != hipSuccess) return fail(AU_EDEVICE, std::string("k_coef: ") + hipGetErrorString(e));
        const int64_t n_units = (int64_t)nd * chunks;
        if (n_units > (int64_t)0x7fffffff) return fail(AU_EINVAL, "too many work units");
        T* out = (T*)d_efield + (size_t)d0 * p.S * 2 * p.N;
        e = launch_unfold<T>(p.N, variant, st, ev0, nullptr, nullptr, (int)n_units, spw, X, M, out, tw, nullptr, 0);
        if (e != hipSuccess) return fail(AU_EDEVICE, std::string("k_unfold: ") + hipGetErrorString(e));
    }
    return AU_OK;
}

extern "C" au_status au_unfold_direction_scan_noalloc(const au_table* tb, const au_event* ev, const void* d_volt,
                                                      int32_t n_dir, const double* d_dirs, void* d_efield,
                                                      void* stream, uint64_t* d_counts)
{
    EvParams p;
    au_status s = check_event(tb, ev, &p);
    if (s != AU_OK) return s;
    if (!d_volt || !d_efield || !d_dirs) return fail(AU_EINVAL, "null trace, direction or output pointer");
    if (n_dir < 1) return fail(AU_EINVAL, "n_dir must be >= 1");
    int dev = 0;
    HIP_TRY(hipGetDevice(&dev));
    if (dev != tb->device) return fail(AU_EINVAL, "table lives on another device");
    const size_t xb = ev->prec == AU_PREC_FP64 ? sizeof(XBin<double>) : sizeof(XBin<float>);
    const size_t mb = ev->prec == AU_PREC_FP64 ? sizeof(MBin<double>) : sizeof(MBin<float>);
    const size_t x_bytes = align256((size_t)p.S * p.nb * xb);
    const size_t m_dir = (size_t)p.nb * mb;  // one direction's coefficients
    if (x_bytes + m_dir > kScratchBytes)
        return fail(AU_EINVAL, "event too large for the 32 MiB scratch: n_stations * n_band spectra (" +
                                   std::to_string(x_bytes) + " B) plus one direction's coefficients (" +
                                   std::to_string(m_dir) + " B) must fit");
    const size_t fit = m_dir ? (kScratchBytes - x_bytes) / m_dir : (size_t)n_dir;
    const int chunk = (int)std::min<size_t>(fit, (size_t)n_dir);
    unsigned char* base = nullptr;
    s = scratch_address(dev, &base);
    if (s != AU_OK) return s;
    hipStream_t st = (hipStream_t)stream;
    if (ev->prec == AU_PREC_FP64)
        return run_scan_scratch<double>(tb, ev, p, d_volt, n_dir, d_dirs, d_efield, base, x_bytes, chunk, st,
                                        d_counts);
    return run_scan_scratch<float>(tb, ev, p, d_volt, n_dir, d_dirs, d_efield, base, x_bytes, chunk, st, d_counts);
}

static au_status pattern_response(const au_table* tb, const au_event* ev, int32_t n_dir, const double* h_dirs,
                                  void* d_resp, void* stream, double wq)
{
    EvParams p;
    au_status s = check_event(tb, ev, &p);
    if (s != AU_OK) return s;
    if (!h_dirs || !d_resp || n_dir < 1) return fail(AU_EINVAL, "bad direction list or output");
    if (!dirs_finite(h_dirs, n_dir)) return fail(AU_EINVAL, "directions must be finite");
    if (p.nb == 0) return AU_OK;
    hipStream_t st = (hipStream_t)stream;
    double* dirs = nullptr;
    hipError_t e = hipMallocAsync((void**)&dirs, sizeof(double) * 2 * n_dir, st);
    if (e != hipSuccess) return fail(AU_ENOMEM, "hipMallocAsync(dirs)");
    HIP_TRY(hipMemcpyAsync(dirs, h_dirs, sizeof(double) * 2 * n_dir, hipMemcpyHostToDevice, st));
    EvDesc ev0{};
    ev0.S = p.S;
    ev0.N = p.N;
    ev0.D = n_dir;
    ev0.k_lo = p.k_lo;
    ev0.nb = p.nb;
    const bool f64 = ev->prec == AU_PREC_FP64;
#define RESP_(TT, T)                                                                        \
    hipLaunchKernelGGL((k_coef<TT, T, true>), dim3(n_dir), dim3(kBlock), 0, st,            \
                       (const C2<TT>*)tb->d_nodes, tb->g, ev0, nullptr, nullptr, dirs, 0.0, 0.0, \
                       ev->fs_hz, 0.0, 0.0, (MBin<T>*)d_resp, nullptr, wq, nullptr, 0)
    if (f64)
        RESP_(double, double);
    else if (tb->dtype == AU_F64)
        RESP_(double, float);
    else
        RESP_(float, float);
#undef RESP_
    e = hipGetLastError();
    if (e != hipSuccess) return fail(AU_EDEVICE, std::string("k_coef(resp): ") + hipGetErrorString(e));
    HIP_TRY(hipFreeAsync(dirs, st));
    return AU_OK;
}

extern "C" au_status au_pattern_response(const au_table* tb, const au_event* ev, int32_t n_dir,
                                         const double* h_dirs, void* d_resp, void* stream)
{
    return pattern_response(tb, ev, n_dir, h_dirs, d_resp, stream, 0.0);
}

extern "C" au_status au_pattern_response_quantized(const au_table* tb, const au_event* ev, int32_t n_dir,
                                                   const double* h_dirs, int32_t weight_bits, void* d_resp,
                                                   void* stream)
{
    if (weight_bits < 1 || weight_bits > 30) return fail(AU_EINVAL, "weight_bits must be in [1, 30]");
    return pattern_response(tb, ev, n_dir, h_dirs, d_resp, stream, std::ldexp(1.0, weight_bits));
}

// ---------------------------------------------------------------------------
// batched plans: many uneven events, one launch sequence per trace length
// ---------------------------------------------------------------------------

struct ClassPlan {
    int N = 0;
    uint64_t station_unfolds = 0;
    int n_sunits = 0, n_cunits = 0, n_uunits = 0;
    EvDesc* d_evs = nullptr;
    int2* d_sunits = nullptr;
    int2* d_cunits = nullptr;
    int4* d_uunits = nullptr;
    unsigned int* d_counter = nullptr;
    int persistent_blocks = 0;
    int variant = 0;
    int* d_xcd_off = nullptr;
    int xcd_max_list = 0;
    int max_nb = 0;  // largest band of the class's events (bins)
    bool fused = false;  // spectrum and unfold in k_unfold_fused (units: event, station range)
};

struct au_plan {
    const au_table* tb = nullptr;
    int device = 0;
    int prec = 0, tin = 0, flags = 0;
    int64_t fs = 0;
    double fb = 0, sg = 0;
    void* d_mem = nullptr;
    void* d_x = nullptr;
    void* d_m = nullptr;
    double* d_dirs = nullptr;
    std::vector<ClassPlan> classes;
    uint64_t station_unfolds = 0;
    hipStream_t cap_stream = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    const void* g_volt = nullptr;
    void* g_efield = nullptr;
    uint64_t* g_counts = nullptr;
    // stage timing (au_plan_timing): one event before the first launch and
    // one after every launch of a run; elapsed times summed per stage
    bool timing = false;
    std::vector<hipEvent_t> ev;
    std::vector<double> stage_ms;  // [class][spectrum, coef, unfold]
    uint64_t timed_runs = 0;
};

template <typename T>
static au_status enqueue_class_t(const au_table* tb, int tin, int64_t fs, double fb, double sg,
                                 const ClassLaunch& c, const void* volt, void* efield, void* Xv, void* Mv,
                                 const double* dirs, hipStream_t st, uint64_t* d_counts,
                                 hipEvent_t* stage_events)
{
    const C2<T>* tw = twiddles<T>(tb->device);
    if (tw == nullptr) return fail(AU_EDEVICE, "twiddle tables missing on this device");
    XBin<T>* X = (XBin<T>*)Xv;
    MBin<T>* M = (MBin<T>*)Mv;
    EvDesc ev0{};
    hipError_t e;
    if constexpr (sizeof(T) == 4) {
        if (c.fused) {
            // no spectrum stage: coefficients, then the fused kernel
            if (stage_events) HIP_TRY(hipEventRecord(stage_events[0], st));
            if (tb->dtype == AU_F64)
                launch_coef<double, T>(st, tb, ev0, c.d_evs, c.d_cunits, c.n_cunits, dirs, 0, 0, fs, fb, sg, M,
                                       (unsigned long long*)d_counts);
            else
                launch_coef<float, T>(st, tb, ev0, c.d_evs, c.d_cunits, c.n_cunits, dirs, 0, 0, fs, fb, sg, M,
                                      (unsigned long long*)d_counts);
            e = hipGetLastError();
            if (e != hipSuccess) return fail(AU_EDEVICE, std::string("k_coef: ") + hipGetErrorString(e));
            if (stage_events) HIP_TRY(hipEventRecord(stage_events[1], st));
            if (tin == AU_F64)
                e = launch_fused<double>(c.N, st, (const double*)volt, c.d_evs, c.d_uunits, c.n_uunits, M,
                                         (float*)efield, tw, c.d_counter, c.d_xcd_off);
            else
                e = launch_fused<float>(c.N, st, (const float*)volt, c.d_evs, c.d_uunits, c.n_uunits, M,
                                        (float*)efield, tw, c.d_counter, c.d_xcd_off);
            if (e != hipSuccess) return fail(AU_EDEVICE, std::string("k_unfold_fused: ") + hipGetErrorString(e));
            if (stage_events) HIP_TRY(hipEventRecord(stage_events[2], st));
            return AU_OK;
        }
    }
    if (tin == AU_F64)
        e = launch_spectrum<double, T>(c.N, st, (const double*)volt, ev0, c.d_evs, c.d_sunits, c.n_sunits, c.max_nb, X, tw);
    else
        e = launch_spectrum<float, T>(c.N, st, (const float*)volt, ev0, c.d_evs, c.d_sunits, c.n_sunits, c.max_nb, X, tw);
    if (e != hipSuccess) return fail(AU_EDEVICE, std::string("k_spectrum: ") + hipGetErrorString(e));
    if (stage_events) HIP_TRY(hipEventRecord(stage_events[0], st));
    if (c.n_cunits > 0) {
        if (tb->dtype == AU_F64)
            launch_coef<double, T>(st, tb, ev0, c.d_evs, c.d_cunits, c.n_cunits, dirs, 0, 0, fs, fb, sg, M,
                                   (unsigned long long*)d_counts);
        else
            launch_coef<float, T>(st, tb, ev0, c.d_evs, c.d_cunits, c.n_cunits, dirs, 0, 0, fs, fb, sg, M,
                                  (unsigned long long*)d_counts);
        e = hipGetLastError();
        if (e != hipSuccess) return fail(AU_EDEVICE, std::string("k_coef: ") + hipGetErrorString(e));
    }
    if (stage_events) HIP_TRY(hipEventRecord(stage_events[1], st));
    e = launch_unfold<T>(c.N, c.variant, st, ev0, c.d_evs, c.d_uunits, c.n_uunits, kStationsPerUnit, X, M,
                         (T*)efield, tw, c.d_counter, c.persistent_blocks, c.d_xcd_off, c.xcd_max_list);
    if (e != hipSuccess) return fail(AU_EDEVICE, std::string("k_unfold: ") + hipGetErrorString(e));
    if (stage_events) HIP_TRY(hipEventRecord(stage_events[2], st));
    return AU_OK;
}

au_status au::enqueue_class(const au_table* tb, int prec, int tin, int64_t fs, double fb, double sg,
                            const ClassLaunch& c, const void* volt, void* efield, void* X, void* M,
                            const double* dirs, hipStream_t st, uint64_t* d_counts, hipEvent_t* stage_events)
{
    return prec == AU_PREC_FP64
               ? enqueue_class_t<double>(tb, tin, fs, fb, sg, c, volt, efield, X, M, dirs, st, d_counts, stage_events)
               : enqueue_class_t<float>(tb, tin, fs, fb, sg, c, volt, efield, X, M, dirs, st, d_counts, stage_events);
}

int au::current_variant(int prec, int n) { return unfold_variant(prec, n); }

int au::persistent_blocks(int prec, int n, int variant, int device)
{
    return prec == AU_PREC_FP64 ? persistent_blocks_for<double>(n, variant, device)
                                : persistent_blocks_for<float>(n, variant, device);
}

static au_status plan_enqueue(au_plan* pl, const void* d_volt, void* d_efield, hipStream_t st,
                              uint64_t* d_counts)
{
    const bool tm = pl->timing && !pl->ev.empty();
    if (tm) HIP_TRY(hipEventRecord(pl->ev[0], st));
    int ei = 1;
    const bool pers = (pl->flags & AU_PLAN_PERSISTENT) != 0;
    for (const ClassPlan& cp : pl->classes) {
        ClassLaunch c;
        c.N = cp.N;
        c.variant = cp.variant;
        c.d_evs = cp.d_evs;
        c.d_sunits = cp.d_sunits;
        c.n_sunits = cp.n_sunits;
        c.d_cunits = cp.d_cunits;
        c.n_cunits = cp.n_cunits;
        c.d_uunits = cp.d_uunits;
        c.n_uunits = cp.n_uunits;
        c.d_counter = (pers || cp.fused) ? cp.d_counter : nullptr;
        c.fused = cp.fused;
        c.persistent_blocks = cp.persistent_blocks;
        c.d_xcd_off = cp.d_xcd_off;
        c.xcd_max_list = cp.xcd_max_list;
        c.max_nb = cp.max_nb;
        au_status s = enqueue_class(pl->tb, pl->prec, pl->tin, pl->fs, pl->fb, pl->sg, c, d_volt, d_efield,
                                    pl->d_x, pl->d_m, pl->d_dirs, st, d_counts, tm ? &pl->ev[ei] : nullptr);
        if (s != AU_OK) return s;
        ei += 3;
    }
    if (tm) {
        HIP_TRY(hipEventSynchronize(pl->ev[ei - 1]));
        for (int i = 1; i < ei; ++i) {
            float ms = 0.f;
            HIP_TRY(hipEventElapsedTime(&ms, pl->ev[i - 1], pl->ev[i]));
            pl->stage_ms[i - 1] += ms;
        }
        ++pl->timed_runs;
    }
    return AU_OK;
}

extern "C" au_status au_plan_free(au_plan* pl)
{
    if (!pl) return AU_OK;
    if (pl->exec) (void)hipGraphExecDestroy(pl->exec);
    if (pl->graph) (void)hipGraphDestroy(pl->graph);
    if (pl->cap_stream) (void)hipStreamDestroy(pl->cap_stream);
    if (pl->d_mem) (void)hipFree(pl->d_mem);
    for (hipEvent_t e : pl->ev) (void)hipEventDestroy(e);
    delete pl;
    return AU_OK;
}

extern "C" au_status au_plan_create(const au_table* tb, const au_batch* b, au_plan** out)
{
    if (!b || !out) return fail(AU_EINVAL, "null argument");
    au_status s = check_common(tb, b->fs_hz, b->band_lo_hz, b->band_hi_hz, b->prec, b->trace_dtype,
                               b->fallback_rel, b->singular_rel);
    if (s != AU_OK) return s;
    if (b->n_events < 1 || !b->n_stations || !b->n_samples || !b->n_dirs || !b->h_dirs ||
        !b->volt_offset || !b->efield_offset)
        return fail(AU_EINVAL, "batch arrays missing");
    if (b->flags & ~(AU_PLAN_GRAPH | AU_PLAN_PERSISTENT | AU_PLAN_XCD | AU_PLAN_FUSED))
        return fail(AU_EINVAL, "unknown plan flags");
    int dev = 0;
    HIP_TRY(hipGetDevice(&dev));
    if (dev != tb->device) return fail(AU_EINVAL, "table lives on another device");
    const int E = b->n_events;
    const bool f64 = b->prec == AU_PREC_FP64;
    const size_t xb = f64 ? sizeof(XBin<double>) : sizeof(XBin<float>);
    const size_t mb = f64 ? sizeof(MBin<double>) : sizeof(MBin<float>);
    std::vector<EvParams> ps(E);
    std::vector<EvDesc> descs(E);
    int64_t dir_total = 0, x_total = 0, m_total = 0;
    uint64_t su = 0;
    for (int e = 0; e < E; ++e) {
        s = check_n(tb, b->n_stations[e], b->n_samples[e], b->fs_hz, b->band_lo_hz, b->band_hi_hz, &ps[e]);
        if (s != AU_OK) return fail(s, "event " + std::to_string(e) + ": " + g_err);
        if (b->n_dirs[e] < 1) return fail(AU_EINVAL, "event " + std::to_string(e) + ": n_dirs must be >= 1");
        if (b->volt_offset[e] < 0 || b->efield_offset[e] < 0)
            return fail(AU_EINVAL, "negative buffer offset");
    }
    // trace-length classes whose events all have few directions take the
    // fused spectrum + unfold kernel (no spectrum rows in the plan's memory)
    std::map<int, std::pair<int, int>> cls_max;  // N -> (most directions, widest band)
    for (int e = 0; e < E; ++e) {
        auto& m = cls_max[ps[e].N];
        m.first = std::max(m.first, b->n_dirs[e]);
        m.second = std::max(m.second, ps[e].nb);
    }
    auto class_fused = [&](int n) {
        const auto& m = cls_max[n];
        return (b->flags & AU_PLAN_FUSED) && fused_eligible(b->prec, n, m.first, m.second);
    };
    for (int e = 0; e < E; ++e) {
        EvDesc& d = descs[e];
        d = EvDesc{};
        d.volt_off = b->volt_offset[e];
        d.efield_off = b->efield_offset[e];
        d.x_off = class_fused(ps[e].N) ? 0 : x_total;
        d.m_off = m_total;
        d.dir_off = dir_total;
        d.S = ps[e].S;
        d.N = ps[e].N;
        d.D = b->n_dirs[e];
        d.k_lo = ps[e].k_lo;
        d.nb = ps[e].nb;
        if (!class_fused(ps[e].N)) x_total += (int64_t)d.S * d.nb;
        m_total += (int64_t)d.D * d.nb;
        dir_total += d.D;
        su += (uint64_t)d.S * d.D;
    }
    if (!dirs_finite(b->h_dirs, dir_total)) return fail(AU_EINVAL, "directions must be finite");
    // group by trace length; units sorted longest first
    std::vector<int> ns;
    for (int e = 0; e < E; ++e)
        if (std::find(ns.begin(), ns.end(), descs[e].N) == ns.end()) ns.push_back(descs[e].N);
    std::sort(ns.begin(), ns.end(), std::greater<int>());
    struct HostClass {
        int N;
        bool fused = false;
        std::vector<EvDesc> evs;
        std::vector<int2> su, cu;
        std::vector<int4> uu;
        std::vector<int> xcd_off;
        int xcd_max = 0;
    };
    std::vector<HostClass> hc;
    for (int n : ns) {
        HostClass c;
        c.N = n;
        c.fused = class_fused(n);
        for (int e = 0; e < E; ++e) {
            if (descs[e].N != n) continue;
            const int ci = (int)c.evs.size();
            c.evs.push_back(descs[e]);
            if (c.fused) {
                // units (event, -, station range) covering every direction
                for (int d = 0; d < descs[e].D; ++d) c.cu.push_back(int2{ci, d});
                for (int s0 = 0; s0 < descs[e].S; s0 += kFusedStations)
                    c.uu.push_back(int4{ci, 0, s0, std::min(descs[e].S, s0 + kFusedStations)});
                continue;
            }
            for (int st = 0; st < descs[e].S; ++st) c.su.push_back(int2{ci, st});
            for (int d = 0; d < descs[e].D; ++d) {
                c.cu.push_back(int2{ci, d});
                // events with many directions have units to spare: chunks of
                // twice the stations halve the per-unit start (work fetch and
                // the first station's loads) -- measured +1.5 % on 256
                // directions per event, and a loss at 16 directions per event
                const int cs = descs[e].D >= kWideUnitMinDirs ? 2 * kStationsPerUnit : kStationsPerUnit;
                for (int s0 = 0; s0 < descs[e].S; s0 += cs)
                    c.uu.push_back(int4{ci, d, s0, std::min(descs[e].S, s0 + cs)});
            }
        }
        if (b->flags & AU_PLAN_XCD) {
            // all units of one event (its directions' station chunks) go to one
            // of 8 lists, the list with the least work so far (work =
            // stations): the event's spectrum rows and each direction's
            // coefficient row are then fetched into one XCD's L2 only
            std::vector<std::vector<int4>> lists(8);
            std::vector<int64_t> load(8, 0);
            for (size_t i = 0; i < c.uu.size();) {
                size_t j = i;
                int64_t work = 0;
                while (j < c.uu.size() && c.uu[j].x == c.uu[i].x) {
                    work += c.uu[j].w - c.uu[j].z;
                    ++j;
                }
                const int x = (int)(std::min_element(load.begin(), load.end()) - load.begin());
                lists[x].insert(lists[x].end(), c.uu.begin() + i, c.uu.begin() + j);
                load[x] += work;
                i = j;
            }
            c.uu.clear();
            c.xcd_off.assign(1, 0);
            for (auto& l : lists) {
                c.uu.insert(c.uu.end(), l.begin(), l.end());
                c.xcd_off.push_back((int)c.uu.size());
                c.xcd_max = std::max(c.xcd_max, (int)l.size());
            }
        } else {
            std::stable_sort(c.uu.begin(), c.uu.end(),
                             [](const int4& a, const int4& bb) { return (a.w - a.z) > (bb.w - bb.z); });
        }
        if (c.uu.size() > 0x7fffffffu || c.cu.size() > 0x7fffffffu || c.su.size() > 0x7fffffffu)
            return fail(AU_EINVAL, "too many work units in one trace-length class");
        hc.push_back(std::move(c));
    }
    // one device allocation for everything the plan owns
    size_t off = 0;
    auto take = [&](size_t bytes) {
        const size_t o = off;
        off += align256(bytes + 1);
        return o;
    };
    const size_t o_x = take((size_t)x_total * xb);
    const size_t o_m = take((size_t)m_total * mb);
    const size_t o_dirs = take((size_t)dir_total * 2 * sizeof(double));
    struct Offs {
        size_t evs, su, cu, uu, ctr, xoff;
    };
    std::vector<Offs> co;
    for (auto& c : hc)
        co.push_back(Offs{take(c.evs.size() * sizeof(EvDesc)), take(c.su.size() * sizeof(int2)),
                          take(c.cu.size() * sizeof(int2)), take(c.uu.size() * sizeof(int4)),
                          take(8 * sizeof(unsigned int)), take(9 * sizeof(int))});
    au_plan* pl = new au_plan();
    pl->tb = tb;
    pl->device = dev;
    pl->prec = b->prec;
    pl->tin = b->trace_dtype;
    pl->flags = b->flags;
    pl->fs = b->fs_hz;
    pl->fb = b->fallback_rel;
    pl->sg = b->singular_rel;
    pl->station_unfolds = su;
    hipError_t e = hipMalloc(&pl->d_mem, off);
    if (e != hipSuccess) {
        au_plan_free(pl);
        return fail(AU_ENOMEM, std::string("hipMalloc(plan): ") + hipGetErrorString(e));
    }
    unsigned char* base = (unsigned char*)pl->d_mem;
    pl->d_x = base + o_x;
    pl->d_m = base + o_m;
    pl->d_dirs = (double*)(base + o_dirs);
#define PLAN_TRY(expr)                                                                      \
    do {                                                                                    \
        hipError_t e_ = (expr);                                                             \
        if (e_ != hipSuccess) {                                                             \
            au_plan_free(pl);                                                               \
            return fail(AU_EDEVICE, std::string(#expr) + ": " + hipGetErrorString(e_));    \
        }                                                                                   \
    } while (0)
    PLAN_TRY(hipMemcpy(pl->d_dirs, b->h_dirs, (size_t)dir_total * 2 * sizeof(double), hipMemcpyHostToDevice));
    for (size_t i = 0; i < hc.size(); ++i) {
        ClassPlan c;
        c.N = hc[i].N;
        c.fused = hc[i].fused;
        for (const EvDesc& d : hc[i].evs) {
            c.station_unfolds += (uint64_t)d.S * d.D;
            c.max_nb = std::max(c.max_nb, d.nb);
        }
        c.n_sunits = (int)hc[i].su.size();
        c.n_cunits = (int)hc[i].cu.size();
        c.n_uunits = (int)hc[i].uu.size();
        c.d_evs = (EvDesc*)(base + co[i].evs);
        c.d_sunits = (int2*)(base + co[i].su);
        c.d_cunits = (int2*)(base + co[i].cu);
        c.d_uunits = (int4*)(base + co[i].uu);
        c.d_counter = (unsigned int*)(base + co[i].ctr);
        if (!hc[i].xcd_off.empty()) {
            c.d_xcd_off = (int*)(base + co[i].xoff);
            c.xcd_max_list = hc[i].xcd_max;
            PLAN_TRY(hipMemcpy(c.d_xcd_off, hc[i].xcd_off.data(), 9 * sizeof(int), hipMemcpyHostToDevice));
        }
        PLAN_TRY(hipMemcpy(c.d_evs, hc[i].evs.data(), hc[i].evs.size() * sizeof(EvDesc), hipMemcpyHostToDevice));
        PLAN_TRY(hipMemcpy(c.d_sunits, hc[i].su.data(), hc[i].su.size() * sizeof(int2), hipMemcpyHostToDevice));
        PLAN_TRY(hipMemcpy(c.d_cunits, hc[i].cu.data(), hc[i].cu.size() * sizeof(int2), hipMemcpyHostToDevice));
        PLAN_TRY(hipMemcpy(c.d_uunits, hc[i].uu.data(), hc[i].uu.size() * sizeof(int4), hipMemcpyHostToDevice));
        c.variant = unfold_variant(b->prec, c.N);
        c.persistent_blocks = f64 ? persistent_blocks_for<double>(c.N, c.variant, dev)
                                  : persistent_blocks_for<float>(c.N, c.variant, dev);
        pl->classes.push_back(c);
    }
    if (pl->flags & AU_PLAN_GRAPH) PLAN_TRY(hipStreamCreateWithFlags(&pl->cap_stream, hipStreamNonBlocking));
#undef PLAN_TRY
    *out = pl;
    return AU_OK;
}

extern "C" au_status au_plan_timing(au_plan* pl, int32_t enable)
{
    if (!pl) return fail(AU_EINVAL, "null plan");
    if (enable && (pl->flags & AU_PLAN_GRAPH)) return fail(AU_EINVAL, "stage timing needs a plan without AU_PLAN_GRAPH");
    if (enable && pl->ev.empty()) {
        pl->ev.resize(3 * pl->classes.size() + 1);
        for (auto& e : pl->ev) HIP_TRY(hipEventCreate(&e));
    }
    pl->timing = enable != 0;
    pl->stage_ms.assign(3 * pl->classes.size(), 0.0);
    pl->timed_runs = 0;
    return AU_OK;
}

extern "C" au_status au_plan_classes(const au_plan* pl, int32_t max, int32_t* n_samples,
                                     uint64_t* station_unfolds, int32_t* variants, int32_t* n_classes)
{
    if (!pl || !n_classes) return fail(AU_EINVAL, "null argument");
    *n_classes = (int32_t)pl->classes.size();
    for (int32_t i = 0; i < max && i < (int32_t)pl->classes.size(); ++i) {
        if (n_samples) n_samples[i] = pl->classes[i].N;
        if (station_unfolds) station_unfolds[i] = pl->classes[i].station_unfolds;
        if (variants) variants[i] = pl->classes[i].variant;
    }
    return AU_OK;
}

extern "C" au_status au_plan_stage_ms(const au_plan* pl, int32_t max, double* ms, uint64_t* runs)
{
    if (!pl || !ms || !runs) return fail(AU_EINVAL, "null argument");
    for (int32_t i = 0; i < max && i < (int32_t)pl->stage_ms.size(); ++i) ms[i] = pl->stage_ms[i];
    *runs = pl->timed_runs;
    return AU_OK;
}

extern "C" au_status au_plan_units(const au_plan* pl, uint64_t* n)
{
    if (!pl || !n) return fail(AU_EINVAL, "null argument");
    *n = pl->station_unfolds;
    return AU_OK;
}

extern "C" au_status au_plan_run(au_plan* pl, const void* d_volt, void* d_efield, void* stream,
                                 uint64_t* d_counts)
{
    if (!pl || !d_volt || !d_efield) return fail(AU_EINVAL, "null argument");
    int dev = 0;
    HIP_TRY(hipGetDevice(&dev));
    if (dev != pl->device) return fail(AU_EINVAL, "plan lives on another device");
    hipStream_t st = (hipStream_t)stream;
    const bool f64 = pl->prec == AU_PREC_FP64;
    (void)f64;
    if (!(pl->flags & AU_PLAN_GRAPH)) return plan_enqueue(pl, d_volt, d_efield, st, d_counts);
    if (pl->exec == nullptr || pl->g_volt != d_volt || pl->g_efield != d_efield || pl->g_counts != d_counts) {
        if (pl->exec) {
            (void)hipGraphExecDestroy(pl->exec);
            pl->exec = nullptr;
        }
        if (pl->graph) {
            (void)hipGraphDestroy(pl->graph);
            pl->graph = nullptr;
        }
        HIP_TRY(hipStreamBeginCapture(pl->cap_stream, hipStreamCaptureModeThreadLocal));
        au_status s = plan_enqueue(pl, d_volt, d_efield, pl->cap_stream, d_counts);
        hipGraph_t g = nullptr;
        hipError_t e = hipStreamEndCapture(pl->cap_stream, &g);
        if (s != AU_OK) {
            if (g) (void)hipGraphDestroy(g);
            return s;
        }
        if (e != hipSuccess) return fail(AU_EDEVICE, std::string("hipStreamEndCapture: ") + hipGetErrorString(e));
        pl->graph = g;
        HIP_TRY(hipGraphInstantiate(&pl->exec, pl->graph, nullptr, nullptr, 0));
        pl->g_volt = d_volt;
        pl->g_efield = d_efield;
        pl->g_counts = d_counts;
    }
    HIP_TRY(hipGraphLaunch(pl->exec, st));
    return AU_OK;
}


// Per trace-length class, time every built unfold variant inside the plan
// itself (its own work lists, placement and persistent grid), with HIP events
// around the class's unfold launch, and keep the fastest.
extern "C" au_status au_plan_autotune(au_plan* pl, const void* d_volt, void* d_efield, int32_t reps, void* stream,
                                      double* ms, int32_t* best)
{
    if (!pl || !d_volt || !d_efield) return fail(AU_EINVAL, "null argument");
    if (reps < 1) return fail(AU_EINVAL, "reps must be >= 1");
    int dev = 0;
    HIP_TRY(hipGetDevice(&dev));
    if (dev != pl->device) return fail(AU_EINVAL, "plan lives on another device");
    hipStream_t st = (hipStream_t)stream;
    const bool was_timing = pl->timing;
    const std::vector<double> saved_ms = pl->stage_ms;
    const uint64_t saved_runs = pl->timed_runs;
    if (pl->ev.empty()) {
        pl->ev.resize(3 * pl->classes.size() + 1);
        for (auto& e : pl->ev) HIP_TRY(hipEventCreate(&e));
    }
    const int tsize = pl->prec == AU_PREC_FP64 ? 8 : 4;
    au_status rc = AU_OK;
    for (size_t i = 0; i < pl->classes.size() && rc == AU_OK; ++i) {
        ClassPlan& cp = pl->classes[i];
        if (cp.fused) {  // one fixed shape: nothing to tune
            if (ms)
                for (int v = 0; v < kNumVariants; ++v) ms[i * kNumVariants + v] = -1.0;
            if (best) best[i] = -1;
            continue;
        }
        double best_ms = 1e300;
        int best_v = cp.variant;
        for (int v = 0; v < kNumVariants && rc == AU_OK; ++v) {
            if (ms) ms[i * kNumVariants + v] = -1.0;
            if (!variant_built(cp.N, v, tsize)) continue;
            cp.variant = v;
            cp.persistent_blocks = au::persistent_blocks(pl->prec, cp.N, v, pl->device);
            pl->timing = false;
            rc = plan_enqueue(pl, d_volt, d_efield, st, nullptr);  // warm-up
            pl->timing = true;
            pl->stage_ms.assign(3 * pl->classes.size(), 0.0);
            pl->timed_runs = 0;
            for (int r = 0; r < reps && rc == AU_OK; ++r) rc = plan_enqueue(pl, d_volt, d_efield, st, nullptr);
            if (rc != AU_OK) break;
            const double t = pl->stage_ms[3 * i + 2] / reps;
            if (ms) ms[i * kNumVariants + v] = t;
            if (t < best_ms) {
                best_ms = t;
                best_v = v;
            }
        }
        cp.variant = best_v;
        cp.persistent_blocks = au::persistent_blocks(pl->prec, cp.N, best_v, pl->device);
        if (best) best[i] = best_v;
    }
    pl->timing = was_timing;
    pl->stage_ms = saved_ms;
    pl->timed_runs = saved_runs;
    if (pl->exec) {  // the captured graph holds the old launch shapes
        (void)hipGraphExecDestroy(pl->exec);
        pl->exec = nullptr;
    }
    if (pl->graph) {
        (void)hipGraphDestroy(pl->graph);
        pl->graph = nullptr;
    }
    return rc;
}

// ---------------------------------------------------------------------------
// unfold-kernel variants and the autotuner
// ---------------------------------------------------------------------------

static au_status check_variant_args(int32_t prec, int32_t n)
{
    if (prec != AU_PREC_FP32 && prec != AU_PREC_FP64) return fail(AU_EINVAL, "bad precision");
    if (n < 16 || n > 4096 || (n & (n - 1)) != 0) return fail(AU_EINVAL, "n_samples must be a power of two in [16, 4096]");
    return AU_OK;
}

extern "C" au_status au_unfold_variant_count(int32_t* count, int32_t* e_values, int32_t* rmax,
                                             int32_t* twmode, int32_t* wave, int32_t* pair, int32_t* pp)
{
    if (!count) return fail(AU_EINVAL, "null argument");
    *count = kNumVariants;
    for (int v = 0; v < kNumVariants; ++v) {
        if (e_values) e_values[v] = kUnfoldVariants[v].E;
        if (rmax) rmax[v] = kUnfoldVariants[v].rmax;
        if (twmode) twmode[v] = kUnfoldVariants[v].twmode;
        if (wave) wave[v] = kUnfoldVariants[v].wave ? 1 : 0;
        if (pair) pair[v] = kUnfoldVariants[v].pair ? 1 : 0;
        if (pp) pp[v] = kUnfoldVariants[v].pp ? 1 : 0;
    }
    return AU_OK;
}

extern "C" au_status au_set_unfold_variant(int32_t prec, int32_t n_samples, int32_t variant)
{
    au_status s = check_variant_args(prec, n_samples);
    if (s != AU_OK) return s;
    if (!variant_built(n_samples, variant, prec == AU_PREC_FP64 ? 8 : 4))
        return fail(AU_EINVAL, "variant not available for this trace length");
    std::lock_guard<std::mutex> lk(g_var_mu);
    g_variant[prec == AU_PREC_FP32 ? 1 : 0][ilog2(n_samples)] = variant;
    return AU_OK;
}

extern "C" au_status au_get_unfold_variant(int32_t prec, int32_t n_samples, int32_t* variant)
{
    au_status s = check_variant_args(prec, n_samples);
    if (s != AU_OK) return s;
    if (!variant) return fail(AU_EINVAL, "null argument");
    *variant = unfold_variant(prec, n_samples);
    return AU_OK;
}

// Deterministic filler for autotuning traces (a hash of the index mapped to
// [-1, 1)); the values do not matter for timing but avoid denormals.
template <typename Tin>
__global__ void k_fill_hash(Tin* p, int64_t n)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    uint32_t h = (uint32_t)i * 2654435761u;
    h ^= h >> 16;
    h *= 2246822519u;
    h ^= h >> 13;
    p[i] = (Tin)((double)(h & 0xffffff) / (double)0x800000 - 1.0);
}

extern "C" au_status au_autotune(const au_table* tb, const au_event* ev, int32_t n_dir, int32_t reps,
                                 double* ms, int32_t* best)
{
    EvParams p;
    au_status s = check_event(tb, ev, &p);
    if (s != AU_OK) return s;
    if (n_dir < 1 || reps < 1) return fail(AU_EINVAL, "n_dir and reps must be >= 1");
    int dev = 0;
    HIP_TRY(hipGetDevice(&dev));
    if (dev != tb->device) return fail(AU_EINVAL, "table lives on another device");
    const size_t in_el = (size_t)p.S * 2 * p.N;
    const size_t out_el = (size_t)n_dir * p.S * 2 * p.N;
    const size_t in_b = in_el * (ev->trace_dtype == AU_F64 ? 8 : 4);
    const size_t out_b = out_el * (ev->prec == AU_PREC_FP64 ? 8 : 4);
    const WsLayout w = ws_layout(p, ev->prec, n_dir);
    std::vector<double> dirs(2 * (size_t)n_dir);
    for (int d = 0; d < n_dir; ++d) {
        dirs[2 * d] = tb->g.zen0 + (d + 0.5) * (tb->g.dzen * (tb->g.n_zen - 1)) / n_dir;
        dirs[2 * d + 1] = tb->g.az0 + d * (360.0 / n_dir);
    }
    void *d_in = nullptr, *d_out = nullptr, *d_ws = nullptr;
    hipStream_t st = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    au_status rc = AU_OK;
    double best_ms = 1e300;
    int best_v = -1;
    auto cleanup = [&]() {
        if (e0) (void)hipEventDestroy(e0);
        if (e1) (void)hipEventDestroy(e1);
        if (st) (void)hipStreamDestroy(st);
        if (d_in) (void)hipFree(d_in);
        if (d_out) (void)hipFree(d_out);
        if (d_ws) (void)hipFree(d_ws);
    };
#define TUNE_TRY(expr)                                                                       \
    do {                                                                                     \
        hipError_t e_ = (expr);                                                              \
        if (e_ != hipSuccess) {                                                              \
            cleanup();                                                                       \
            return fail(AU_EDEVICE, std::string(#expr) + ": " + hipGetErrorString(e_));     \
        }                                                                                    \
    } while (0)
    TUNE_TRY(hipMalloc(&d_in, in_b));
    TUNE_TRY(hipMalloc(&d_out, out_b));
    TUNE_TRY(hipMalloc(&d_ws, w.total));
    TUNE_TRY(hipStreamCreateWithFlags(&st, hipStreamNonBlocking));
    TUNE_TRY(hipEventCreate(&e0));
    TUNE_TRY(hipEventCreate(&e1));
    const int fill_blocks = (int)((in_el + 255) / 256);
    if (ev->trace_dtype == AU_F64)
        hipLaunchKernelGGL(k_fill_hash<double>, dim3(fill_blocks), dim3(256), 0, st, (double*)d_in, (int64_t)in_el);
    else
        hipLaunchKernelGGL(k_fill_hash<float>, dim3(fill_blocks), dim3(256), 0, st, (float*)d_in, (int64_t)in_el);
    TUNE_TRY(hipGetLastError());
    for (int v = 0; v < kNumVariants; ++v) {
        if (ms) ms[v] = -1.0;
        if (!variant_built(p.N, v, ev->prec == AU_PREC_FP64 ? 8 : 4)) continue;
        for (int r = 0; r <= reps && rc == AU_OK; ++r) {
            if (r == 1) TUNE_TRY(hipEventRecord(e0, st));
            rc = ev->prec == AU_PREC_FP64
                     ? run_event<double>(tb, ev, p, d_in, n_dir, dirs.data(), 0, 0, d_out, d_ws, st, nullptr, v)
                     : run_event<float>(tb, ev, p, d_in, n_dir, dirs.data(), 0, 0, d_out, d_ws, st, nullptr, v);
        }
        if (rc != AU_OK) break;
        TUNE_TRY(hipEventRecord(e1, st));
        TUNE_TRY(hipEventSynchronize(e1));
        float t = 0.f;
        TUNE_TRY(hipEventElapsedTime(&t, e0, e1));
        const double avg = (double)t / reps;
        if (ms) ms[v] = avg;
        if (avg < best_ms) {
            best_ms = avg;
            best_v = v;
        }
    }
#undef TUNE_TRY
    cleanup();
    if (rc != AU_OK) return rc;
    if (best_v < 0) return fail(AU_EINVAL, "no variant could be timed");
    if (best) *best = best_v;
    return au_set_unfold_variant(ev->prec, p.N, best_v);
}

// ---------------------------------------------------------------------------
// HBM copy probe: the achievable-bandwidth reference for the roofline and
// the calibration kernel for the memory-traffic counters.
// ---------------------------------------------------------------------------

// Each thread moves four 16-byte words per trip (all loads issued before the
// stores) on a grid-stride loop; the tail (fewer than 4 words per thread) is
// handled one word at a time.
__global__ __launch_bounds__(256) void k_copy16(const uint4* __restrict__ src, uint4* __restrict__ dst, int64_t n16)
{
    const int64_t nthr = (int64_t)gridDim.x * blockDim.x;
    const int64_t tid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int64_t i = tid;
    for (; i + 3 * nthr < n16; i += 4 * nthr) {
        uint4 v[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) v[k] = src[i + k * nthr];
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            __builtin_nontemporal_store(v[k].x, &dst[i + k * nthr].x);
            __builtin_nontemporal_store(v[k].y, &dst[i + k * nthr].y);
            __builtin_nontemporal_store(v[k].z, &dst[i + k * nthr].z);
            __builtin_nontemporal_store(v[k].w, &dst[i + k * nthr].w);
        }
    }
    for (; i < n16; i += nthr) {
        const uint4 v = src[i];
        __builtin_nontemporal_store(v.x, &dst[i].x);
        __builtin_nontemporal_store(v.y, &dst[i].y);
        __builtin_nontemporal_store(v.z, &dst[i].z);
        __builtin_nontemporal_store(v.w, &dst[i].w);
    }
}

// Write-only probe: the unfold kernel's HBM stream is almost all writes.
__global__ __launch_bounds__(256) void k_fill16(uint4* __restrict__ dst, int64_t n16, uint32_t value)
{
    const int64_t nthr = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n16; i += nthr) {
        __builtin_nontemporal_store(value, &dst[i].x);
        __builtin_nontemporal_store(value, &dst[i].y);
        __builtin_nontemporal_store(value, &dst[i].z);
        __builtin_nontemporal_store(value, &dst[i].w);
    }
}

extern "C" au_status au_hbm_copy(void* d_dst, const void* d_src, uint64_t bytes, void* stream)
{
    if (!d_dst || !d_src) return fail(AU_EINVAL, "null pointer");
    if (bytes % 16 != 0 || ((uintptr_t)d_dst | (uintptr_t)d_src) % 16 != 0)
        return fail(AU_EINVAL, "copy size and addresses must be multiples of 16 bytes");
    if (bytes == 0) return AU_OK;
    int dev = 0, cus = 256;
    HIP_TRY(hipGetDevice(&dev));
    (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    const int64_t n16 = (int64_t)(bytes / 16);
    const int64_t want = (n16 + 255) / 256;
    const int grid = (int)std::min<int64_t>(want, (int64_t)cus * 32);
    hipLaunchKernelGGL(k_copy16, dim3(grid), dim3(256), 0, (hipStream_t)stream, (const uint4*)d_src, (uint4*)d_dst, n16);
    HIP_TRY(hipGetLastError());
    return AU_OK;
}

extern "C" au_status au_hbm_fill(void* d_dst, uint64_t bytes, uint32_t value, void* stream)
{
    if (!d_dst) return fail(AU_EINVAL, "null pointer");
    if (bytes % 16 != 0 || (uintptr_t)d_dst % 16 != 0)
        return fail(AU_EINVAL, "fill size and address must be multiples of 16 bytes");
    if (bytes == 0) return AU_OK;
    int dev = 0, cus = 256;
    HIP_TRY(hipGetDevice(&dev));
    (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    const int64_t n16 = (int64_t)(bytes / 16);
    const int grid = (int)std::min<int64_t>((n16 + 255) / 256, (int64_t)cus * 32);
    hipLaunchKernelGGL(k_fill16, dim3(grid), dim3(256), 0, (hipStream_t)stream, (uint4*)d_dst, n16, value);
    HIP_TRY(hipGetLastError());
    return AU_OK;
}

// ---------------------------------------------------------------------------
// envelope peaks of a direction scan
// ---------------------------------------------------------------------------

// Stations per envelope workgroup: up to 8 for large scans, fewer when
// directions x stations would leave the GPU short of workgroups (the
// reconstruction loop's one-direction launches).
static int env_spw(int S, int64_t n_dir)
{
    const int64_t want = 4 * 256;  // workgroups: a few per CU
    int spw = 8;
    while (spw > 1 && n_dir * ((S + spw - 1) / spw) < want) spw /= 2;
    return spw;
}

template <typename T, int N>
static hipError_t launch_env_n(hipStream_t st, const EvDesc& ev0, int spw, int n_units, const XBin<T>* X,
                               const MBin<T>* M, T* efield, T* peak, int* arg, const C2<T>* tw,
                               const int* skip = nullptr, const EvDesc* evs = nullptr,
                               const int4* units = nullptr, int skip_stride = 0, bool total_only = false)
{
    constexpr int E = N >= 1024 ? 8 : (N < 16 ? N : 16);
    constexpr int TT = N / E;
    constexpr int G = groups_per_block<T, N, E, env_bufs<T, E>()>();
    constexpr size_t LDS = ((size_t)G * env_bufs<T, E>() * lds_elems<N>() + env_ltw<T, N, E>()) * sizeof(C2<T>);
    hipLaunchKernelGGL((k_unfold_env<T, N, E>), dim3(n_units), dim3(G * TT), LDS, st, ev0, spw, X, M,
                       efield, peak, arg, tw, skip, evs, units, skip_stride, total_only ? 1 : 0);
    return hipGetLastError();
}

template <typename T>
static au_status run_envelope(const au_table* tb, const au_event* ev, const EvParams& p, const void* d_volt,
                              int n_dir, const double* h_dirs, void* d_efield, void* d_peak, int32_t* d_arg,
                              void* d_work, hipStream_t st, uint64_t* d_counts)
{
    const WsLayout w = ws_layout(p, ev->prec, n_dir);
    unsigned char* base = (unsigned char*)d_work;
    XBin<T>* X = (XBin<T>*)base;
    MBin<T>* M = (MBin<T>*)(base + w.x);
    double* dirs = (double*)(base + w.x + w.m);
    HIP_TRY(hipMemcpyAsync(dirs, h_dirs, sizeof(double) * 2 * n_dir, hipMemcpyHostToDevice, st));
    EvDesc ev0{};
    ev0.S = p.S;
    ev0.N = p.N;
    ev0.D = n_dir;
    ev0.k_lo = p.k_lo;
    ev0.nb = p.nb;
    const C2<T>* tw = twiddles<T>(tb->device);
    if (tw == nullptr) return fail(AU_EDEVICE, "twiddle tables missing on this device");
    hipError_t e;
    if (ev->trace_dtype == AU_F64)
        e = launch_spectrum<double, T>(p.N, st, (const double*)d_volt, ev0, nullptr, nullptr, p.S, ev0.nb, X, tw);
    else
        e = launch_spectrum<float, T>(p.N, st, (const float*)d_volt, ev0, nullptr, nullptr, p.S, ev0.nb, X, tw);
    if (e != hipSuccess) return fail(AU_EDEVICE, std::string("k_spectrum: ") + hipGetErrorString(e));
    if (tb->dtype == AU_F64)
        launch_coef<double, T>(st, tb, ev0, nullptr, nullptr, n_dir, dirs, 0, 0, ev->fs_hz, ev->fallback_rel,
                               ev->singular_rel, M, (unsigned long long*)d_counts);
    else
        launch_coef<float, T>(st, tb, ev0, nullptr, nullptr, n_dir, dirs, 0, 0, ev->fs_hz, ev->fallback_rel,
                              ev->singular_rel, M, (unsigned long long*)d_counts);
    e = hipGetLastError();
    if (e != hipSuccess) return fail(AU_EDEVICE, std::string("k_coef: ") + hipGetErrorString(e));
    const int spw = env_spw(p.S, n_dir);
    const int chunks = (p.S + spw - 1) / spw;
    const int64_t n_units = (int64_t)n_dir * chunks;
    if (n_units > (int64_t)0x7fffffff) return fail(AU_EINVAL, "too many work units");
    switch (p.N) {
#define X_(NN)                                                                                              \
    case NN:                                                                                                \
        e = launch_env_n<T, NN>(st, ev0, spw, (int)n_units, X, M, (T*)d_efield, (T*)d_peak, (int*)d_arg, tw); \
        break;
        AU_FOR_EACH_N(X_)
#undef X_
        default: e = hipErrorInvalidValue;
    }
    if (e != hipSuccess) return fail(AU_EDEVICE, std::string("k_unfold_env: ") + hipGetErrorString(e));
    return AU_OK;
}

extern "C" au_status au_unfold_envelope_scan(const au_table* tb, const au_event* ev, const void* d_volt,
                                             int32_t n_dir, const double* h_dirs, void* d_efield, void* d_peak,
                                             int32_t* d_arg, void* d_work, uint64_t work_bytes, void* stream,
                                             uint64_t* d_counts)
{
    EvParams p;
    au_status s = check_event(tb, ev, &p);
    if (s != AU_OK) return s;
    if (!d_volt || !d_peak || !d_arg || !h_dirs) return fail(AU_EINVAL, "null argument");
    if (n_dir < 1) return fail(AU_EINVAL, "n_dir must be >= 1");
    if (!dirs_finite(h_dirs, n_dir)) return fail(AU_EINVAL, "directions must be finite");
    int dev = 0;
    HIP_TRY(hipGetDevice(&dev));
    if (dev != tb->device) return fail(AU_EINVAL, "table lives on another device");
    const WsLayout w = ws_layout(p, ev->prec, n_dir);
    hipStream_t st = (hipStream_t)stream;
    void* work = d_work;
    bool pooled = false;
    if (work == nullptr) {
        hipError_t e = hipMallocAsync(&work, w.total, st);
        if (e != hipSuccess) return fail(AU_ENOMEM, std::string("hipMallocAsync: ") + hipGetErrorString(e));
        pooled = true;
    } else if (work_bytes < w.total) {
        return fail(AU_ENOMEM, "workspace smaller than au_workspace_bytes");
    }
    s = ev->prec == AU_PREC_FP64
            ? run_envelope<double>(tb, ev, p, d_volt, n_dir, h_dirs, d_efield, d_peak, d_arg, work, st, d_counts)
            : run_envelope<float>(tb, ev, p, d_volt, n_dir, h_dirs, d_efield, d_peak, d_arg, work, st, d_counts);
    if (pooled) {
        hipError_t e = hipFreeAsync(work, st);
        if (s == AU_OK && e != hipSuccess)
            return fail(AU_EDEVICE, std::string("hipFreeAsync: ") + hipGetErrorString(e));
    }
    return s;
}

// ---------------------------------------------------------------------------
// reconstruction loop (section 2, Fig. 1): voltage timing -> triangulation ->
// unfold -> envelope timing, repeated on the device with no host round trip;
// a device stop flag turns the steps after convergence into no-ops
// ---------------------------------------------------------------------------

namespace {

constexpr double kCMPerNs = 0.299792458;
constexpr int kMaxReconIter = 1024;

// larger value wins; equal values: the smaller index
template <typename V>
__device__ inline void amax_merge(V& v, int& i, V ov, int oi)
{
    if (ov > v || (ov == v && oi < i)) {
        v = ov;
        i = oi;
    }
}

// block-wide argmax over kBlock threads, result in thread 0
__device__ void block_argmax(double& v, int& i)
{
    __shared__ double sv[kBlock / 64];
    __shared__ int si[kBlock / 64];
    for (int off = 32; off >= 1; off >>= 1) amax_merge(v, i, __shfl_xor(v, off), __shfl_xor(i, off));
    if ((threadIdx.x & 63) == 0) {
        sv[threadIdx.x >> 6] = v;
        si[threadIdx.x >> 6] = i;
    }
    __syncthreads();
    if (threadIdx.x == 0)
        for (int w = 1; w < kBlock / 64; ++w) amax_merge(v, i, sv[w], si[w]);
}

// block-wide sums of K doubles over kBlock threads, result in every thread
template <int K>
__device__ void block_sum(double (&v)[K])
{
    __shared__ double sv[K][kBlock / 64];
#pragma unroll
    for (int k = 0; k < K; ++k) {
        for (int off = 32; off >= 1; off >>= 1) v[k] += __shfl_xor(v[k], off);
        if ((threadIdx.x & 63) == 0) sv[k][threadIdx.x >> 6] = v[k];
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < K; ++k) {
        v[k] = 0.0;
        for (int w = 0; w < kBlock / 64; ++w) v[k] += sv[k][w];
    }
    __syncthreads();
}

}  // namespace

// First station times: the smallest sample maximising V_0^2 + V_1^2, in double
// with every operation rounded on its own (no contraction into fma), so the
// decision is the one a plain double evaluation takes.  One block per station.
template <typename Tin>
__global__ __launch_bounds__(kBlock) void k_volt_timing(const Tin* __restrict__ volt, int N, int* __restrict__ t0,
                                                         const EvDesc* __restrict__ evs,
                                                         const int2* __restrict__ units)
{
#pragma clang fp contract(off)
    // station blockIdx.x of one event, or units[blockIdx.x] = (event, station)
    const Tin* __restrict__ v0 =
        units != nullptr ? volt + evs[units[blockIdx.x].x].volt_off + (int64_t)units[blockIdx.x].y * 2 * N
                         : volt + (int64_t)blockIdx.x * 2 * N;
    const Tin* __restrict__ v1 = v0 + N;
    double bv = -1.0;
    int bi = 0;
    for (int j = threadIdx.x; j < N; j += kBlock) {
        const double a = (double)v0[j], b = (double)v1[j];
        const double pw = a * a + b * b;
        amax_merge(bv, bi, pw, j);
    }
    block_argmax(bv, bi);
    if (threadIdx.x == 0) t0[blockIdx.x] = bi;
}

// One step of the loop, one block.  state: [0] stop, [1] directions produced,
// [2] converged, [3] degenerate station geometry.  For it >= 1 the total-field
// envelope maxima of the previous unfold become times row it; when no station
// time changed the loop has converged and stops.  Otherwise (and at it = 0,
// whose row holds the voltage maxima) the plane wave t = t0 + p x + q y is
// fitted by least squares about the centroid and the direction of arrival,
// n = (-c p, -c q) on the ground, is written to dirs[it] and cur.  last: the
// step after the final unfold, convergence check only.
// Many events: workgroup e takes event e, whose stations are [so, so + S) of
// the Stot stations (ev_st[e] = (so, S)), with state, cur and dirs
// (max_iter directions) per event.  One event: ev_st == nullptr, Stot = S.
// The work of workgroup e (thread 0 writes the results).
__device__ __forceinline__ void recon_step_block(int e, int it, int last, int S, double dt_ns,
                                                 const double* __restrict__ pos, const int* __restrict__ env_arg,
                                                 int* __restrict__ hist, double* dirs, double* cur, int* state,
                                                 const int2* __restrict__ ev_st, int Stot, int max_iter)
{
    int so = 0;
    if (ev_st != nullptr) {
        so = ev_st[e].x;
        S = ev_st[e].y;
    }
    state += 4 * e;
    cur += 2 * e;
    dirs += (int64_t)2 * max_iter * e;
    pos += 2 * (int64_t)so;
    env_arg += 3 * (int64_t)so;
    if (it == 0) {
        // the first step starts the event's state (the workspace may hold a
        // previous call's); nothing reads it before this step
        if (threadIdx.x == 0) state[0] = state[1] = state[2] = state[3] = 0;
    } else if (state[0]) {
        return;
    }
    int* __restrict__ row = hist + (int64_t)it * Stot + so;
    if (it > 0) {
        int changed = 0;
        for (int s = threadIdx.x; s < S; s += kBlock) {
            const int t = env_arg[3 * s + 2];
            changed |= t != row[s - Stot];
            row[s] = t;
        }
        changed = __syncthreads_or(changed);
        if (!changed || last) {
            if (threadIdx.x == 0) {
                state[0] = 1;
                state[2] = !changed;
            }
            return;
        }
    }
    double m[3] = {0.0, 0.0, 0.0};
    for (int s = threadIdx.x; s < S; s += kBlock) {
        m[0] += pos[2 * s];
        m[1] += pos[2 * s + 1];
        m[2] += (double)row[s] * dt_ns;
    }
    block_sum(m);
    const double inv_s = 1.0 / (double)S;
    const double mx = m[0] * inv_s, my = m[1] * inv_s, mt = m[2] * inv_s;
    double c[5] = {0.0, 0.0, 0.0, 0.0, 0.0};  // xx, xy, yy, xt, yt about the centroid
    for (int s = threadIdx.x; s < S; s += kBlock) {
        const double dx = pos[2 * s] - mx, dy = pos[2 * s + 1] - my, dt = (double)row[s] * dt_ns - mt;
        c[0] += dx * dx;
        c[1] += dx * dy;
        c[2] += dy * dy;
        c[3] += dx * dt;
        c[4] += dy * dt;
    }
    block_sum(c);
    if (threadIdx.x != 0) return;
    const double det = c[0] * c[2] - c[1] * c[1];
    const double p = (c[2] * c[3] - c[1] * c[4]) / det, q = (c[0] * c[4] - c[1] * c[3]) / det;
    const double nx = -kCMPerNs * p, ny = -kCMPerNs * q;
    const double sn = fmin(1.0, sqrt(nx * nx + ny * ny));
    double az = atan2(ny, nx) * (180.0 / M_PI);
    if (az < 0.0) az += 360.0;
    const double zen = asin(sn) * (180.0 / M_PI);
    if (!(det > 1e-12 * c[0] * c[2]) || !isfinite(zen) || !isfinite(az)) {
        cur[0] = 0.0;
        cur[1] = 0.0;
        state[3] = 1;
        state[0] = 1;
        return;
    }
    dirs[2 * it] = zen;
    dirs[2 * it + 1] = az;
    cur[0] = zen;
    cur[1] = az;
    state[1] = it + 1;
}

__global__ __launch_bounds__(kBlock) void k_recon_step(int it, int last, int S, double dt_ns,
                                                        const double* __restrict__ pos,
                                                        const int* __restrict__ env_arg, int* __restrict__ hist,
                                                        double* __restrict__ dirs, double* __restrict__ cur,
                                                        int* __restrict__ state, const int2* __restrict__ ev_st,
                                                        int Stot, int max_iter)
{
    recon_step_block(blockIdx.x, it, last, S, dt_ns, pos, env_arg, hist, dirs, cur, state, ev_st, Stot, max_iter);
}

// One event's step `it` (not the last) and, unless it stopped the loop, the
// coefficient rows of the direction it produced: the step's two
// single-workgroup launches (k_recon_step, then k_coef of one direction
// skipped on the stop flag) as one.  The step's thread 0 writes the direction
// and the flag before the barrier that precedes the coefficients' reads.
template <typename Tt, typename T>
__global__ __launch_bounds__(kBlock) void k_recon_step_coef(int it, int S, double dt_ns,
                                                             const double* __restrict__ pos,
                                                             const int* __restrict__ env_arg,
                                                             int* __restrict__ hist, double* dirs, double* cur,
                                                             int* state, int max_iter,
                                                             const C2<Tt>* __restrict__ nodes, GridDev gd,
                                                             EvDesc ev0, int64_t fs, double fallback_rel,
                                                             double singular_rel, MBin<T>* __restrict__ M)
{
    recon_step_block(0, it, 0, S, dt_ns, pos, env_arg, hist, dirs, cur, state, nullptr, S, max_iter);
    __syncthreads();
    coef_block<Tt, T, false>(0, nodes, gd, ev0, nullptr, nullptr, cur, 0.0, 0.0, fs, fallback_rel, singular_rel, M,
                             nullptr, 0.0, state, 0);
}

namespace {

struct ReconLayout {
    size_t base, hist, dirs, cur, state, pos, peak, arg, total;
};

ReconLayout recon_layout(const EvParams& p, int prec, int max_iter)
{
    ReconLayout r;
    r.base = ws_layout(p, prec, 1).total;
    r.hist = align256((size_t)(max_iter + 1) * p.S * sizeof(int32_t));
    r.dirs = align256((size_t)max_iter * 2 * sizeof(double));
    r.cur = 256;
    r.state = 256;
    r.pos = align256((size_t)p.S * 2 * sizeof(double));
    r.peak = align256((size_t)p.S * 3 * (prec == AU_PREC_FP64 ? sizeof(double) : sizeof(float)));
    r.arg = align256((size_t)p.S * 3 * sizeof(int32_t));
    r.total = r.base + r.hist + r.dirs + r.cur + r.state + r.pos + r.peak + r.arg;
    return r;
}

au_status check_recon(const au_table* tb, const au_event* ev, int32_t max_iter, EvParams* p)
{
    au_status s = check_event(tb, ev, p);
    if (s != AU_OK) return s;
    if (p->S < 3) return fail(AU_EINVAL, "the reconstruction needs at least 3 stations");
    if (max_iter < 1 || max_iter > kMaxReconIter) return fail(AU_EINVAL, "max_iter must be in [1, 1024]");
    return AU_OK;
}

}  // namespace

// A pinned host buffer of the calling thread of at least `bytes` (null if it
// cannot be allocated: callers then copy to pageable memory).  One per
// thread that calls it, grown as needed and never freed otherwise (a few
// KiB: one reconstruction's station positions and results).  Every call
// that uses it waits for its stream before returning, so growing it frees
// no buffer that a copy still uses.
static void* pinned_scratch(size_t bytes)
{
    thread_local void* buf = nullptr;
    thread_local size_t cap = 0;
    if (bytes > cap) {
        if (buf != nullptr) (void)hipHostFree(buf);
        buf = nullptr;
        cap = 0;
        if (hipHostMalloc(&buf, bytes, hipHostMallocDefault) != hipSuccess) {
            buf = nullptr;
            (void)hipGetLastError();
            return nullptr;
        }
        cap = bytes;
    }
    return buf;
}

template <typename T>
static au_status run_reconstruct(const au_table* tb, const au_event* ev, const EvParams& p, const void* d_volt,
                                 const double* h_pos, int max_iter, void* d_efield, void* d_peak, void* d_work,
                                 hipStream_t st, double* h_dirs, int32_t* h_times, int32_t* h_state)
{
    const ReconLayout r = recon_layout(p, ev->prec, max_iter);
    const WsLayout w = ws_layout(p, ev->prec, 1);
    unsigned char* base = (unsigned char*)d_work;
    XBin<T>* X = (XBin<T>*)base;
    MBin<T>* M = (MBin<T>*)(base + w.x);
    unsigned char* q = base + r.base;
    int* hist = (int*)q;
    double* dirs = (double*)(q += r.hist);
    double* cur = (double*)(q += r.dirs);
    int* state = (int*)(q += r.cur);
    double* pos = (double*)(q += r.state);
    T* peak = d_peak ? (T*)d_peak : (T*)(q += r.pos);
    int* arg = (int*)(base + r.total - r.arg);
    // The thread's pinned buffer: the results region (times, directions,
    // state), then the station positions, which go up from there as an
    // asynchronous copy instead of a staged pageable one.  (The previous call
    // on this thread ended with a wait for its stream.)
    const size_t res_bytes = r.hist + r.dirs + r.cur + sizeof(int32_t) * 4;
    const size_t pos_bytes = sizeof(double) * 2 * p.S;
    unsigned char* hb = (unsigned char*)pinned_scratch(res_bytes + pos_bytes);
    if (hb != nullptr) {
        std::memcpy(hb + res_bytes, h_pos, pos_bytes);
        HIP_TRY(hipMemcpyAsync(pos, hb + res_bytes, pos_bytes, hipMemcpyHostToDevice, st));
    } else {
        HIP_TRY(hipMemcpyAsync(pos, h_pos, pos_bytes, hipMemcpyHostToDevice, st));
    }
    EvDesc ev0{};
    ev0.S = p.S;
    ev0.N = p.N;
    ev0.D = 1;
    ev0.k_lo = p.k_lo;
    ev0.nb = p.nb;
    const C2<T>* tw = twiddles<T>(tb->device);
    if (tw == nullptr) return fail(AU_EDEVICE, "twiddle tables missing on this device");
    hipError_t e;
    if (ev->trace_dtype == AU_F64) {
        e = launch_spectrum<double, T>(p.N, st, (const double*)d_volt, ev0, nullptr, nullptr, p.S, ev0.nb, X, tw);
        hipLaunchKernelGGL(k_volt_timing<double>, dim3(p.S), dim3(kBlock), 0, st, (const double*)d_volt, p.N, hist,
                           (const EvDesc*)nullptr, (const int2*)nullptr);
    } else {
        e = launch_spectrum<float, T>(p.N, st, (const float*)d_volt, ev0, nullptr, nullptr, p.S, ev0.nb, X, tw);
        hipLaunchKernelGGL(k_volt_timing<float>, dim3(p.S), dim3(kBlock), 0, st, (const float*)d_volt, p.N, hist,
                           (const EvDesc*)nullptr, (const int2*)nullptr);
    }
    if (e == hipSuccess) e = hipGetLastError();
    if (e != hipSuccess) return fail(AU_EDEVICE, std::string("spectrum/timing: ") + hipGetErrorString(e));
    const double dt_ns = 1e9 / (double)ev->fs_hz;
    // The loop's launches, in order: op 2 it is step `it` (with the
    // coefficient rows of its direction; for it = max_iter the final
    // convergence check alone), op 2 it + 1 the unfold and envelope timing of
    // pass `it`.  Once the device stop flag is set every later launch is a
    // no-op, so the host enqueues them in chunks, each ending with a step,
    // and reads the results after each chunk: when the loop has stopped (the
    // usual case after the first chunk, which ends with step 2) the rest is
    // never enqueued.  The results equal those of the whole sequence.
    const int n_ops = 2 * max_iter + 1;
    const int spw = env_spw(p.S, 1);
    const int chunks = (p.S + spw - 1) / spw;
    auto enqueue_op = [&](int op) -> au_status {
        const int it = op / 2;
        hipError_t e = hipSuccess;
        if (op % 2 == 0 && it == max_iter) {
            hipLaunchKernelGGL(k_recon_step, dim3(1), dim3(kBlock), 0, st, it, 1, p.S, dt_ns, (const double*)pos,
                               (const int*)arg, hist, dirs, cur, state, (const int2*)nullptr, p.S, max_iter);
        } else if (op % 2 == 0) {
            if (tb->dtype == AU_F64)
                hipLaunchKernelGGL((k_recon_step_coef<double, T>), dim3(1), dim3(kBlock), 0, st, it, p.S, dt_ns,
                                   (const double*)pos, (const int*)arg, hist, dirs, cur, state, max_iter,
                                   (const C2<double>*)tb->d_nodes, tb->g, ev0, ev->fs_hz, ev->fallback_rel,
                                   ev->singular_rel, M);
            else
                hipLaunchKernelGGL((k_recon_step_coef<float, T>), dim3(1), dim3(kBlock), 0, st, it, p.S, dt_ns,
                                   (const double*)pos, (const int*)arg, hist, dirs, cur, state, max_iter,
                                   (const C2<float>*)tb->d_nodes, tb->g, ev0, ev->fs_hz, ev->fallback_rel,
                                   ev->singular_rel, M);
        } else {
            switch (p.N) {
#define X_(NN)                                                                                               \
    case NN:                                                                                                 \
        e = launch_env_n<T, NN>(st, ev0, spw, chunks, X, M, (T*)d_efield, peak, arg, tw, (const int*)state); \
        break;
                AU_FOR_EACH_N(X_)
#undef X_
                default: e = hipErrorInvalidValue;
            }
        }
        if (e == hipSuccess) e = hipGetLastError();
        if (e != hipSuccess) return fail(AU_EDEVICE, std::string("reconstruction step: ") + hipGetErrorString(e));
        return AU_OK;
    };
    // the results (times, directions, state: one contiguous region of the
    // workspace) in one copy through pinned memory, instead of three staged
    // copies from pageable memory that each wait for the one before
    auto fetch = [&]() -> au_status {
        if (hb != nullptr) {
            HIP_TRY(hipMemcpyAsync(hb, hist, res_bytes, hipMemcpyDeviceToHost, st));
            HIP_TRY(hipStreamSynchronize(st));
            std::memcpy(h_times, hb, sizeof(int32_t) * (size_t)(max_iter + 1) * p.S);
            std::memcpy(h_dirs, hb + r.hist, sizeof(double) * 2 * max_iter);
            std::memcpy(h_state, hb + r.hist + r.dirs + r.cur, sizeof(int32_t) * 4);
            return AU_OK;
        }
        HIP_TRY(hipMemcpyAsync(h_state, state, sizeof(int32_t) * 4, hipMemcpyDeviceToHost, st));
        HIP_TRY(hipMemcpyAsync(h_dirs, dirs, sizeof(double) * 2 * max_iter, hipMemcpyDeviceToHost, st));
        HIP_TRY(hipMemcpyAsync(h_times, hist, sizeof(int32_t) * (size_t)(max_iter + 1) * p.S, hipMemcpyDeviceToHost,
                               st));
        HIP_TRY(hipStreamSynchronize(st));
        return AU_OK;
    };
    int op = 0;
    for (int check = std::min(4, n_ops - 1);; check = std::min(check + 8, n_ops - 1)) {
        for (; op <= check; ++op) {
            const au_status s = enqueue_op(op);
            if (s != AU_OK) return s;
        }
        const au_status s = fetch();
        if (s != AU_OK) return s;
        if (h_state[0] != 0 || op >= n_ops) return AU_OK;
    }
}

extern "C" au_status au_reconstruct_workspace_bytes(const au_table* tb, const au_event* ev, int32_t max_iter,
                                                    uint64_t* bytes)
{
    if (!bytes) return fail(AU_EINVAL, "null argument");
    EvParams p;
    au_status s = check_recon(tb, ev, max_iter, &p);
    if (s != AU_OK) return s;
    *bytes = recon_layout(p, ev->prec, max_iter).total;
    return AU_OK;
}

extern "C" au_status au_reconstruct(const au_table* tb, const au_event* ev, const void* d_volt,
                                    const double* h_pos, int32_t max_iter, double* h_dirs, int32_t* h_times,
                                    int32_t* n_dirs, int32_t* converged, void* d_efield, void* d_peak,
                                    void* d_work, uint64_t work_bytes, void* stream)
{
    EvParams p;
    au_status s = check_recon(tb, ev, max_iter, &p);
    if (s != AU_OK) return s;
    if (!d_volt || !h_pos || !h_dirs || !h_times || !n_dirs || !converged) return fail(AU_EINVAL, "null argument");
    for (int64_t i = 0; i < 2 * (int64_t)p.S; ++i)
        if (!std::isfinite(h_pos[i]) || std::fabs(h_pos[i]) > 1e7)
            return fail(AU_EINVAL, "station positions must be finite and within 1e7 m");
    int dev = 0;
    HIP_TRY(hipGetDevice(&dev));
    if (dev != tb->device) return fail(AU_EINVAL, "table lives on another device");
    const ReconLayout r = recon_layout(p, ev->prec, max_iter);
    hipStream_t st = (hipStream_t)stream;
    void* work = d_work;
    bool pooled = false;
    if (work == nullptr) {
        hipError_t e = hipMallocAsync(&work, r.total, st);
        if (e != hipSuccess) return fail(AU_ENOMEM, std::string("hipMallocAsync: ") + hipGetErrorString(e));
        pooled = true;
    } else if (work_bytes < r.total) {
        return fail(AU_ENOMEM, "workspace smaller than au_reconstruct_workspace_bytes");
    }
    int32_t state[4] = {0, 0, 0, 0};
    s = ev->prec == AU_PREC_FP64
            ? run_reconstruct<double>(tb, ev, p, d_volt, h_pos, max_iter, d_efield, d_peak, work, st, h_dirs,
                                      h_times, state)
            : run_reconstruct<float>(tb, ev, p, d_volt, h_pos, max_iter, d_efield, d_peak, work, st, h_dirs,
                                     h_times, state);
    if (pooled) {
        hipError_t e = hipFreeAsync(work, st);
        if (s == AU_OK && e != hipSuccess)
            return fail(AU_EDEVICE, std::string("hipFreeAsync: ") + hipGetErrorString(e));
    }
    if (s != AU_OK) return s;
    *n_dirs = state[1];
    *converged = state[2];
    if (state[3]) return fail(AU_EINVAL, "degenerate station geometry (collinear or coincident stations)");
    return AU_OK;
}

// ---------------------------------------------------------------------------
// direction fit: plane-wave timing-consistency score over candidate
// directions, device argmin and local refinement grids, no host round trip
// between levels
// ---------------------------------------------------------------------------

// Score of every candidate (one block each): r_s = t_s dt - tau_s with
// tau_s = -(n . x_s) / c, chi2 = sum_s (r_s - mean r)^2 (ns^2), and the summed
// squared total-field envelope peaks.  t_s and the peaks are component 2 of
// the envelope scan's [D][S][3] outputs.
template <typename T>
__global__ __launch_bounds__(kBlock) void k_dir_score(int S, const double* __restrict__ pos,
                                                       const double* __restrict__ dirs, const int* __restrict__ arg,
                                                       const T* __restrict__ peak, double dt_ns,
                                                       double* __restrict__ chi2, double* __restrict__ power)
{
    const int d = blockIdx.x;
    const double zr = dirs[2 * d] * (M_PI / 180.0), ar = dirs[2 * d + 1] * (M_PI / 180.0);
    const double nx = sin(zr) * cos(ar), ny = sin(zr) * sin(ar);
    const int* __restrict__ t = arg + (int64_t)d * S * 3;
    double m[1] = {0.0};
    for (int s = threadIdx.x; s < S; s += kBlock)
        m[0] += (double)t[3 * s + 2] * dt_ns + (nx * pos[2 * s] + ny * pos[2 * s + 1]) / kCMPerNs;
    block_sum(m);
    const double mean = m[0] / (double)S;
    double acc[2] = {0.0, 0.0};
    for (int s = threadIdx.x; s < S; s += kBlock) {
        const double r = (double)t[3 * s + 2] * dt_ns + (nx * pos[2 * s] + ny * pos[2 * s + 1]) / kCMPerNs - mean;
        const double p = (double)peak[((int64_t)d * S + s) * 3 + 2];
        acc[0] += r * r;
        acc[1] += p * p;
    }
    block_sum(acc);
    if (threadIdx.x == 0) {
        chi2[d] = acc[0];
        power[d] = acc[1];
    }
}

// Best candidate of a level (smallest chi2, the first on ties) into best and
// result; then, if next is non-null, the k x k grid of the next level around
// it: zenith zc + (i - (k-1)/2) hz clamped to [0, 90], azimuth
// ac + (j - (k-1)/2) ha wrapped to [0, 360), every operation rounded on its
// own so the grid is exactly the plain double evaluation.
__global__ __launch_bounds__(kBlock) void k_dir_best(int nc, const double* __restrict__ chi2,
                                                      const double* __restrict__ cand, int* __restrict__ best,
                                                      double* __restrict__ result, double hz, double ha, int k,
                                                      double* __restrict__ next)
{
#pragma clang fp contract(off)
    __shared__ double centre[2];
    double v = -INFINITY;
    int bi = 0;
    for (int d = threadIdx.x; d < nc; d += kBlock) amax_merge(v, bi, -chi2[d], d);
    block_argmax(v, bi);
    if (threadIdx.x == 0) {
        *best = bi;
        centre[0] = result[0] = cand[2 * bi];
        centre[1] = result[1] = cand[2 * bi + 1];
    }
    __syncthreads();
    if (next == nullptr) return;
    const double m = 0.5 * (double)(k - 1);
    for (int q = threadIdx.x; q < k * k; q += kBlock) {
        const int i = q / k, j = q - (q / k) * k;
        double z = centre[0] + ((double)i - m) * hz;
        z = z < 0.0 ? 0.0 : (z > 90.0 ? 90.0 : z);
        double a = centre[1] + ((double)j - m) * ha;
        a = a - 360.0 * floor(a / 360.0);
        if (a >= 360.0) a -= 360.0;
        next[2 * q] = z;
        next[2 * q + 1] = a;
    }
}

namespace {

constexpr int kMaxFitLevels = 16;
constexpr int kMaxFitK = 15;

struct FitLayout {
    size_t x, m, dirs, chi2, power, best, result, pos, peak, arg, total;
    int64_t n_cand, d_max;
};

FitLayout fit_layout(const EvParams& p, int prec, int n_dir, int levels, int k)
{
    FitLayout f;
    f.n_cand = (int64_t)n_dir + (int64_t)levels * k * k;
    f.d_max = std::max<int64_t>(n_dir, (int64_t)k * k);
    const size_t tsz = prec == AU_PREC_FP64 ? sizeof(double) : sizeof(float);
    const WsLayout w = ws_layout(p, prec, (int)f.d_max);
    f.x = w.x;
    f.m = w.m;
    f.dirs = align256((size_t)f.n_cand * 2 * sizeof(double));
    f.chi2 = align256((size_t)f.n_cand * sizeof(double));
    f.power = f.chi2;
    f.best = align256((size_t)(levels + 1) * sizeof(int32_t));
    f.result = 256;
    f.pos = align256((size_t)p.S * 2 * sizeof(double));
    f.peak = align256((size_t)f.d_max * p.S * 3 * tsz);
    f.arg = align256((size_t)f.d_max * p.S * 3 * sizeof(int32_t));
    f.total = f.x + f.m + f.dirs + f.chi2 + f.power + f.best + f.result + f.pos + f.peak + f.arg;
    return f;
}

au_status check_fit(const au_table* tb, const au_event* ev, int32_t n_dir, int32_t levels, int32_t k,
                    double step_zen, double step_az, EvParams* p)
{
    au_status s = check_event(tb, ev, p);
    if (s != AU_OK) return s;
    if (p->S < 3) return fail(AU_EINVAL, "the direction fit needs at least 3 stations");
    if (n_dir < 1) return fail(AU_EINVAL, "n_dir must be >= 1");
    if (levels < 0 || levels > kMaxFitLevels) return fail(AU_EINVAL, "levels must be in [0, 16]");
    if (k < 1 || k > kMaxFitK) return fail(AU_EINVAL, "k must be in [1, 15]");
    if (levels > 0 && (!(step_zen > 0.0) || !(step_az > 0.0) || !std::isfinite(step_zen) ||
                       !std::isfinite(step_az) || step_zen > 90.0 || step_az > 360.0))
        return fail(AU_EINVAL, "steps must be in (0, 90] and (0, 360]");
    const int64_t units = std::max<int64_t>(n_dir, (int64_t)k * k) * p->S;  // at one station per workgroup
    if (units > (int64_t)0x7fffffff) return fail(AU_EINVAL, "too many work units");
    return AU_OK;
}

}  // namespace

template <typename T>
static au_status run_fit(const au_table* tb, const au_event* ev, const EvParams& p, const void* d_volt,
                         const double* h_pos, int n_dir, const double* h_dirs, int levels, int k, double step_zen,
                         double step_az, void* d_work, hipStream_t st, double* h_level_dirs, double* h_chi2,
                         double* h_power, int32_t* h_best, double* h_result)
{
    const FitLayout f = fit_layout(p, ev->prec, n_dir, levels, k);
    unsigned char* q = (unsigned char*)d_work;
    XBin<T>* X = (XBin<T>*)q;
    MBin<T>* M = (MBin<T>*)(q += f.x);
    double* dirs = (double*)(q += f.m);
    double* chi2 = (double*)(q += f.dirs);
    double* power = (double*)(q += f.chi2);
    int* best = (int*)(q += f.power);
    double* result = (double*)(q += f.best);
    double* pos = (double*)(q += f.result);
    T* peak = (T*)(q += f.pos);
    int* arg = (int*)(q += f.peak);
    HIP_TRY(hipMemcpyAsync(dirs, h_dirs, sizeof(double) * 2 * n_dir, hipMemcpyHostToDevice, st));
    HIP_TRY(hipMemcpyAsync(pos, h_pos, sizeof(double) * 2 * p.S, hipMemcpyHostToDevice, st));
    EvDesc ev0{};
    ev0.S = p.S;
    ev0.N = p.N;
    ev0.k_lo = p.k_lo;
    ev0.nb = p.nb;
    const C2<T>* tw = twiddles<T>(tb->device);
    if (tw == nullptr) return fail(AU_EDEVICE, "twiddle tables missing on this device");
    hipError_t e = ev->trace_dtype == AU_F64
                       ? launch_spectrum<double, T>(p.N, st, (const double*)d_volt, ev0, nullptr, nullptr, p.S, ev0.nb, X, tw)
                       : launch_spectrum<float, T>(p.N, st, (const float*)d_volt, ev0, nullptr, nullptr, p.S, ev0.nb, X, tw);
    if (e != hipSuccess) return fail(AU_EDEVICE, std::string("k_spectrum: ") + hipGetErrorString(e));
    const double dt_ns = 1e9 / (double)ev->fs_hz;
    int64_t off = 0;
    for (int lv = 0; lv <= levels; ++lv) {
        const int nc = lv == 0 ? n_dir : k * k;
        const int spw = env_spw(p.S, nc);
        const int chunks = (p.S + spw - 1) / spw;
        double* cand = dirs + 2 * off;
        ev0.D = nc;
        if (tb->dtype == AU_F64)
            launch_coef<double, T>(st, tb, ev0, nullptr, nullptr, nc, cand, 0, 0, ev->fs_hz, ev->fallback_rel,
                                   ev->singular_rel, M, nullptr);
        else
            launch_coef<float, T>(st, tb, ev0, nullptr, nullptr, nc, cand, 0, 0, ev->fs_hz, ev->fallback_rel,
                                  ev->singular_rel, M, nullptr);
        switch (p.N) {
#define X_(NN)                                                                                       \
    case NN:                                                                                         \
        e = launch_env_n<T, NN>(st, ev0, spw, nc * chunks, X, M, (T*)nullptr, peak, arg, tw, nullptr,   \
                                nullptr, nullptr, 0, true);                                          \
        break;
            AU_FOR_EACH_N(X_)
#undef X_
            default: e = hipErrorInvalidValue;
        }
        if (e != hipSuccess) return fail(AU_EDEVICE, std::string("direction fit scan: ") + hipGetErrorString(e));
        hipLaunchKernelGGL(k_dir_score<T>, dim3(nc), dim3(kBlock), 0, st, p.S, (const double*)pos,
                           (const double*)cand, (const int*)arg, (const T*)peak, dt_ns, chi2 + off, power + off);
        const double sc = std::ldexp(1.0, -(lv + 1));
        hipLaunchKernelGGL(k_dir_best, dim3(1), dim3(kBlock), 0, st, nc, (const double*)(chi2 + off),
                           (const double*)cand, best + lv, result, step_zen * sc, step_az * sc, k,
                           lv < levels ? dirs + 2 * (off + nc) : nullptr);
        e = hipGetLastError();
        if (e != hipSuccess) return fail(AU_EDEVICE, std::string("direction fit score: ") + hipGetErrorString(e));
        off += nc;
    }
    if (levels > 0 && h_level_dirs)
        HIP_TRY(hipMemcpyAsync(h_level_dirs, dirs + 2 * n_dir, sizeof(double) * 2 * (size_t)levels * k * k,
                               hipMemcpyDeviceToHost, st));
    if (h_chi2) HIP_TRY(hipMemcpyAsync(h_chi2, chi2, sizeof(double) * f.n_cand, hipMemcpyDeviceToHost, st));
    if (h_power) HIP_TRY(hipMemcpyAsync(h_power, power, sizeof(double) * f.n_cand, hipMemcpyDeviceToHost, st));
    if (h_best) HIP_TRY(hipMemcpyAsync(h_best, best, sizeof(int32_t) * (levels + 1), hipMemcpyDeviceToHost, st));
    HIP_TRY(hipMemcpyAsync(h_result, result, sizeof(double) * 2, hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    return AU_OK;
}

extern "C" au_status au_direction_fit_workspace_bytes(const au_table* tb, const au_event* ev, int32_t n_dir,
                                                      int32_t levels, int32_t k, uint64_t* bytes)
{
    if (!bytes) return fail(AU_EINVAL, "null argument");
    EvParams p;
    au_status s = check_fit(tb, ev, n_dir, levels, k, 1.0, 1.0, &p);
    if (s != AU_OK) return s;
    *bytes = fit_layout(p, ev->prec, n_dir, levels, k).total;
    return AU_OK;
}

extern "C" au_status au_direction_fit(const au_table* tb, const au_event* ev, const void* d_volt, const double* h_pos,
                                      int32_t n_dir, const double* h_dirs, int32_t levels, int32_t k,
                                      double step_zen, double step_az, double* h_level_dirs, double* h_chi2,
                                      double* h_power, int32_t* h_best, double* h_result, void* d_work,
                                      uint64_t work_bytes, void* stream)
{
    EvParams p;
    au_status s = check_fit(tb, ev, n_dir, levels, k, step_zen, step_az, &p);
    if (s != AU_OK) return s;
    if (!d_volt || !h_pos || !h_dirs || !h_result) return fail(AU_EINVAL, "null argument");
    if (!dirs_finite(h_dirs, n_dir)) return fail(AU_EINVAL, "directions must be finite");
    for (int64_t i = 0; i < 2 * (int64_t)p.S; ++i)
        if (!std::isfinite(h_pos[i]) || std::fabs(h_pos[i]) > 1e7)
            return fail(AU_EINVAL, "station positions must be finite and within 1e7 m");
    int dev = 0;
    HIP_TRY(hipGetDevice(&dev));
    if (dev != tb->device) return fail(AU_EINVAL, "table lives on another device");
    const FitLayout f = fit_layout(p, ev->prec, n_dir, levels, k);
    hipStream_t st = (hipStream_t)stream;
    void* work = d_work;
    bool pooled = false;
    if (work == nullptr) {
        hipError_t e = hipMallocAsync(&work, f.total, st);
        if (e != hipSuccess) return fail(AU_ENOMEM, std::string("hipMallocAsync: ") + hipGetErrorString(e));
        pooled = true;
    } else if (work_bytes < f.total) {
        return fail(AU_ENOMEM, "workspace smaller than au_direction_fit_workspace_bytes");
    }
    s = ev->prec == AU_PREC_FP64
            ? run_fit<double>(tb, ev, p, d_volt, h_pos, n_dir, h_dirs, levels, k, step_zen, step_az, work, st,
                              h_level_dirs, h_chi2, h_power, h_best, h_result)
            : run_fit<float>(tb, ev, p, d_volt, h_pos, n_dir, h_dirs, levels, k, step_zen, step_az, work, st,
                             h_level_dirs, h_chi2, h_power, h_best, h_result);
    if (pooled) {
        hipError_t e = hipFreeAsync(work, st);
        if (s == AU_OK && e != hipSuccess)
            return fail(AU_EDEVICE, std::string("hipFreeAsync: ") + hipGetErrorString(e));
    }
    return s;
}

// ---------------------------------------------------------------------------
// the reconstruction loop over many events at once: every step is one launch
// over all events (per-event stop flags), so the per-event launch and
// synchronisation costs of the one-event form are paid once per batch
// ---------------------------------------------------------------------------

namespace {

struct BatchReconLayout {
    size_t x, m, hist, dirs, cur, state, pos, peak, arg, evs, sunits, cunits, eunits, evst, total;
};

BatchReconLayout batch_recon_layout(int prec, int64_t stot, int n_events, int nb, int max_iter, int64_t n_eunits)
{
    const size_t tsz = prec == AU_PREC_FP64 ? sizeof(double) : sizeof(float);
    BatchReconLayout r;
    r.x = align256((size_t)stot * nb * 4 * tsz + 1);
    r.m = align256((size_t)n_events * nb * 8 * tsz + 1);
    r.hist = align256((size_t)(max_iter + 1) * stot * sizeof(int32_t));
    r.dirs = align256((size_t)n_events * max_iter * 2 * sizeof(double));
    r.cur = align256((size_t)n_events * 2 * sizeof(double));
    r.state = align256((size_t)n_events * 4 * sizeof(int32_t));
    r.pos = align256((size_t)stot * 2 * sizeof(double));
    r.peak = align256((size_t)stot * 3 * tsz);
    r.arg = align256((size_t)stot * 3 * sizeof(int32_t));
    r.evs = align256((size_t)n_events * sizeof(EvDesc));
    r.sunits = align256((size_t)stot * sizeof(int2));
    r.cunits = align256((size_t)n_events * sizeof(int2));
    r.eunits = align256((size_t)n_eunits * sizeof(int4));
    r.evst = align256((size_t)n_events * sizeof(int2));
    r.total = r.x + r.m + r.hist + r.dirs + r.cur + r.state + r.pos + r.peak + r.arg + r.evs + r.sunits +
              r.cunits + r.eunits + r.evst;
    return r;
}

// Validates the batch; fills p (common sizes, S = the largest event), the
// station total and the envelope unit count for its stations-per-workgroup.
au_status check_recon_batch(const au_table* tb, const au_event* ev, int32_t n_events, const int32_t* h_ns,
                            const int64_t* h_voff, int32_t max_iter, EvParams* p, int64_t* stot, int* spw,
                            int64_t* n_eunits)
{
    if (!ev || !h_ns || !h_voff) return fail(AU_EINVAL, "null argument");
    if (n_events < 1) return fail(AU_EINVAL, "n_events must be >= 1");
    if (max_iter < 1 || max_iter > kMaxReconIter) return fail(AU_EINVAL, "max_iter must be in [1, 1024]");
    int smax = 0;
    int64_t tot = 0;
    for (int32_t e = 0; e < n_events; ++e) {
        if (h_ns[e] < 3) return fail(AU_EINVAL, "every event needs at least 3 stations");
        if (h_voff[e] < 0) return fail(AU_EINVAL, "negative trace offset");
        smax = std::max(smax, (int)h_ns[e]);
        tot += h_ns[e];
    }
    if (tot > (int64_t)0x7fffffff / 4) return fail(AU_EINVAL, "too many stations");
    au_event e1 = *ev;
    e1.n_stations = smax;
    au_status s = check_event(tb, &e1, p);
    if (s != AU_OK) return s;
    *stot = tot;
    *spw = env_spw((int)std::min<int64_t>(tot, 0x7fffffff), 1);
    int64_t nu = 0;
    for (int32_t e = 0; e < n_events; ++e) nu += (h_ns[e] + *spw - 1) / *spw;
    *n_eunits = nu;
    return AU_OK;
}

}  // namespace

template <typename T>
static au_status run_reconstruct_batch(const au_table* tb, const au_event* ev, const EvParams& p, int32_t n_events,
                                       const int32_t* h_ns, const int64_t* h_voff, const void* d_volt,
                                       const double* h_pos, int max_iter, int64_t stot, int spw, int64_t n_eunits,
                                       void* d_work, hipStream_t st, double* h_dirs, int32_t* h_times,
                                       int32_t* h_n_dirs, int32_t* h_converged)
{
    const BatchReconLayout r = batch_recon_layout(ev->prec, stot, n_events, p.nb, max_iter, n_eunits);
    unsigned char* q = (unsigned char*)d_work;
    XBin<T>* X = (XBin<T>*)q;
    MBin<T>* M = (MBin<T>*)(q += r.x);
    int* hist = (int*)(q += r.m);
    double* dirs = (double*)(q += r.hist);
    double* cur = (double*)(q += r.dirs);
    int* state = (int*)(q += r.cur);
    double* pos = (double*)(q += r.state);
    T* peak = (T*)(q += r.pos);
    int* arg = (int*)(q += r.peak);
    EvDesc* evs = (EvDesc*)(q += r.arg);
    int2* sunits = (int2*)(q += r.evs);
    int2* cunits = (int2*)(q += r.sunits);
    int4* eunits = (int4*)(q += r.cunits);
    int2* evst = (int2*)(q += r.eunits);
    // descriptors, built on the host and copied once
    std::vector<EvDesc> hevs((size_t)n_events);
    std::vector<int2> hsu((size_t)stot), hcu((size_t)n_events), hst((size_t)n_events);
    std::vector<int4> heu;
    heu.reserve((size_t)n_eunits);
    int64_t so = 0;
    for (int32_t e = 0; e < n_events; ++e) {
        EvDesc d{};
        d.volt_off = h_voff[e];
        d.efield_off = 3 * so;  // the event's [1][S][3] peak and sample block
        d.x_off = so * p.nb;
        d.m_off = (int64_t)e * p.nb;
        d.dir_off = e;
        d.S = h_ns[e];
        d.N = p.N;
        d.D = 1;
        d.k_lo = p.k_lo;
        d.nb = p.nb;
        hevs[(size_t)e] = d;
        for (int s = 0; s < h_ns[e]; ++s) hsu[(size_t)(so + s)] = int2{e, s};
        for (int s0 = 0; s0 < h_ns[e]; s0 += spw) heu.push_back(int4{e, 0, s0, std::min((int)h_ns[e], s0 + spw)});
        hcu[(size_t)e] = int2{e, 0};
        hst[(size_t)e] = int2{(int)so, h_ns[e]};
        so += h_ns[e];
    }
    HIP_TRY(hipMemcpyAsync(evs, hevs.data(), hevs.size() * sizeof(EvDesc), hipMemcpyHostToDevice, st));
    HIP_TRY(hipMemcpyAsync(sunits, hsu.data(), hsu.size() * sizeof(int2), hipMemcpyHostToDevice, st));
    HIP_TRY(hipMemcpyAsync(cunits, hcu.data(), hcu.size() * sizeof(int2), hipMemcpyHostToDevice, st));
    HIP_TRY(hipMemcpyAsync(eunits, heu.data(), heu.size() * sizeof(int4), hipMemcpyHostToDevice, st));
    HIP_TRY(hipMemcpyAsync(evst, hst.data(), hst.size() * sizeof(int2), hipMemcpyHostToDevice, st));
    HIP_TRY(hipMemcpyAsync(pos, h_pos, sizeof(double) * 2 * stot, hipMemcpyHostToDevice, st));
    // (each event's state is cleared by its first step)
    EvDesc ev0{};
    ev0.N = p.N;
    ev0.k_lo = p.k_lo;
    ev0.nb = p.nb;
    const C2<T>* tw = twiddles<T>(tb->device);
    if (tw == nullptr) return fail(AU_EDEVICE, "twiddle tables missing on this device");
    hipError_t e;
    if (ev->trace_dtype == AU_F64) {
        e = launch_spectrum<double, T>(p.N, st, (const double*)d_volt, ev0, evs, sunits, (int)stot, p.nb, X, tw);
        hipLaunchKernelGGL(k_volt_timing<double>, dim3((unsigned)stot), dim3(kBlock), 0, st, (const double*)d_volt,
                           p.N, hist, (const EvDesc*)evs, (const int2*)sunits);
    } else {
        e = launch_spectrum<float, T>(p.N, st, (const float*)d_volt, ev0, evs, sunits, (int)stot, p.nb, X, tw);
        hipLaunchKernelGGL(k_volt_timing<float>, dim3((unsigned)stot), dim3(kBlock), 0, st, (const float*)d_volt,
                           p.N, hist, (const EvDesc*)evs, (const int2*)sunits);
    }
    if (e == hipSuccess) e = hipGetLastError();
    if (e != hipSuccess) return fail(AU_EDEVICE, std::string("spectrum/timing: ") + hipGetErrorString(e));
    const double dt_ns = 1e9 / (double)ev->fs_hz;
    for (int it = 0; it <= max_iter; ++it) {
        const int last = it == max_iter;
        hipLaunchKernelGGL(k_recon_step, dim3(n_events), dim3(kBlock), 0, st, it, last, 0, dt_ns, (const double*)pos,
                           (const int*)arg, hist, dirs, cur, state, (const int2*)evst, (int)stot, max_iter);
        if (last) break;
        if (tb->dtype == AU_F64)
            launch_coef<double, T>(st, tb, ev0, evs, cunits, n_events, cur, 0, 0, ev->fs_hz, ev->fallback_rel,
                                   ev->singular_rel, M, nullptr, (const int*)state, 4);
        else
            launch_coef<float, T>(st, tb, ev0, evs, cunits, n_events, cur, 0, 0, ev->fs_hz, ev->fallback_rel,
                                  ev->singular_rel, M, nullptr, (const int*)state, 4);
        switch (p.N) {
#define X_(NN)                                                                                          \
    case NN:                                                                                            \
        e = launch_env_n<T, NN>(st, ev0, spw, (int)n_eunits, X, M, (T*)nullptr, peak, arg, tw,          \
                                (const int*)state, (const EvDesc*)evs, (const int4*)eunits, 4, true);   \
        break;
            AU_FOR_EACH_N(X_)
#undef X_
            default: e = hipErrorInvalidValue;
        }
        if (e != hipSuccess) return fail(AU_EDEVICE, std::string("reconstruction step: ") + hipGetErrorString(e));
    }
    std::vector<int32_t> hstate((size_t)n_events * 4);
    HIP_TRY(hipMemcpyAsync(hstate.data(), state, sizeof(int32_t) * 4 * n_events, hipMemcpyDeviceToHost, st));
    HIP_TRY(hipMemcpyAsync(h_dirs, dirs, sizeof(double) * 2 * max_iter * (size_t)n_events, hipMemcpyDeviceToHost,
                           st));
    HIP_TRY(hipMemcpyAsync(h_times, hist, sizeof(int32_t) * (size_t)(max_iter + 1) * stot, hipMemcpyDeviceToHost,
                           st));
    HIP_TRY(hipStreamSynchronize(st));
    for (int32_t k = 0; k < n_events; ++k) {
        h_n_dirs[k] = hstate[4 * (size_t)k + 1];
        h_converged[k] = hstate[4 * (size_t)k + 3] ? -1 : hstate[4 * (size_t)k + 2];
    }
    return AU_OK;
}

extern "C" au_status au_reconstruct_batch_workspace_bytes(const au_table* tb, const au_event* ev, int32_t n_events,
                                                          const int32_t* h_n_stations, const int64_t* h_volt_offset,
                                                          int32_t max_iter, uint64_t* bytes)
{
    if (!bytes) return fail(AU_EINVAL, "null argument");
    EvParams p;
    int64_t stot = 0, nu = 0;
    int spw = 1;
    au_status s = check_recon_batch(tb, ev, n_events, h_n_stations, h_volt_offset, max_iter, &p, &stot, &spw, &nu);
    if (s != AU_OK) return s;
    *bytes = batch_recon_layout(ev->prec, stot, n_events, p.nb, max_iter, nu).total;
    return AU_OK;
}

extern "C" au_status au_reconstruct_batch(const au_table* tb, const au_event* ev, int32_t n_events,
                                          const int32_t* h_n_stations, const int64_t* h_volt_offset,
                                          const void* d_volt, const double* h_pos, int32_t max_iter,
                                          double* h_dirs, int32_t* h_times, int32_t* h_n_dirs,
                                          int32_t* h_converged, void* d_work, uint64_t work_bytes, void* stream)
{
    EvParams p;
    int64_t stot = 0, nu = 0;
    int spw = 1;
    au_status s = check_recon_batch(tb, ev, n_events, h_n_stations, h_volt_offset, max_iter, &p, &stot, &spw, &nu);
    if (s != AU_OK) return s;
    if (!d_volt || !h_pos || !h_dirs || !h_times || !h_n_dirs || !h_converged) return fail(AU_EINVAL, "null argument");
    for (int64_t i = 0; i < 2 * stot; ++i)
        if (!std::isfinite(h_pos[i]) || std::fabs(h_pos[i]) > 1e7)
            return fail(AU_EINVAL, "station positions must be finite and within 1e7 m");
    int dev = 0;
    HIP_TRY(hipGetDevice(&dev));
    if (dev != tb->device) return fail(AU_EINVAL, "table lives on another device");
    const BatchReconLayout r = batch_recon_layout(ev->prec, stot, n_events, p.nb, max_iter, nu);
    hipStream_t st = (hipStream_t)stream;
    void* work = d_work;
    bool pooled = false;
    if (work == nullptr) {
        hipError_t e = hipMallocAsync(&work, r.total, st);
        if (e != hipSuccess) return fail(AU_ENOMEM, std::string("hipMallocAsync: ") + hipGetErrorString(e));
        pooled = true;
    } else if (work_bytes < r.total) {
        return fail(AU_ENOMEM, "workspace smaller than au_reconstruct_batch_workspace_bytes");
    }
    s = ev->prec == AU_PREC_FP64
            ? run_reconstruct_batch<double>(tb, ev, p, n_events, h_n_stations, h_volt_offset, d_volt, h_pos,
                                            max_iter, stot, spw, nu, work, st, h_dirs, h_times, h_n_dirs,
                                            h_converged)
            : run_reconstruct_batch<float>(tb, ev, p, n_events, h_n_stations, h_volt_offset, d_volt, h_pos,
                                           max_iter, stot, spw, nu, work, st, h_dirs, h_times, h_n_dirs,
                                           h_converged);
    if (pooled) {
        hipError_t e = hipFreeAsync(work, st);
        if (s == AU_OK && e != hipSuccess)
            return fail(AU_EDEVICE, std::string("hipFreeAsync: ") + hipGetErrorString(e));
    }
    return s;
}
