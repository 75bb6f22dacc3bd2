// au_device.h -- device building blocks for gfx950: complex arithmetic,
// in-register small DFTs and a Stockham FFT whose passes exchange data
// through LDS.
//
// The FFT replaces the library FFT calls of the original reconstruction
// (arXiv:1507.07733, section 4) with a transform that lives entirely inside
// one workgroup: an N-point transform is spread over N/E threads, each
// holding E complex values in registers.  A pass of radix R (R divides E)
// has every thread run E/R radix-R butterflies on values it already holds;
// between passes the values are exchanged through LDS.  With the Stockham
// (self-sorting) ordering, thread t always holds elements t + (N/E)*i of the
// current sequence, so the first pass reads its inputs straight from
// registers and the last pass leaves the result in natural order in the
// same layout -- loads and stores of whole traces are fully coalesced and
// only passes-1 LDS round trips are needed.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace au {

template <typename T>
struct alignas(2 * sizeof(T)) C2 {
    T re, im;
};

template <typename T>
__device__ __forceinline__ C2<T> cadd(C2<T> a, C2<T> b) { return {a.re + b.re, a.im + b.im}; }
template <typename T>
__device__ __forceinline__ C2<T> csub(C2<T> a, C2<T> b) { return {a.re - b.re, a.im - b.im}; }
template <typename T>
__device__ __forceinline__ C2<T> cmul(C2<T> a, C2<T> b)
{
    return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};
}
template <typename T>
__device__ __forceinline__ C2<T> cconj(C2<T> a) { return {a.re, -a.im}; }
// a * (SIGN * i)
template <int SIGN, typename T>
__device__ __forceinline__ C2<T> cmul_si(C2<T> a)
{
    return SIGN > 0 ? C2<T>{-a.im, a.re} : C2<T>{a.im, -a.re};
}

// cos(2 pi m / 32) for m = 0..8 (first quadrant), from the half-angle closed
// forms cos(pi/4) = sqrt(2)/2, cos(x/2) = sqrt((1 + cos x) / 2).
__device__ constexpr double kQuadCos32[9] = {
    1.0,
    0.980785280403230449126182236134239037,
    0.923879532511286756128183189396788287,
    0.831469612302545237078788377617905757,
    0.707106781186547524400844362104849039,
    0.555570233019602224742830813948532874,
    0.382683432365089771728459984030398867,
    0.195090322016128267848284868477022241,
    0.0,
};

// exp(SIGN * 2 pi i * m / 32) for a compile-time-foldable m in [0, 32).
template <int SIGN>
__device__ __forceinline__ constexpr void root32(int m, double& c, double& s)
{
    const int q = (m >> 3) & 3, r = m & 7;
    const double c0 = kQuadCos32[r], s0 = kQuadCos32[8 - r];
    double cc = c0, ss = s0;
    if (q == 1) { cc = -s0; ss = c0; }
    if (q == 2) { cc = -c0; ss = -s0; }
    if (q == 3) { cc = s0; ss = -c0; }
    c = cc;
    s = SIGN > 0 ? ss : -ss;
}

// x * exp(SIGN * 2 pi i k / R), R <= 32, k a constant after unrolling.
template <int R, int SIGN, typename T>
__device__ __forceinline__ C2<T> twiddle_const(int k, C2<T> x)
{
    const int m = (k * (32 / R)) & 31;
    if (m == 0) return x;
    if (m == 8) return cmul_si<SIGN>(x);
    if (m == 16) return C2<T>{-x.re, -x.im};
    if (m == 24) return cmul_si<-SIGN>(x);
    double c, s;
    root32<SIGN>(m, c, s);
    return cmul(x, C2<T>{(T)c, (T)s});
}

// In-register DFT of size R (power of two, <= 32):
//   v[k] <- sum_n v[n] exp(SIGN 2 pi i n k / R)
// by radix-2 decimation in time down to a radix-4 base case.
template <int R, int SIGN, typename T>
struct Dft {
    static __device__ __forceinline__ void run(C2<T>* v)
    {
        C2<T> a[R / 2], b[R / 2];
#pragma unroll
        for (int i = 0; i < R / 2; ++i) {
            a[i] = v[2 * i];
            b[i] = v[2 * i + 1];
        }
        Dft<R / 2, SIGN, T>::run(a);
        Dft<R / 2, SIGN, T>::run(b);
#pragma unroll
        for (int k = 0; k < R / 2; ++k) {
            const C2<T> t = twiddle_const<R, SIGN>(k, b[k]);
            v[k] = cadd(a[k], t);
            v[k + R / 2] = csub(a[k], t);
        }
    }
};

template <int SIGN, typename T>
struct Dft<4, SIGN, T> {
    static __device__ __forceinline__ void run(C2<T>* v)
    {
        const C2<T> t0 = cadd(v[0], v[2]);
        const C2<T> t1 = csub(v[0], v[2]);
        const C2<T> t2 = cadd(v[1], v[3]);
        const C2<T> t3 = cmul_si<SIGN>(csub(v[1], v[3]));
        v[0] = cadd(t0, t2);
        v[2] = csub(t0, t2);
        v[1] = cadd(t1, t3);
        v[3] = csub(t1, t3);
    }
};

template <int SIGN, typename T>
struct Dft<2, SIGN, T> {
    static __device__ __forceinline__ void run(C2<T>* v)
    {
        const C2<T> a = v[0], b = v[1];
        v[0] = cadd(a, b);
        v[1] = csub(a, b);
    }
};

template <int SIGN, typename T>
struct Dft<1, SIGN, T> {
    static __device__ __forceinline__ void run(C2<T>*) {}
};

// Fused multiply-add butterflies (the tangent form of Linzer and Feig,
// "Modified FFTs for fused multiply-add architectures", Math. Comp. 60,
// 1993).  With a twiddle w = c (1 + i t),
//   a +- rot w b = a +- c rot u,   u = b (1 + i t) = (b.re - t b.im, b.im + t b.re),
// two FMAs give u and one FMA each output component: 6 operations where a
// complex multiply and two complex additions take 8.  rot is 1, +i or -i
// (ROT 0, +1, -1), an exchange of components that costs nothing.  A cosine
// that is exactly zero (+-90 deg) is stored as 2^-40 (float) or 2^-90
// (double): c u then differs from the exact product by that fraction of
// |b.re|, far below the rounding of the result, and t stays finite (the
// rounding of u, of relative size u (1 + |t|) |b|, shrinks by |c| in c u,
// so the tangent's size costs no accuracy).
// Leaves a + rot w b in a and a - rot w b in b.
template <int ROT, typename T>
__device__ __forceinline__ void lf_pair(C2<T>& a, C2<T>& b, const C2<T> tc)
{
    const T t = tc.re, c = tc.im;
    const T ur = fma(-t, b.im, b.re);
    const T ui = fma(t, b.re, b.im);
    const T pr = ROT == 0 ? ur : (ROT > 0 ? -ui : ui);
    const T pi = ROT == 0 ? ui : (ROT > 0 ? ur : -ur);
    const C2<T> hi{fma(c, pr, a.re), fma(c, pi, a.im)};
    const C2<T> lo{fma(-c, pr, a.re), fma(-c, pi, a.im)};
    a = hi;
    b = lo;
}

// Radix-R butterfly of a Stockham pass with its input twiddles w^r (w =
// exp(SIGN 2 pi i k / (NS R))) folded in:
//   v[q] <- sum_r v[r] w^r exp(SIGN 2 pi i r q / R),
// with L the (tangent, cosine) pairs of w (R = 2); w, w^2 (R = 4); w, w^2,
// w^4 and w exp(SIGN i pi / 4) (R = 8).  Split r = r1 + (R/2) r2: the first
// radix-2 stage pairs v[r1] with v[r1 + R/2] through w^(R/2); the sums feed
// the even outputs as an R/2-point transform twiddled by w, the differences
// the odd outputs as one twiddled by w exp(SIGN 2 pi i / R); inside the
// 4-point transforms the factors SIGN i of exp(SIGN 2 pi i / 4) are
// exchanges of components (ROT).  72 operations for R = 8 against 82 for
// seven complex multiplies and an 8-point transform.
template <int R, int SIGN, typename T>
__device__ __forceinline__ void lf_dft(C2<T>* v, const C2<T>* L)
{
    static_assert(R == 2 || R == 4 || R == 8, "fused multiply-add butterflies: radix 2, 4 or 8");
    if constexpr (R == 2) {
        lf_pair<0>(v[0], v[1], L[0]);
    } else if constexpr (R == 4) {
        lf_pair<0>(v[0], v[2], L[1]);
        lf_pair<0>(v[1], v[3], L[1]);
        lf_pair<0>(v[0], v[1], L[0]);
        lf_pair<SIGN>(v[2], v[3], L[0]);
        const C2<T> y1 = v[2], y2 = v[1];
        v[1] = y1;
        v[2] = y2;
    } else {
#pragma unroll
        for (int r = 0; r < 4; ++r) lf_pair<0>(v[r], v[r + 4], L[2]);
        // even outputs: 4-point transform of the sums, twiddle w
        lf_pair<0>(v[0], v[2], L[1]);
        lf_pair<0>(v[1], v[3], L[1]);
        lf_pair<0>(v[0], v[1], L[0]);
        lf_pair<SIGN>(v[2], v[3], L[0]);
        // odd outputs: of the differences, twiddle w exp(SIGN i pi / 4), whose
        // square is (SIGN i) w^2
        lf_pair<SIGN>(v[4], v[6], L[1]);
        lf_pair<SIGN>(v[5], v[7], L[1]);
        lf_pair<0>(v[4], v[5], L[3]);
        lf_pair<SIGN>(v[6], v[7], L[3]);
        const C2<T> y[8] = {v[0], v[4], v[2], v[6], v[1], v[5], v[3], v[7]};
#pragma unroll
        for (int q = 0; q < 8; ++q) v[q] = y[q];
    }
}

// Twiddle table: tw[q] = exp(-2 pi i q / kTwN), q in [0, kTwN).  Any
// N-point transform with N | kTwN indexes it with stride kTwN / N.
constexpr int kTwN = 4096;

template <int SIGN, typename T>
__device__ __forceinline__ C2<T> twiddle_tab(const C2<T>* __restrict__ tw, int q)
{
    const C2<T> w = tw[q];
    return SIGN < 0 ? w : cconj(w);
}

// ---------------------------------------------------------------------------
// Compile-time roots of unity: exp(2 pi i p / q) for integers p, q.  The
// turn fraction is reduced exactly to a quadrant and then to [0, pi/4], where
// the Taylor series of sin and cos converge to double precision in 14 terms.
// ---------------------------------------------------------------------------
struct CxRoot {
    double c, s;
};

constexpr double cx_half_pi = 1.57079632679489661923132169163975144;

constexpr double cx_sin_series(double x)
{
    double term = x, sum = x;
    for (int n = 1; n < 14; ++n) {
        term *= -x * x / (double)((2 * n) * (2 * n + 1));
        sum += term;
    }
    return sum;
}

constexpr double cx_cos_series(double x)
{
    double term = 1.0, sum = 1.0;
    for (int n = 1; n < 14; ++n) {
        term *= -x * x / (double)((2 * n - 1) * (2 * n));
        sum += term;
    }
    return sum;
}

constexpr CxRoot cx_root(long long p, long long q)
{
    p %= q;
    if (p < 0) p += q;
    const long long quad = (4 * p) / q;       // quarter turns
    const long long rem = 4 * p - quad * q;   // remaining angle = (pi/2) rem / q
    double c0 = 1.0, s0 = 0.0;
    if (2 * rem <= q) {
        const double x = cx_half_pi * (double)rem / (double)q;
        c0 = cx_cos_series(x);
        s0 = cx_sin_series(x);
    } else {
        const double x = cx_half_pi * (double)(q - rem) / (double)q;
        c0 = cx_sin_series(x);
        s0 = cx_cos_series(x);
    }
    if (rem == 0) {
        c0 = 1.0;
        s0 = 0.0;
    }
    switch (quad & 3) {
        case 0: return CxRoot{c0, s0};
        case 1: return CxRoot{-s0, c0};
        case 2: return CxRoot{-c0, -s0};
        default: return CxRoot{s0, -c0};
    }
}

// s_waitcnt vmcnt(0) (expcnt and lgkmcnt left alone): every vector-memory
// operation issued so far has completed.
__device__ __forceinline__ void vmem_wait_all() { __builtin_amdgcn_s_waitcnt(0x0F70); }

// LDS slot of sequence element i, an XOR swizzle of the low index bits (a
// permutation of every aligned block of 16 or 8 elements) chosen per
// element size.  Measured on gfx950: a wave's 8-byte reads are served 32
// lanes per cycle from 64 four-byte banks and its 8-byte writes 16 lanes per
// cycle from 32 banks; its 16-byte writes 8 lanes per cycle from 32 banks,
// and its 16-byte reads about 16 lanes per cycle from 64 banks.  Under those
// models the layouts keep the gathers (consecutive elements) and the radix-8
// scatters (lane strides of 8 and 64 elements) nearly free of bank
// conflicts: 8-byte (complex float) elements XOR bits 0-3 with bits 4-7 and
// bit 3 with bit 6; 16-byte (complex double) elements XOR bits 0-2 with bits
// 3-5 and with bits 4-6.  (One pad slot per 16 elements left the gathers and
// the stride-8 scatters two-way conflicted: LDS cycles per FFT -35 % for
// complex float at N = 4096, 8 values per thread.)
template <typename T>
__device__ __forceinline__ constexpr int lpad(int i)
{
    if constexpr (sizeof(T) == 8)
        return i ^ ((i >> 3) & 7) ^ ((i >> 4) & 7);
    else
        return i ^ ((i >> 4) & 15) ^ (((i >> 6) & 1) << 3);
}

// Elements per LDS buffer: the N slots of the sequence plus 16 spare ones
// (lds_pad_slot, lds_zero_slot) that no transform touches.
template <int N>
constexpr int lds_elems() { return N + 16; }
template <int N>
constexpr int lds_pad_slot() { return N; }
template <int N>
constexpr int lds_zero_slot() { return N + 1; }

// ---------------------------------------------------------------------------
// Pass structure.  An N-point transform runs on TT = N/E threads holding E
// values each; the pass that starts from completed sub-transforms of length
// NS has radix R = min(RMAX, N/NS), and each thread runs B = E/R of its
// butterflies (butterfly j = t + TT m, m < B).
//
// Twiddle modes (the pass multiplies input r of butterfly j by
// exp(SIGN 2 pi i r k / (NS R)), k = j mod NS):
//   TW_TABLE: read from the table each time.
//   TW_REG:   every (m, r) factor of every pass in registers, loaded once.
//   TW_SPLIT: R-1 registers per pass.  If NS <= TT then k = t mod NS for
//             every m and the registers hold the factors themselves; if
//             NS > TT then k = t + (TT m mod NS) and the factor splits into
//             exp(SIGN 2 pi i r t / (NS R)) (register) times
//             exp(SIGN 2 pi i r (TT m mod NS) / (NS R)) (compile-time
//             constant).
// ---------------------------------------------------------------------------
//   TW_HYB:   passes with NS < TT (k = t mod NS for every m: only NS
//             distinct factors sets) read them from a per-workgroup LDS
//             table of NS (R-1) entries per pass; the passes with NS >= TT
//             keep theirs in registers as TW_REG.  Saves the registers of
//             the early passes for one LDS read per factor.
//   TW_LF:    TW_HYB's placement (an LDS table for NS < TT, registers for
//             NS >= TT) for the fused multiply-add butterflies of lf_dft:
//             per (pass, k) the (tangent, cosine) pairs of the angles the
//             radix-R butterfly needs (lf_entries) instead of R-1 roots.
//   TW_LFR:   the TW_LF pairs of every pass in registers (no LDS table
//             reads: for shapes with registers to spare whose transform is
//             bound by LDS bandwidth, as FP64 at one workgroup per CU).
//   TW_LFW:   TW_LFR's twiddles and butterflies in the 4096-point
//             transform whose first two exchanges stay inside the
//             wavefront (fft4096_xw): one through the wavefront's own LDS
//             slots with no workgroup barrier, one as a register transpose;
//             one workgroup exchange per transform instead of three.
enum { TW_TABLE = 0, TW_REG = 1, TW_SPLIT = 2, TW_HYB = 3, TW_LF = 4, TW_LFR = 5, TW_LFW = 6 };

// Twiddles of the early passes in a per-workgroup LDS table.
constexpr bool tw_lds_early(int mode) { return mode == TW_HYB || mode == TW_LF; }
// Fused multiply-add butterflies with (tangent, cosine) twiddle pairs.
constexpr bool tw_lf(int mode) { return mode == TW_LF || mode == TW_LFR || mode == TW_LFW; }
// Every pass's twiddles in registers.
constexpr bool tw_all_reg(int mode) { return mode == TW_REG || mode == TW_LFR || mode == TW_LFW; }
// (tangent, cosine) pairs per butterfly of a radix-R pass in TW_LF, TW_LFR, TW_LFW.
constexpr int lf_entries(int r) { return r == 8 ? 4 : (r == 4 ? 2 : 1); }
// Twiddle entries per butterfly of a radix-R pass.
constexpr int tw_per(int mode, int r) { return tw_lf(mode) ? lf_entries(r) : r - 1; }

template <int N, int RMAX>
constexpr int pass_radix(int ns) { return (N / ns < RMAX) ? N / ns : RMAX; }

template <int N, int E, int RMAX, int TWMODE>
constexpr int tw_offset(int ns_target)
{
    int off = 0;
    for (int ns = 1; ns < ns_target && ns < N; ns *= pass_radix<N, RMAX>(ns)) {
        if (ns == 1) continue;
        const int r = pass_radix<N, RMAX>(ns);
        if (tw_lds_early(TWMODE) && ns < N / E) continue;
        off += (tw_all_reg(TWMODE) || tw_lds_early(TWMODE)) ? (E / r) * tw_per(TWMODE, r) : (r - 1);
    }
    return off;
}

// Offset of pass NS in the TW_HYB / TW_LF LDS table, and the table's length.
template <int N, int E, int RMAX, int TWMODE = TW_HYB>
constexpr int ltw_offset(int ns_target)
{
    int off = 0;
    for (int ns = 1; ns < ns_target && ns < N; ns *= pass_radix<N, RMAX>(ns)) {
        if (ns == 1) continue;
        if (ns >= N / E) break;
        off += ns * tw_per(TWMODE, pass_radix<N, RMAX>(ns));
    }
    return off;
}
template <int N, int E, int RMAX, int TWMODE = TW_HYB>
constexpr int ltw_count()
{
    return ltw_offset<N, E, RMAX, TWMODE>(N);
}

// The fused multiply-add twiddle table follows the kTwN roots in the same
// allocation: entry 4 q + e (q < kTwN / 2) holds (tan a_e, cos a_e) for the
// angles a_0 = 2 pi q / kTwN, a_1 = 2 a_0, a_2 = 4 a_0, a_3 = a_0 + pi / 4
// (exp(+i ...) convention; a cosine that is exactly zero is stored as a tiny
// value of its sign, see lf_pair).  For the exp(-i ...) transform every
// tangent changes sign.
constexpr int kLfQ = 2048;
template <int SIGN, typename T>
__device__ __forceinline__ C2<T> lf_tab(const C2<T>* __restrict__ tw, int q, int e)
{
    const C2<T> v = tw[kTwN + 4 * q + e];
    return SIGN > 0 ? v : C2<T>{-v.re, v.im};
}
// TW_LF registers and LDS tables hold the exp(+i ...) entries for either
// direction; a transform in the other direction takes them with the tangent
// negated (folded into the butterflies' FMAs), so one set serves both.
template <int SIGN, typename T>
__device__ __forceinline__ C2<T> lf_sign(const C2<T> v)
{
    return SIGN > 0 ? v : C2<T>{-v.re, v.im};
}

template <int N, int E, int RMAX, int TWMODE>
constexpr int tw_count()
{
    return TWMODE == TW_TABLE ? 1 : (tw_offset<N, E, RMAX, TWMODE>(N) > 0 ? tw_offset<N, E, RMAX, TWMODE>(N) : 1);
}

template <typename T, int N, int E, int RMAX, int TWMODE, int NS, int SIGN>
__device__ __forceinline__ void load_twiddles_from(C2<T>* __restrict__ w, const C2<T>* __restrict__ tw, int t)
{
    if constexpr (NS < N) {
        constexpr int R = pass_radix<N, RMAX>(NS);
        if constexpr (NS > 1) {
            constexpr int TT = N / E, B = E / R, STRIDE = kTwN / (NS * R);
            constexpr int OFF = tw_offset<N, E, RMAX, TWMODE>(NS);
            if constexpr (tw_lds_early(TWMODE) && NS < TT) {
                // in the LDS table (fill_lds_twiddles)
            } else if constexpr (tw_lf(TWMODE)) {
                constexpr int LE = lf_entries(R);
#pragma unroll
                for (int m = 0; m < B; ++m) {
                    const int k = (t + TT * m) & (NS - 1);
#pragma unroll
                    for (int e = 0; e < LE; ++e) w[OFF + m * LE + e] = lf_tab<+1>(tw, k * STRIDE, e);
                }
            } else if constexpr (TWMODE == TW_REG || TWMODE == TW_HYB) {
#pragma unroll
                for (int m = 0; m < B; ++m) {
                    const int k = (t + TT * m) & (NS - 1);
#pragma unroll
                    for (int r = 1; r < R; ++r) w[OFF + m * (R - 1) + r - 1] = twiddle_tab<SIGN>(tw, r * k * STRIDE);
                }
            } else {
                // TW_SPLIT: k = t mod NS (NS <= TT) or the t part of k (NS > TT)
                const int k = (NS <= TT) ? (t & (NS - 1)) : t;
#pragma unroll
                for (int r = 1; r < R; ++r) w[OFF + r - 1] = twiddle_tab<SIGN>(tw, r * k * STRIDE);
            }
        }
        load_twiddles_from<T, N, E, RMAX, TWMODE, NS * R, SIGN>(w, tw, t);
    }
}

template <typename T, int N, int E, int RMAX, int TWMODE, int SIGN>
__device__ __forceinline__ void load_twiddles(C2<T>* __restrict__ w, const C2<T>* __restrict__ tw, int t)
{
    if constexpr (TWMODE != TW_TABLE) load_twiddles_from<T, N, E, RMAX, TWMODE, 1, SIGN>(w, tw, t);
}

// The TW_HYB LDS table: entry LOFF(NS) + k (R-1) + r - 1 = exp(SIGN 2 pi i r k / (NS R))
// for every pass with 1 < NS < TT; filled cooperatively by nthr threads.
template <typename T, int N, int E, int RMAX, int TWMODE, int NS, int SIGN>
__device__ __forceinline__ void fill_lds_twiddles_from(C2<T>* __restrict__ ltw, const C2<T>* __restrict__ tw,
                                                       int tid, int nthr)
{
    if constexpr (NS < N && NS < N / E) {
        constexpr int R = pass_radix<N, RMAX>(NS);
        if constexpr (NS > 1) {
            constexpr int STRIDE = kTwN / (NS * R);
            constexpr int LOFF = ltw_offset<N, E, RMAX, TWMODE>(NS);
            constexpr int PER = tw_per(TWMODE, R);
            for (int i = tid; i < NS * PER; i += nthr) {
                if constexpr (TWMODE == TW_LF) {
                    // entry-major (entry e of every k, then e + 1): the lanes of a
                    // wave, k = t mod NS, then read consecutive elements
                    const int e = i / NS, k = i - e * NS;
                    ltw[LOFF + i] = lf_tab<+1>(tw, k * STRIDE, e);
                } else {
                    const int k = i / PER, e = i - k * PER;
                    ltw[LOFF + i] = twiddle_tab<SIGN>(tw, (e + 1) * k * STRIDE);
                }
            }
        }
        fill_lds_twiddles_from<T, N, E, RMAX, TWMODE, NS * R, SIGN>(ltw, tw, tid, nthr);
    }
}

template <typename T, int N, int E, int RMAX, int SIGN, int TWMODE = TW_HYB>
__device__ __forceinline__ void fill_lds_twiddles(C2<T>* __restrict__ ltw, const C2<T>* __restrict__ tw, int tid,
                                                  int nthr)
{
    fill_lds_twiddles_from<T, N, E, (RMAX < E ? RMAX : E), TWMODE, 1, SIGN>(ltw, tw, tid, nthr);
}

// Buffer-resource access to one range the whole wavefront addresses alike (a
// station's output trace, its spectrum row): the base sits in scalar
// registers and each lane supplies a 32-bit byte offset, so the accesses
// issue no per-lane 64-bit address arithmetic.  `bytes` bounds the range
// (the hardware drops stores and zeroes loads whose lane offset is past it;
// callers keep every offset inside it regardless).  Word 3 is the CDNA raw
// buffer format: 32-bit data, no swizzle.
__device__ __forceinline__ __amdgpu_buffer_rsrc_t buffer_range(const void* base, unsigned bytes)
{
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(base), 0, (int)bytes, 0x00020000);
}

// cache-policy operand of the buffer builtins: streaming (non-temporal)
constexpr int kBufNT = 2;

__device__ __forceinline__ void buffer_store_nt(float v, __amdgpu_buffer_rsrc_t r, unsigned voff, int soff)
{
    __builtin_amdgcn_raw_buffer_store_b32(__float_as_uint(v), r, (int)voff, soff, kBufNT);
}

__device__ __forceinline__ void buffer_store_nt(double v, __amdgpu_buffer_rsrc_t r, unsigned voff, int soff)
{
    typedef unsigned u32x2 __attribute__((ext_vector_type(2)));
    __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u32x2, v), r, (int)voff, soff, kBufNT);
}

// 16-byte record at byte offset voff of a buffer range.
template <typename V>
__device__ __forceinline__ V buffer_load16(__amdgpu_buffer_rsrc_t r, unsigned voff)
{
    static_assert(sizeof(V) == 16, "16-byte record");
    return __builtin_bit_cast(V, __builtin_amdgcn_raw_buffer_load_b128(r, (int)voff, 0, 0));
}

// Store of a 16-byte record at byte offset voff of a buffer range (default
// cache policy).  A lane whose offset is at or past the range's end stores
// nothing: the buffer unit's range check drops it.
template <typename V>
__device__ __forceinline__ void buffer_store16(const V& v, __amdgpu_buffer_rsrc_t r, unsigned voff)
{
    static_assert(sizeof(V) == 16, "16-byte record");
    typedef unsigned u32x4 __attribute__((ext_vector_type(4)));
    __builtin_amdgcn_raw_buffer_store_b128(__builtin_bit_cast(u32x4, v), r, (int)voff, 0, 0);
}

// Workgroup barrier that orders LDS only.  The exchanges between FFT passes
// (and the small LDS reductions) need every LDS write before the barrier
// visible after it; no thread reads another thread's global writes.  The
// full barrier's fence also covers global memory and so waits (vmcnt 0) for
// every store the wave still has in flight -- the previous station's output
// -- at each exchange.
__device__ __forceinline__ void lds_barrier()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
    __builtin_amdgcn_s_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

// Synchronisation between the LDS scatter of one pass and the gather of the
// next: an LDS workgroup barrier, or -- when one wavefront owns the
// transform -- only a wave-level fence (LDS operations of one wave complete
// in order).
template <bool WAVE>
__device__ __forceinline__ void lds_sync()
{
    if constexpr (WAVE) {
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    } else {
        lds_barrier();
    }
}

// One Stockham pass (and, recursively, all later ones) of an N-point
// transform held as x[i] = seq[t + TT i] by thread t of its group.
// Butterfly j takes seq[j + r N/R], r < R; with j = t + TT m it finds them in
// x[m + r B].  It multiplies input r by exp(SIGN 2 pi i r k / (NS R)),
// k = j mod NS, runs the R-point DFT, and output r belongs at position
// (j - k) R + k + r NS of the next sequence (natural order after the last
// pass, which therefore stays in registers).  LDS positions use lpad().
template <typename T, int N, int E, int RMAX, int TWMODE, bool WAVE, int NS, int SIGN>
__device__ __forceinline__ void fft_pass(C2<T> (&x)[E], C2<T>* __restrict__ lds,
                                         const C2<T>* __restrict__ tw, const C2<T>* __restrict__ w, int t,
                                         const C2<T>* __restrict__ ltw)
{
    constexpr int R = pass_radix<N, RMAX>(NS);
    constexpr int TT = N / E;
    constexpr int B = E / R;
    constexpr bool LAST = (NS * R == N);
    static_assert(R >= 2 && E % R == 0, "radix");
#pragma unroll
    for (int m = 0; m < B; ++m) {
        const int j = t + TT * m;
        const int k = j & (NS - 1);
        C2<T> v[R];
#pragma unroll
        for (int r = 0; r < R; ++r) v[r] = x[m + r * B];
        if constexpr (tw_lf(TWMODE) && NS > 1) {
            constexpr int LE = lf_entries(R);
            constexpr int OFF = tw_offset<N, E, RMAX, TWMODE>(NS);
            C2<T> L[LE];
#pragma unroll
            for (int e = 0; e < LE; ++e) {
                if constexpr (TWMODE == TW_LF && NS < TT)
                    L[e] = lf_sign<SIGN>(ltw[ltw_offset<N, E, RMAX, TW_LF>(NS) + e * NS + k]);
                else
                    L[e] = lf_sign<SIGN>(w[OFF + m * LE + e]);
            }
            lf_dft<R, SIGN>(v, L);
        } else {
            if constexpr (NS > 1) {
                constexpr int STRIDE = kTwN / (NS * R);
                constexpr int OFF = tw_offset<N, E, RMAX, TWMODE>(NS);
#pragma unroll
                for (int r = 1; r < R; ++r) {
                    C2<T> wr;
                    if constexpr (TWMODE == TW_TABLE) {
                        wr = twiddle_tab<SIGN>(tw, r * k * STRIDE);
                    } else if constexpr (TWMODE == TW_REG || (TWMODE == TW_HYB && NS >= TT)) {
                        wr = w[OFF + m * (R - 1) + r - 1];
                    } else if constexpr (TWMODE == TW_HYB) {
                        wr = ltw[ltw_offset<N, E, RMAX>(NS) + k * (R - 1) + r - 1];
                    } else {
                        wr = w[OFF + r - 1];
                        if constexpr (NS > TT) {
                            const int p = (r * ((TT * m) % NS)) % (NS * R);
                            if (p != 0) {
                                constexpr int Q = NS * R;
                                const CxRoot cr = cx_root(SIGN > 0 ? p : Q - p, Q);
                                wr = cmul(wr, C2<T>{(T)cr.c, (T)cr.s});
                            }
                        }
                    }
                    v[r] = cmul(v[r], wr);
                }
            }
            Dft<R, SIGN, T>::run(v);
        }
        if constexpr (LAST) {
#pragma unroll
            for (int r = 0; r < R; ++r) x[m + r * B] = v[r];
        } else {
            const int base = (j - k) * R + k;
#pragma unroll
            for (int r = 0; r < R; ++r) lds[lpad<T>(base + r * NS)] = v[r];
        }
    }
    if constexpr (!LAST) {
        lds_sync<WAVE>();
#pragma unroll
        for (int i = 0; i < E; ++i) x[i] = lds[lpad<T>(t + TT * i)];
        lds_sync<WAVE>();
        fft_pass<T, N, E, RMAX, TWMODE, WAVE, NS * R, SIGN>(x, lds, tw, w, t, ltw);
    }
}

// Number of passes of an N-point transform with radix at most RMAX.
template <int N, int RMAX>
constexpr int num_passes()
{
    int p = 0;
    for (int ns = 1; ns < N; ns *= pass_radix<N, RMAX>(ns)) ++p;
    return p;
}

// Ping-pong form of fft_pass: pass p scatters into `la`, one barrier, gathers
// from `la`, and pass p+1 scatters into `lb`.  A buffer is written again only
// two exchanges after it was last read, and every thread has passed the
// barrier in between, so one barrier per exchange suffices (against two with
// a single buffer).
template <typename T, int N, int E, int RMAX, int TWMODE, bool WAVE, int NS, int SIGN>
__device__ __forceinline__ void fft_pass_pp(C2<T> (&x)[E], C2<T>* __restrict__ la, C2<T>* __restrict__ lb,
                                            const C2<T>* __restrict__ tw, const C2<T>* __restrict__ w, int t,
                                            const C2<T>* __restrict__ ltw)
{
    constexpr int R = pass_radix<N, RMAX>(NS);
    constexpr int TT = N / E;
    constexpr int B = E / R;
    constexpr bool LAST = (NS * R == N);
    static_assert(R >= 2 && E % R == 0, "radix");
#pragma unroll
    for (int m = 0; m < B; ++m) {
        const int j = t + TT * m;
        const int k = j & (NS - 1);
        C2<T> v[R];
#pragma unroll
        for (int r = 0; r < R; ++r) v[r] = x[m + r * B];
        if constexpr (tw_lf(TWMODE) && NS > 1) {
            constexpr int LE = lf_entries(R);
            constexpr int OFF = tw_offset<N, E, RMAX, TWMODE>(NS);
            C2<T> L[LE];
#pragma unroll
            for (int e = 0; e < LE; ++e) {
                if constexpr (TWMODE == TW_LF && NS < TT)
                    L[e] = lf_sign<SIGN>(ltw[ltw_offset<N, E, RMAX, TW_LF>(NS) + e * NS + k]);
                else
                    L[e] = lf_sign<SIGN>(w[OFF + m * LE + e]);
            }
            lf_dft<R, SIGN>(v, L);
        } else {
            if constexpr (NS > 1) {
                constexpr int STRIDE = kTwN / (NS * R);
                constexpr int OFF = tw_offset<N, E, RMAX, TWMODE>(NS);
#pragma unroll
                for (int r = 1; r < R; ++r) {
                    C2<T> wr;
                    if constexpr (TWMODE == TW_TABLE) {
                        wr = twiddle_tab<SIGN>(tw, r * k * STRIDE);
                    } else if constexpr (TWMODE == TW_REG || (TWMODE == TW_HYB && NS >= TT)) {
                        wr = w[OFF + m * (R - 1) + r - 1];
                    } else if constexpr (TWMODE == TW_HYB) {
                        wr = ltw[ltw_offset<N, E, RMAX>(NS) + k * (R - 1) + r - 1];
                    } else {
                        wr = w[OFF + r - 1];
                        if constexpr (NS > TT) {
                            const int p = (r * ((TT * m) % NS)) % (NS * R);
                            if (p != 0) {
                                constexpr int Q = NS * R;
                                const CxRoot cr = cx_root(SIGN > 0 ? p : Q - p, Q);
                                wr = cmul(wr, C2<T>{(T)cr.c, (T)cr.s});
                            }
                        }
                    }
                    v[r] = cmul(v[r], wr);
                }
            }
            Dft<R, SIGN, T>::run(v);
        }
        if constexpr (LAST) {
#pragma unroll
            for (int r = 0; r < R; ++r) x[m + r * B] = v[r];
        } else {
            const int base = (j - k) * R + k;
#pragma unroll
            for (int r = 0; r < R; ++r) la[lpad<T>(base + r * NS)] = v[r];
        }
    }
    if constexpr (!LAST) {
        lds_sync<WAVE>();
#pragma unroll
        for (int i = 0; i < E; ++i) x[i] = la[lpad<T>(t + TT * i)];
        fft_pass_pp<T, N, E, RMAX, TWMODE, WAVE, NS * R, SIGN>(x, lb, la, tw, w, t, ltw);
    }
}

// Two transforms of the same length and direction run in lockstep: every
// pass applies the same twiddles to both, scatters x into `la` and y into
// `lb`, and one barrier pair per exchange serves both (the per-transform
// barrier count of the ping-pong form, with twice the independent work
// between barriers).
template <typename T, int N, int E, int RMAX, int TWMODE, int NS, int SIGN>
__device__ __forceinline__ void fft_pass2(C2<T> (&x)[E], C2<T> (&y)[E], C2<T>* __restrict__ la,
                                          C2<T>* __restrict__ lb, const C2<T>* __restrict__ tw,
                                          const C2<T>* __restrict__ w, int t, const C2<T>* __restrict__ ltw)
{
    constexpr int R = pass_radix<N, RMAX>(NS);
    constexpr int TT = N / E;
    constexpr int B = E / R;
    constexpr bool LAST = (NS * R == N);
    static_assert(R >= 2 && E % R == 0 && TWMODE != TW_SPLIT, "radix");
#pragma unroll
    for (int m = 0; m < B; ++m) {
        const int j = t + TT * m;
        const int k = j & (NS - 1);
        C2<T> u[R], v[R];
#pragma unroll
        for (int r = 0; r < R; ++r) {
            u[r] = x[m + r * B];
            v[r] = y[m + r * B];
        }
        if constexpr (tw_lf(TWMODE) && NS > 1) {
            constexpr int LE = lf_entries(R);
            constexpr int OFF = tw_offset<N, E, RMAX, TWMODE>(NS);
            C2<T> L[LE];
#pragma unroll
            for (int e = 0; e < LE; ++e) {
                if constexpr (TWMODE == TW_LF && NS < TT)
                    L[e] = lf_sign<SIGN>(ltw[ltw_offset<N, E, RMAX, TW_LF>(NS) + e * NS + k]);
                else
                    L[e] = lf_sign<SIGN>(w[OFF + m * LE + e]);
            }
            lf_dft<R, SIGN>(u, L);
            lf_dft<R, SIGN>(v, L);
        } else {
            if constexpr (NS > 1) {
                constexpr int STRIDE = kTwN / (NS * R);
                constexpr int OFF = tw_offset<N, E, RMAX, TWMODE>(NS);
#pragma unroll
                for (int r = 1; r < R; ++r) {
                    C2<T> wr;
                    if constexpr (TWMODE == TW_TABLE)
                        wr = twiddle_tab<SIGN>(tw, r * k * STRIDE);
                    else if constexpr (TWMODE == TW_HYB && NS < TT)
                        wr = ltw[ltw_offset<N, E, RMAX>(NS) + k * (R - 1) + r - 1];
                    else
                        wr = w[OFF + m * (R - 1) + r - 1];
                    u[r] = cmul(u[r], wr);
                    v[r] = cmul(v[r], wr);
                }
            }
            Dft<R, SIGN, T>::run(u);
            Dft<R, SIGN, T>::run(v);
        }
        if constexpr (LAST) {
#pragma unroll
            for (int r = 0; r < R; ++r) {
                x[m + r * B] = u[r];
                y[m + r * B] = v[r];
            }
        } else {
            const int base = (j - k) * R + k;
#pragma unroll
            for (int r = 0; r < R; ++r) {
                la[lpad<T>(base + r * NS)] = u[r];
                lb[lpad<T>(base + r * NS)] = v[r];
            }
        }
    }
    if constexpr (!LAST) {
        lds_barrier();
#pragma unroll
        for (int i = 0; i < E; ++i) {
            x[i] = la[lpad<T>(t + TT * i)];
            y[i] = lb[lpad<T>(t + TT * i)];
        }
        lds_barrier();
        fft_pass2<T, N, E, RMAX, TWMODE, NS * R, SIGN>(x, y, la, lb, tw, w, t, ltw);
    }
}

template <typename T, int N, int E, int SIGN, int TWMODE, int RMAX>
__device__ __forceinline__ void fft2(C2<T> (&x)[E], C2<T> (&y)[E], C2<T>* __restrict__ la, C2<T>* __restrict__ lb,
                                     const C2<T>* __restrict__ tw, int t, const C2<T>* __restrict__ w,
                                     const C2<T>* __restrict__ ltw = nullptr)
{
    static_assert((N & (N - 1)) == 0 && N >= E && (E & (E - 1)) == 0 && RMAX <= 32, "sizes");
    fft_pass2<T, N, E, (RMAX < E ? RMAX : E), TWMODE, 1, SIGN>(x, y, la, lb, tw, w, t, ltw);
}

// Full transform with ping-pong buffers; the first exchange writes `la`.
// The caller must not write `la` or `lb` again until every thread of the
// group has passed a barrier that follows its last gather.
template <typename T, int N, int E, int SIGN, int TWMODE, int RMAX, bool WAVE>
__device__ __forceinline__ void fft_pp(C2<T> (&x)[E], C2<T>* __restrict__ la, C2<T>* __restrict__ lb,
                                       const C2<T>* __restrict__ tw, int t, const C2<T>* __restrict__ w,
                                       const C2<T>* __restrict__ ltw = nullptr)
{
    static_assert((N & (N - 1)) == 0 && N >= E && (E & (E - 1)) == 0 && RMAX <= 32, "sizes");
    fft_pass_pp<T, N, E, (RMAX < E ? RMAX : E), TWMODE, WAVE, 1, SIGN>(x, la, lb, tw, w, t, ltw);
}

// ---------------------------------------------------------------------------
// The 4096-point transform with two of its three exchanges inside the
// wavefront (TW_LFW, 8 values per thread, 512 threads t = 64 w + l, wave w,
// lane l = 8 lh + ll).  Positions p = 512 p3 + 64 p2 + 8 p1 + p0 in base-8
// digits; the input is loaded digit-reversed (position p holds element
// 512 p0 + 64 p1 + 8 p2 + p3), and four decimation-in-time radix-8 passes
// combine along p0, p1, p2, p3 in turn, leaving the output in natural order.
// Pass s multiplies input r by exp(SIGN 2 pi i r k / 8^s), k the number
// formed by the digits below the one it combines, and runs the 8-point DFT:
// with the layouts below k = t mod 8^(s-1), the factor of Stockham pass
// NS = 8^(s-1) for thread t, so the TW_LFR registers serve unchanged.
// Register index r holds the digit a pass combines; the other digits sit in
// the thread index:
//   pass 1: r = p0, w = p3, lh = p2, ll = p1
//   pass 2: r = p1, w = p3, lh = p2, ll = p0   (r <-> ll: the wavefront's LDS block)
//   pass 3: r = p2, w = p3, lh = p1, ll = p0   (r <-> lh: register transpose)
//   pass 4: r = p3, w = p2, lh = p1, ll = p0   (r <-> w: workgroup exchange)
// so the output is x[r] = X[t + 512 r], as after the Stockham passes.  The
// register transpose of lane bits 3-5 costs at most one VALU move per
// 32-bit word and bit (a bank-masked DPP rotation for bit 3, plus a copy per
// pair of words; one lane swap per two words for bits 4 and 5); lane bits
// 0-2 would take two (a DPP move and a select), so that transpose goes
// through LDS, where a wavefront needs no barrier.

// Slot of position q in the LDS buffers of fft4096_xw: an XOR of bits 0-2
// with bits 6-8 (a permutation of each aligned block of 8 positions, so a
// block of 512 stays in place), which keeps the gathers and the exchange (64
// consecutive positions per wave) and the staging scatter (consecutive bins
// k to positions 64 (k mod 8) + ...) free of bank conflicts for 8- and
// 16-byte elements.
__device__ __forceinline__ constexpr int xw_slot(int q) { return q ^ ((q >> 6) & 7); }
// The digit-reversed input order in base-8 digits 0 and 2 of a 4096-point
// index (an involution): element e sits at the gather position xw_pos(e) of
// the thread and register pass 1 takes it from, and position q holds element
// xw_pos(q).
__device__ __forceinline__ constexpr int xw_pos(int e)
{
    return (e & 0xE38) | ((e & 7) << 6) | ((e >> 6) & 7);
}

// One transpose step of a pair of 32-bit words held in registers r0 and
// r1 = r0 + RB by every lane: lanes whose bit LB is clear take their
// partner's (lane ^ LB) r0 word into r1, lanes whose bit is set take the
// partner's r1 word into r0.  LB 16 and 32: the gfx950 lane-swap
// instructions, which perform exactly this exchange between two registers.
// LB 8: a DPP rotation by 8 within the row of 16 lanes (lane i's word to
// lane i + 8 mod 16) that writes only the lanes taking a word (bank mask:
// lanes 4 b .. 4 b + 3 form bank b of a row), the others keeping theirs.
template <int LB>
__device__ __forceinline__ void xw_swap_words(unsigned& a, unsigned& b)
{
    static_assert(LB == 8 || LB == 16 || LB == 32, "lane bits 3-5");
    if constexpr (LB == 16) {
        const auto r = __builtin_amdgcn_permlane16_swap(a, b, false, false);
        a = r[0];
        b = r[1];
    } else if constexpr (LB == 32) {
        const auto r = __builtin_amdgcn_permlane32_swap(a, b, false, false);
        a = r[0];
        b = r[1];
    } else {
        const unsigned b0 = b;
        b = __builtin_amdgcn_update_dpp(b, a, 0x128, 0xF, 0x3, false);   // banks 0, 1 <- lane + 8
        a = __builtin_amdgcn_update_dpp(a, b0, 0x128, 0xF, 0xC, false);  // banks 2, 3 <- lane - 8
    }
}

template <int LB, typename T>
__device__ __forceinline__ void xw_swap(C2<T>& x0, C2<T>& x1)
{
    struct Words {
        unsigned v[sizeof(C2<T>) / 4];
    };
    Words a = __builtin_bit_cast(Words, x0), b = __builtin_bit_cast(Words, x1);
#pragma unroll
    for (int i = 0; i < (int)(sizeof(C2<T>) / 4); ++i) xw_swap_words<LB>(a.v[i], b.v[i]);
    x0 = __builtin_bit_cast(C2<T>, a);
    x1 = __builtin_bit_cast(C2<T>, b);
}

// Transpose of the register index (bits 0-2) with lane bits 3-5: the value
// of lane bits 3-5 = a in register b moves to lane bits 3-5 = b, register a.
template <typename T>
__device__ __forceinline__ void xw_transpose_hi(C2<T> (&x)[8])
{
#pragma unroll
    for (int bit = 0; bit < 3; ++bit) {
#pragma unroll
        for (int r0 = 0; r0 < 8; ++r0) {
            if ((r0 >> bit) & 1) continue;
            if (bit == 0) xw_swap<8>(x[r0], x[r0 + 1]);
            if (bit == 1) xw_swap<16>(x[r0], x[r0 + 2]);
            if (bit == 2) xw_swap<32>(x[r0], x[r0 + 4]);
        }
    }
}

// One radix-8 pass in registers: inputs r times the pass-NS factors of the
// thread (TW_LFR registers, none for NS = 1), then the 8-point DFT.
template <typename T, int NS, int SIGN, int TWMODE = TW_LFW>
__device__ __forceinline__ void xw_pass(C2<T> (&x)[8], const C2<T>* __restrict__ w,
                                        const C2<T>* __restrict__ ltw = nullptr, int t = 0)
{
    if constexpr (NS > 1) {
        constexpr int LE = lf_entries(8);
        constexpr int OFF = tw_offset<4096, 8, 8, TWMODE>(NS);
        C2<T> L[LE];
#pragma unroll
        for (int e = 0; e < LE; ++e) {
            // TW_LF: the early passes' pairs from the LDS table
            if constexpr (tw_lds_early(TWMODE) && NS < 512)
                L[e] = lf_sign<SIGN>(ltw[ltw_offset<4096, 8, 8, TW_LF>(NS) + e * NS + (t & (NS - 1))]);
            else
                L[e] = lf_sign<SIGN>(w[OFF + e]);
        }
        lf_dft<8, SIGN>(x, L);
    } else {
        Dft<8, SIGN, T>::run(x);
    }
}

// x[r] holds position t + 512 r of the digit-reversed input (see above);
// returns x[r] = output element t + 512 r.  `la` is a buffer of
// lds_elems<4096>() slots that no other thread group uses; the caller must
// not write it again before every thread has passed a barrier that follows
// this call (it holds one exchange between a barrier and the gathers after
// it).  The first transpose goes through the wavefront's own 512 slots of
// `la` (a wavefront's LDS operations complete in order, and every other
// wavefront's reads of `la` from the previous call precede the caller's
// barrier before this one), with no workgroup barrier.
template <typename T, int SIGN>
__device__ __forceinline__ void fft4096_xw(C2<T> (&x)[8], C2<T>* __restrict__ la, const C2<T>* __restrict__ w,
                                           int t)
{
    xw_pass<T, 1, SIGN>(x, w);
    {
        // in the wavefront's own block of `la`, the slots its workgroup
        // exchange below writes (xw_slot keeps a block in place): register b
        // of lane l at 64 b + (l ^ b); lane (lh, ll) reads register a at
        // 64 ll + ((8 lh + a) ^ ll) -- for 16 consecutive lanes 8 (lh mod 2)
        // + (a ^ ll) mod 16 are distinct, so no two share a bank
        C2<T>* __restrict__ blk = la + 512 * (t >> 6);
        const int l = t & 63, ll = t & 7, lh8 = t & 0x38;
#pragma unroll
        for (int b = 0; b < 8; ++b) blk[64 * b + (l ^ b)] = x[b];
        lds_sync<true>();
#pragma unroll
        for (int a = 0; a < 8; ++a) x[a] = blk[64 * ll + ((lh8 + a) ^ ll)];
    }
    xw_pass<T, 8, SIGN>(x, w);
    xw_transpose_hi(x);
    xw_pass<T, 64, SIGN>(x, w);
    const int wv = t >> 6, l = t & 63;
#pragma unroll
    for (int r = 0; r < 8; ++r) la[xw_slot(512 * wv + 64 * r + l)] = x[r];
    lds_barrier();
#pragma unroll
    for (int r = 0; r < 8; ++r) x[r] = la[xw_slot(512 * r + 64 * wv + l)];
    xw_pass<T, 512, SIGN>(x, w);
}

// Two 4096-point transforms (x and y, the same layout, direction and
// twiddles) in fft4096_xw's form: both first transposes, one after the
// other, in the wavefront's own block of `la`; both second transposes in
// registers; the workgroup exchange of x through `la` and, after its
// barrier, that of y through `lb` (the caller's staging buffer: every
// wavefront's gathers from it precede its first exchange write, so the
// first barrier also ends every use of `lb` by the caller).  The caller
// must not write `la` or `lb` again before every thread has passed a
// barrier that follows this call.
template <typename T, int SIGN, int TWMODE>
__device__ __forceinline__ void fft4096_xw2(C2<T> (&x)[8], C2<T> (&y)[8], C2<T>* __restrict__ la,
                                            C2<T>* __restrict__ lb, const C2<T>* __restrict__ w, int t,
                                            const C2<T>* __restrict__ ltw)
{
    xw_pass<T, 1, SIGN, TWMODE>(x, w, ltw, t);
    xw_pass<T, 1, SIGN, TWMODE>(y, w, ltw, t);
    {
        C2<T>* __restrict__ blk = la + 512 * (t >> 6);
        const int l = t & 63, ll = t & 7, lh8 = t & 0x38;
#pragma unroll
        for (int b = 0; b < 8; ++b) blk[64 * b + (l ^ b)] = x[b];
        lds_sync<true>();
#pragma unroll
        for (int a = 0; a < 8; ++a) x[a] = blk[64 * ll + ((lh8 + a) ^ ll)];
#pragma unroll
        for (int b = 0; b < 8; ++b) blk[64 * b + (l ^ b)] = y[b];
        lds_sync<true>();
#pragma unroll
        for (int a = 0; a < 8; ++a) y[a] = blk[64 * ll + ((lh8 + a) ^ ll)];
    }
    xw_pass<T, 8, SIGN, TWMODE>(x, w, ltw, t);
    xw_pass<T, 8, SIGN, TWMODE>(y, w, ltw, t);
    xw_transpose_hi(x);
    xw_transpose_hi(y);
    xw_pass<T, 64, SIGN, TWMODE>(x, w, ltw, t);
    xw_pass<T, 64, SIGN, TWMODE>(y, w, ltw, t);
    const int wv = t >> 6, l = t & 63;
#pragma unroll
    for (int r = 0; r < 8; ++r) la[xw_slot(512 * wv + 64 * r + l)] = x[r];
    lds_barrier();
#pragma unroll
    for (int r = 0; r < 8; ++r) x[r] = la[xw_slot(512 * r + 64 * wv + l)];
#pragma unroll
    for (int r = 0; r < 8; ++r) lb[xw_slot(512 * wv + 64 * r + l)] = y[r];
    lds_barrier();
#pragma unroll
    for (int r = 0; r < 8; ++r) y[r] = lb[xw_slot(512 * r + 64 * wv + l)];
    xw_pass<T, 512, SIGN, TWMODE>(x, w, ltw, t);
    xw_pass<T, 512, SIGN, TWMODE>(y, w, ltw, t);
}

// Full N-point transform of the group's sequence, exp(SIGN ...) kernel, no
// scaling.  Every thread of the group must call it; unless WAVE it contains
// workgroup barriers, so every thread of the workgroup must call it.
// `w` holds the per-thread twiddles of load_twiddles (unused for TW_TABLE).
template <typename T, int N, int E, int SIGN, int TWMODE = TW_TABLE, int RMAX = E, bool WAVE = false>
__device__ __forceinline__ void fft(C2<T> (&x)[E], C2<T>* __restrict__ lds,
                                    const C2<T>* __restrict__ tw, int t,
                                    const C2<T>* __restrict__ w = nullptr,
                                    const C2<T>* __restrict__ ltw = nullptr)
{
    static_assert((N & (N - 1)) == 0 && N >= E && (E & (E - 1)) == 0 && RMAX <= 32, "sizes");
    fft_pass<T, N, E, (RMAX < E ? RMAX : E), TWMODE, WAVE, 1, SIGN>(x, lds, tw, w, t, ltw);
}

}  // namespace au
