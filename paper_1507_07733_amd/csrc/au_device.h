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

// Twiddle table: tw[q] = exp(-2 pi i q / kTwN), q in [0, kTwN).  Any
// N-point transform with N | kTwN indexes it with stride kTwN / N.
constexpr int kTwN = 4096;

template <int SIGN, typename T>
__device__ __forceinline__ C2<T> twiddle_tab(const C2<T>* __restrict__ tw, int q)
{
    const C2<T> w = tw[q];
    return SIGN < 0 ? w : cconj(w);
}

// One Stockham pass (and, recursively, all later ones) of an N-point
// transform held as x[i] = seq[t + (N/E) i] by thread t of its group.
// NS is the length of the sub-transforms already completed.
//
// Butterfly j (j < N/R) takes seq[j + r N/R], r < R; with j = t + (N/E) m it
// finds them in x[m + r E/R].  It multiplies input r by
// exp(SIGN 2 pi i r k / (NS R)), k = j mod NS, runs the R-point DFT, and
// output r belongs at position (j - k) R + k + r NS of the next sequence.
template <typename T, int N, int E, int NS, int SIGN>
__device__ __forceinline__ void fft_pass(C2<T> (&x)[E], C2<T>* __restrict__ lds,
                                         const C2<T>* __restrict__ tw, int t)
{
    constexpr int R = (N / NS < E) ? N / NS : E;
    constexpr int TT = N / E;
    constexpr int B = E / R;
    constexpr bool LAST = (NS * R == N);
    static_assert(R >= 2 || N == 1, "radix");
#pragma unroll
    for (int m = 0; m < B; ++m) {
        const int j = t + TT * m;
        const int k = j & (NS - 1);
        C2<T> v[R];
#pragma unroll
        for (int r = 0; r < R; ++r) v[r] = x[m + r * B];
        if constexpr (NS > 1) {
            constexpr int STRIDE = kTwN / (NS * R);
#pragma unroll
            for (int r = 1; r < R; ++r) v[r] = cmul(v[r], twiddle_tab<SIGN>(tw, r * k * STRIDE));
        }
        Dft<R, SIGN, T>::run(v);
        if constexpr (LAST) {
#pragma unroll
            for (int r = 0; r < R; ++r) x[m + r * B] = v[r];
        } else {
            const int base = (j - k) * R + k;
#pragma unroll
            for (int r = 0; r < R; ++r) lds[base + r * NS] = v[r];
        }
    }
    if constexpr (!LAST) {
        __syncthreads();
#pragma unroll
        for (int i = 0; i < E; ++i) x[i] = lds[t + TT * i];
        __syncthreads();
        fft_pass<T, N, E, NS * R, SIGN>(x, lds, tw, t);
    }
}

// Full N-point transform of the group's sequence, exp(SIGN ...) kernel, no
// scaling.  Every thread of the workgroup must call it (it contains
// workgroup barriers when N > E).
template <typename T, int N, int E, int SIGN>
__device__ __forceinline__ void fft(C2<T> (&x)[E], C2<T>* __restrict__ lds,
                                    const C2<T>* __restrict__ tw, int t)
{
    static_assert((N & (N - 1)) == 0 && N >= E && (E & (E - 1)) == 0 && E <= 32, "sizes");
    fft_pass<T, N, E, 1, SIGN>(x, lds, tw, t);
}

}  // namespace au
