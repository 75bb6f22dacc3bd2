// au_kernels.h -- the three kernels of the unfolding path and their
// per-event descriptors.
//
//   k_spectrum : per (event, station): both channel traces -> one packed
//                complex FFT -> in-band spectra X_0, X_1 (section 4 FFT;
//                computed once per station and reused for every direction).
//   k_coef     : per (event, direction, in-band bin): trilinear pattern
//                interpolation (section 3), 2x2 determinant with the FP64
//                fallback, inverse, band and 1/N folded in.  The result is
//                the station-independent coefficient matrix of the bin.
//   k_unfold   : per (event, direction, station): E = coef * X per bin,
//                Hermitian packing of (E_theta, E_phi) into one complex
//                spectrum, inverse FFT, coalesced store of both traces.
#pragma once

#include "au_device.h"

namespace au {

// Per-event offsets and sizes shared by the kernels.  Offsets are in
// elements of the buffer they index.
struct EvDesc {
    int64_t volt_off;    // into the trace buffer (Tin elements)
    int64_t efield_off;  // into the output buffer (T elements)
    int64_t x_off;       // into the spectra workspace (XBin records)
    int64_t m_off;       // into the coefficient workspace (MBin records)
    int64_t dir_off;     // into the direction list ([2] doubles per entry)
    int32_t S, N, D, k_lo, nb, pad;
};

// In-band spectra of one station at one bin: channel 0 and channel 1.
template <typename T>
struct alignas(16) XBin {
    C2<T> x0, x1;
};

// Coefficients of one (direction, bin) in packed form.  With the solution
// [E_theta; E_phi] = C [X_0; X_1] (C = (1/N) H^-1, zero where the bin is
// singular), the inverse transform's packed spectrum needs
//   Z[k]            = E_theta + i E_phi = p0 X_0 + p1 X_1,
//   conj Z[N - k]   = E_theta - i E_phi = q0 X_0 + q1 X_1,
// so p_j = C_0j + i C_1j and q_j = C_0j - i C_1j.  (The pattern-response
// entry point stores the interpolated H = [p0 p1; q0 q1] in the same record.)
template <typename T>
struct alignas(16) MBin {
    C2<T> p0, p1, q0, q1;
};

// Pattern grid as the kernels see it.
struct GridDev {
    int32_t n_freq, n_zen, n_az, pad;
    int64_t f0_hz, df_hz;
    double zen0, dzen, az0, daz;
};

constexpr int kBlock = 256;

// FFT groups per workgroup for an N-point transform with E values per thread:
// fill kBlock threads, but keep LDS at or under 64 KiB.
template <typename T, int N, int E, int BUFS = 1>
constexpr int groups_per_block()
{
    constexpr int tt = N / E;
    int g = tt >= kBlock ? 1 : kBlock / tt;
    const int cap = 65536 / (BUFS * lds_elems<N>() * (int)sizeof(C2<T>));
    if (g > cap) g = cap;
    return g < 1 ? 1 : g;
}

}  // namespace au
