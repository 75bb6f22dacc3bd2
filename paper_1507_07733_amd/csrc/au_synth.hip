// au_synth.hip -- device generator of the counter-based synthetic trace
// stream (library libausynth.so, separate from the unfolding library: it is
// input synthesis for the large-batch workload and its tests, and holds none
// of the unfolding arithmetic).  The definition -- and a numpy
// implementation that gives bit-identical traces -- is in
// paper_1507_07733_amd/synth.py (stream_traces):
//   r = Philox4x32-10(counter, key = (seed, 0x7733)) (Salmon, Moraes, Dror,
//       Shaw, "Parallel random numbers: as easy as 1, 2, 3", SC'11);
//   noise = (sum of four 22-bit uniforms of r(n, 2s + c, e, 0) - 2) * sqrt(3);
//   t0 = r(0, s, e, 1).x mod N; A = 5 + 15 u, u = 24-bit uniform of r(0, 2s + c, e, 2).x;
//   V[e][s][c][n] = noise + A * D[(n - t0) mod N].
// Every float operation is a single IEEE float32 operation with round to
// nearest even (contraction into fused multiply-adds is switched off).
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>

namespace {

struct U4 {
    uint32_t x, y, z, w;
};

__device__ __forceinline__ U4 philox4x32_10(U4 c, uint32_t k0, uint32_t k1)
{
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        if (r) {
            k0 += 0x9E3779B9u;
            k1 += 0xBB67AE85u;
        }
        const uint32_t lo0 = 0xD2511F53u * c.x, hi0 = __umulhi(0xD2511F53u, c.x);
        const uint32_t lo1 = 0xCD9E8D57u * c.z, hi1 = __umulhi(0xCD9E8D57u, c.z);
        c = U4{hi1 ^ c.y ^ k0, lo1, hi0 ^ c.w ^ k1, lo0};
    }
    return c;
}

constexpr uint32_t kKey1 = 0x7733u;

// grid (ceil(N / 256), 2 S, n_events); out [n_events][S][2][N]
__global__ __launch_bounds__(256) void k_synth_traces(float* __restrict__ out, int event0, int S, int N,
                                                      uint32_t seed, const float* __restrict__ dtab, float sqrt3)
{
    // one rounding per operation: no contraction of a product and a sum into a
    // fused multiply-add (the operations are written here, inside the scope
    // of this pragma, not through library intrinsics that inline from
    // elsewhere)
#pragma clang fp contract(off)
    const int n = blockIdx.x * blockDim.x + threadIdx.x;
    if (n >= N) return;
    const uint32_t sc = blockIdx.y, s = sc >> 1;
    const uint32_t e = (uint32_t)event0 + blockIdx.z;
    const U4 r = philox4x32_10(U4{(uint32_t)n, sc, e, 0u}, seed, kKey1);
    const float u0 = (float)(r.x >> 10) * 0x1p-22f, u1 = (float)(r.y >> 10) * 0x1p-22f;
    const float u2 = (float)(r.z >> 10) * 0x1p-22f, u3 = (float)(r.w >> 10) * 0x1p-22f;
    const float sum = (u0 + u1) + (u2 + u3);
    const float noise = (sum - 2.0f) * sqrt3;
    const uint32_t t0 = philox4x32_10(U4{0u, s, e, 1u}, seed, kKey1).x & (uint32_t)(N - 1);
    const float ua = (float)(philox4x32_10(U4{0u, sc, e, 2u}, seed, kKey1).x >> 8) * 0x1p-24f;
    const float a = 5.0f + 15.0f * ua;
    const float p = a * dtab[((uint32_t)n - t0) & (uint32_t)(N - 1)];
    out[((size_t)blockIdx.z * 2 * S + sc) * N + n] = noise + p;
}

}  // namespace

// Fill d_out [n_events][S][2][N] (float32, device) with events event0 ..
// event0 + n_events - 1 of the stream; d_dirichlet is the float32 table D[N]
// (device).  Enqueued on `stream` (hipStream_t, NULL = default).  Returns 0,
// -1 for bad sizes (N a power of two in [16, 4096], S in [1, 32767],
// n_events in [1, 65535]), -3 if the launch fails.
extern "C" int ausynth_traces(void* d_out, int n_events, int event0, int S, int N, uint32_t seed,
                              const float* d_dirichlet, void* stream)
{
    if (!d_out || !d_dirichlet || N < 16 || N > 4096 || (N & (N - 1)) != 0 || S < 1 || S > 32767 ||
        n_events < 1 || n_events > 65535 || event0 < 0)
        return -1;
    const float sqrt3 = (float)std::sqrt(3.0);
    hipLaunchKernelGGL(k_synth_traces, dim3((N + 255) / 256, 2 * S, n_events), dim3(256), 0, (hipStream_t)stream,
                       (float*)d_out, event0, S, N, seed, d_dirichlet, sqrt3);
    return hipGetLastError() == hipSuccess ? 0 : -3;
}
