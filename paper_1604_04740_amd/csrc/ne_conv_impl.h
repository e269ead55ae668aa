// ne_conv_impl.h -- fused circular convolution device code (shared by the
// convolution entry point and the batched persistent kernel).
//
// Fused: c [M][N] (int8/int32/int64) -> d_hat [M][N] (int32/int64) + flags.
// All M streams of a position are handled by one thread: the staging of
// each 256-tap tile entangles c into eps (section III-C) in LDS, the taps
// are applied with 64-bit multiply-adds, and the epilogue disentangles and
// checks (delta never reaches memory).  Each wavefront covers 64
// consecutive positions, i.e. whole flag words.
#pragma once

#include "ne_arith.h"
#include "ne_internal.h"

namespace ne {
namespace {

constexpr int kConvT = 256;

// Positions [t0, t0 + 256) of every stream; xs is M * 512 int64 and gs 256
// int32 of LDS.  Called by k_circconv_fused and by the batched kernel.
template <int M, typename T>
__device__ __forceinline__ void conv_fused_block(const T *__restrict__ c,
                                                 const int8_t *__restrict__ g,
                                                 void *__restrict__ dhat, int out64,
                                                 uint32_t *__restrict__ flags,
                                                 unsigned long long *__restrict__ n_bad,
                                                 int64_t N, int l, int r, int64_t t0,
                                                 int64_t (*xs)[2 * kConvT], int32_t *gs)
{
    constexpr int kT = kConvT;
    const int tid = threadIdx.x, lane = tid & 63;
    uint64_t acc[M];
#pragma unroll
    for (int s = 0; s < M; ++s)
        acc[s] = 0;
    for (int64_t j0 = 0; j0 < N; j0 += kT) {
        gs[tid] = (j0 + tid < N) ? (int32_t)g[j0 + tid] : 0;
        const int64_t base = t0 - j0 - (kT - 1);
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const int i = tid + h * kT;
            if (i < 2 * kT - 1) {
                int64_t idx = (base + i) % N;
                if (idx < 0)
                    idx += N;
                // slot s holds stream (r + s) mod M: load and entangle in slot order
                int64_t v[M];
#pragma unroll
                for (int s = 0; s < M; ++s)
                    v[s] = (int64_t)c[(int64_t)((r + s) % M) * N + idx];
#pragma unroll
                for (int s = 0; s < M; ++s)
                    xs[s][i] = entangle_word(v[s], v[(s + M - 1) % M], l);
            }
        }
        __syncthreads();
        const int taps = (N - j0 < kT) ? (int)(N - j0) : kT;
        for (int jj = 0; jj < taps; ++jj) {
            const uint64_t gv = (uint64_t)(int64_t)gs[jj];
#pragma unroll
            for (int s = 0; s < M; ++s)
                acc[s] += (uint64_t)xs[s][tid - jj + kT - 1] * gv;
        }
        __syncthreads();
    }
    const int64_t n = t0 + tid;
    const bool valid = n < N;
    int64_t d[M], o[M];
#pragma unroll
    for (int s = 0; s < M; ++s)
        d[s] = (int64_t)acc[s];
    const bool f = disentangle_rot<M>(d, l, o) && valid;
    if (valid) {
#pragma unroll
        for (int s = 0; s < M; ++s) {
            const int64_t idx = (int64_t)((r + s) % M) * N + n;
            if (out64)
                ((int64_t *)dhat)[idx] = o[s];
            else
                ((int32_t *)dhat)[idx] = (int32_t)o[s];
        }
    }
    const uint64_t mask = __ballot(f);
    const int64_t words = (N + 31) / 32, w0 = (t0 + (tid & ~63)) / 32;
    if (flags) {
        if (lane == 0 && w0 < words)
            flags[w0] = (uint32_t)mask;
        if (lane == 32 && w0 + 1 < words)
            flags[w0 + 1] = (uint32_t)(mask >> 32);
    }
    if (n_bad && lane == 0 && mask)
        atomicAdd(n_bad, (unsigned long long)__popcll(mask));
}

template <int M, typename T>
__global__ __launch_bounds__(kConvT) void k_circconv_fused(const T *__restrict__ c,
                                                           const int8_t *__restrict__ g,
                                                           void *__restrict__ dhat, int out64,
                                                           uint32_t *__restrict__ flags,
                                                           unsigned long long *__restrict__ n_bad,
                                                           int64_t N, int l, int r)
{
    __shared__ int64_t xs[M][2 * kConvT];
    __shared__ int32_t gs[kConvT];
    conv_fused_block<M, T>(c, g, dhat, out64, flags, n_bad, N, l, r,
                           (int64_t)blockIdx.x * kConvT, xs, gs);
}

} // namespace
} // namespace ne
