// ne_perm_impl.h -- fused permute / scale / add device code (shared by the
// element-wise entry point and the batched persistent kernel).
#pragma once

#include "ne_arith.h"
#include "ne_internal.h"

namespace ne {
namespace {

constexpr int kPermThreads = 256;

// Fused permute / scale / add: for every position n, gather the M input
// words at perm[n], entangle them (slot s holds stream (r + s) mod M),
// apply delta = scale * eps + (2^l + 1) add, disentangle and check.  The
// entangled words exist only in registers.  Wavefronts cover whole flag
// words (64 consecutive positions).
// Positions [first, last) (first a multiple of 64), visited by the
// workgroup's 256 threads starting at `first + start`, step `stride`.
template <int M, typename T>
__device__ __forceinline__ void perm_fused_range(
    const T *__restrict__ c, const int32_t *__restrict__ perm, const int64_t *__restrict__ scale,
    const int64_t *__restrict__ add, void *__restrict__ dhat, int out64,
    uint32_t *__restrict__ flags, unsigned long long *__restrict__ n_bad, int64_t N, int l, int r,
    int64_t first, int64_t last, int64_t start, int64_t stride)
{
    const int lane = threadIdx.x & 63;
    const int64_t words = (N + 31) / 32;
    unsigned long long count = 0;
    for (int64_t base = first + start + (threadIdx.x & ~63); base < last; base += stride) {
        const int64_t n = base + lane;
        bool f = false;
        if (n < last) {
            int64_t src = perm[n];
            src = src < 0 ? 0 : (src >= N ? N - 1 : src);
            int64_t v[M]; // v[s] = input of stream (r + s) mod M, i.e. slot order
#pragma unroll
            for (int s = 0; s < M; ++s)
                v[s] = (int64_t)c[(int64_t)((r + s) % M) * N + src];
            const uint64_t sc = scale ? (uint64_t)scale[n] : 1u;
            const uint64_t a = add ? (uint64_t)entangle_word(add[n], add[n], l) : 0u;
            int64_t d[M], o[M];
#pragma unroll
            for (int s = 0; s < M; ++s)
                d[s] = (int64_t)(sc * (uint64_t)entangle_word(v[s], v[(s + M - 1) % M], l) + a);
            f = disentangle_rot<M>(d, l, o);
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
        if (flags) {
            const int64_t w0 = base / 32;
            if (lane == 0 && w0 < words)
                flags[w0] = (uint32_t)mask;
            if (lane == 32 && w0 + 1 < words)
                flags[w0 + 1] = (uint32_t)(mask >> 32);
        }
        count += (unsigned long long)__popcll(mask);
    }
    if (n_bad && lane == 0 && count)
        atomicAdd(n_bad, count);
}

template <int M, typename T>
__global__ __launch_bounds__(kPermThreads) void k_permute_scale_fused(
    const T *__restrict__ c, const int32_t *__restrict__ perm, const int64_t *__restrict__ scale,
    const int64_t *__restrict__ add, void *__restrict__ dhat, int out64,
    uint32_t *__restrict__ flags, unsigned long long *__restrict__ n_bad, int64_t N, int l, int r)
{
    perm_fused_range<M, T>(c, perm, scale, add, dhat, out64, flags, n_bad, N, l, r, 0, N,
                           (int64_t)blockIdx.x * kPermThreads,
                           (int64_t)gridDim.x * kPermThreads);
}

} // namespace
} // namespace ne
