// ne_perm_impl.h -- fused permute / scale / add device code (shared by the
// element-wise entry point and the batched persistent kernel).
#pragma once

#include "ne_arith.h"
#include "ne_internal.h"

namespace ne {
namespace {

constexpr int kPermThreads = 256;

// Row layout of the gather source: the M inputs of one position stored
// next to each other, in slot order (slot s = stream (r + s) mod M), padded
// to whole 64-bit words, so that one position's gather is one or two
// aligned loads instead of M loads from M different cache lines.
template <int M, typename T>
struct PermRow {
    static constexpr int Q = (M * (int)sizeof(T) + 7) / 8; // 64-bit words per row
};

// Rows of positions [first, last), threads from `first + start`, step
// `stride`: rows[n][.] = c[(r + s) mod M][n] for every slot s.
template <int M, typename T>
__device__ __forceinline__ void perm_pack_range(const T *__restrict__ c,
                                                uint64_t *__restrict__ rows, int64_t N, int r,
                                                int64_t first, int64_t last, int64_t start,
                                                int64_t stride)
{
    constexpr int Q = PermRow<M, T>::Q;
    for (int64_t n = first + start + threadIdx.x; n < last; n += stride) {
        T v[Q * 8 / sizeof(T)] = {};
#pragma unroll
        for (int s = 0; s < M; ++s)
            v[s] = c[(int64_t)((r + s) % M) * N + n];
        uint64_t q[Q];
        __builtin_memcpy(q, v, sizeof q);
#pragma unroll
        for (int k = 0; k < Q; ++k)
            rows[n * Q + k] = q[k];
    }
}

// Fused permute / scale / add: for every position n, gather the M input
// words at perm[n] (from c, or from its rows when `rows` is given), entangle
// them (slot s holds stream (r + s) mod M), apply
// delta = scale * eps + (2^l + 1) add, disentangle and check.  The
// entangled words exist only in registers.  Wavefronts cover whole flag
// words (64 consecutive positions).
// Positions [first, last) (first a multiple of 64), visited by the
// workgroup's 256 threads starting at `first + start`, step `stride`.
// ENT: the rows already hold entangled 64-bit words (the output of an
// earlier operation of a series), so the entangle step is skipped.
// W: the word (int64_t, w = 64; int32_t, w = 32, then dhat is int32).
template <int M, typename T, bool ENT = false, typename W = int64_t>
__device__ __forceinline__ void perm_fused_range(
    const T *__restrict__ c, const uint64_t *__restrict__ rows, const int32_t *__restrict__ perm,
    const W *__restrict__ scale, const W *__restrict__ add, void *__restrict__ dhat,
    int out64, uint32_t *__restrict__ flags, unsigned long long *__restrict__ n_bad, int64_t N,
    int l, int r, int64_t first, int64_t last, int64_t start, int64_t stride)
{
    constexpr int Q = PermRow<M, T>::Q;
    // U groups of 64 positions per wavefront per round: all their gathers
    // are issued before the first is used (random loads need many in flight)
    constexpr int U = Q <= 2 ? 4 : 2;
    const int lane = threadIdx.x & 63;
    const int64_t words = (N + 31) / 32;
    unsigned long long count = 0;
    for (int64_t base0 = first + start + (threadIdx.x & ~63); base0 < last;
         base0 += U * stride) {
        int64_t src[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int64_t n = base0 + u * stride + lane;
            int64_t x = n < last ? perm[n] : 0;
            src[u] = x < 0 ? 0 : (x >= N ? N - 1 : x);
        }
        int64_t v[U][M]; // v[u][s] = input of stream (r + s) mod M, i.e. slot order
        if (rows) {
            uint64_t q[U][Q];
            if constexpr (ENT && Q % 2 == 0) {
                // entangled rows start 16-byte aligned: 16-byte loads
                typedef unsigned long long v2u __attribute__((ext_vector_type(2)));
                const v2u *rv = (const v2u *)rows;
#pragma unroll
                for (int u = 0; u < U; ++u)
#pragma unroll
                    for (int k = 0; k < Q / 2; ++k) {
                        const v2u t = rv[src[u] * (Q / 2) + k];
                        q[u][2 * k] = t.x;
                        q[u][2 * k + 1] = t.y;
                    }
            } else {
#pragma unroll
                for (int u = 0; u < U; ++u)
#pragma unroll
                    for (int k = 0; k < Q; ++k)
                        q[u][k] = rows[src[u] * Q + k];
            }
#pragma unroll
            for (int u = 0; u < U; ++u) {
                T t[Q * 8 / sizeof(T)];
                __builtin_memcpy(t, q[u], sizeof q[u]);
#pragma unroll
                for (int s = 0; s < M; ++s)
                    v[u][s] = (int64_t)t[s];
            }
        } else {
#pragma unroll
            for (int u = 0; u < U; ++u)
#pragma unroll
                for (int s = 0; s < M; ++s)
                    v[u][s] = (int64_t)c[(int64_t)((r + s) % M) * N + src[u]];
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int64_t base = base0 + u * stride;
            if (base >= last)
                break; // uniform: the same for the whole wavefront
            const int64_t n = base + lane;
            bool f = false;
            if (n < last) {
                typedef typename UWord<W>::type U;
                const U sc = scale ? (U)scale[n] : (U)1;
                const U a = add ? (U)entangle_word(add[n], add[n], l) : (U)0;
                W d[M], o[M];
#pragma unroll
                for (int s = 0; s < M; ++s) {
                    if constexpr (ENT)
                        d[s] = (W)(sc * (U)v[u][s] + a);
                    else
                        d[s] = (W)(sc * (U)entangle_word((W)v[u][s], (W)v[u][(s + M - 1) % M], l) +
                                   a);
                }
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
    }
    if (n_bad && lane == 0 && count)
        atomicAdd(n_bad, count);
}

template <int M, typename T>
__global__ __launch_bounds__(kPermThreads) void k_perm_pack(const T *__restrict__ c,
                                                            uint64_t *__restrict__ rows,
                                                            int64_t N, int r)
{
    perm_pack_range<M, T>(c, rows, N, r, 0, N, (int64_t)blockIdx.x * kPermThreads,
                          (int64_t)gridDim.x * kPermThreads);
}

template <int M, typename T, bool ENT = false, typename W = int64_t>
__global__ __launch_bounds__(kPermThreads) void k_permute_scale_fused(
    const T *__restrict__ c, const uint64_t *__restrict__ rows, const int32_t *__restrict__ perm,
    const W *__restrict__ scale, const W *__restrict__ add, void *__restrict__ dhat,
    int out64, uint32_t *__restrict__ flags, unsigned long long *__restrict__ n_bad, int64_t N,
    int l, int r)
{
    perm_fused_range<M, T, ENT, W>(c, rows, perm, scale, add, dhat, out64, flags, n_bad, N, l, r, 0, N,
                           (int64_t)blockIdx.x * kPermThreads,
                           (int64_t)gridDim.x * kPermThreads);
}

} // namespace
} // namespace ne
