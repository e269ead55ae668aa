// ne_abft_rc.hip -- row/column checksum ABFT (the "RC-check" of Huang and
// Abraham) over M independent subblock products d_m = c_m G, the second
// ABFT method the paper's GEMM comparison measures (section V).
//
// For each subblock the checksums of the inputs give the row and column
// sums the product must have:
//     sum_p d_m[i][p] = sum_k c_m[i][k] (G e)[k]       (row i)
//     sum_i d_m[i][p] = sum_k (e^T c_m)[k] G[k][p]     (column p)
// with e the all-ones vector.  A position whose value is wrong makes its
// row and its column disagree; up to three wrong positions of a subblock
// always leave at least one row or column in disagreement.  All sums are
// exact in 64-bit integers for the sizes the entry points admit.
//
// Kernels, in launch order (the GEMM is the library's plain int8 GEMM):
//   k_rc_zero      clears the accumulation buffers and the flag words
//   k_rc_colsums   e^T c_m (int32 [M][K]) and G e (int32 [K]), 32-row
//                  chunks added with atomics
//   k_rc_rows      one wavefront per row: sum of d and the reference sum
//   k_rc_cols      column sums of d over 32-row chunks into csum
//   k_rc_colref    one workgroup per column of G: the reference column sums,
//                  compared with csum; flags
#include <algorithm>

#include "ne_internal.h"
#include "ne_rc.h"

namespace ne {
namespace {

constexpr int kRcChunk = 32; // rows per block of the column sums

__host__ __device__ inline int64_t rc_align16(int64_t b)
{
    return (b + 15) / 16 * 16;
}

struct RcWs {
    int32_t *as;    // [M][K] column sums of each subblock of c
    int32_t *bs;    // [K] row sums of G (G e), right after as
    int64_t *csum;  // [M][N] column sums of d
};

RcWs rc_ws(void *ws, int64_t M, int64_t K)
{
    RcWs w;
    w.as = (int32_t *)ws;
    w.bs = w.as + M * K;
    w.csum = (int64_t *)((char *)ws + rc_align16((M * K + K) * 4));
    return w;
}

__global__ __launch_bounds__(256) void k_rc_zero(RcWs w, int64_t n32, int64_t n64,
                                                 uint32_t *row_flags, int64_t nrf,
                                                 uint32_t *col_flags, int64_t ncf)
{
    const int64_t stride = (int64_t)gridDim.x * 256;
    const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
    for (int64_t i = t; i < n32; i += stride)
        w.as[i] = 0; // as and bs
    for (int64_t i = t; i < n64; i += stride)
        w.csum[i] = 0;
    for (int64_t i = t; i < nrf; i += stride)
        row_flags[i] = 0;
    for (int64_t i = t; i < ncf; i += stride)
        col_flags[i] = 0;
}

// Block (x, y, z): columns k = 256 x + tid of the rows [32 z, 32 z + 32) of
// subblock y of c (y < M) or of G^T (y == M: its rows are the columns of G,
// so the column sums of G^T are G e).  Every lane loads (from a clamped
// row) before any value is used.
__global__ __launch_bounds__(256) void k_rc_colsums(const int8_t *c, const int8_t *Gt, RcWs w,
                                                    int64_t M, int64_t n, int64_t K, int64_t N)
{
    const int64_t k = (int64_t)blockIdx.x * 256 + threadIdx.x;
    const int64_t y = blockIdx.y;
    const int64_t rows = y < M ? n : N;
    const int64_t r0 = (int64_t)blockIdx.z * kRcChunk;
    if (k >= K || r0 >= rows)
        return;
    const int8_t *src = y < M ? c + y * n * K : Gt;
    int32_t v[kRcChunk];
#pragma unroll
    for (int j = 0; j < kRcChunk; ++j) {
        const int64_t r = r0 + j < rows ? r0 + j : r0;
        v[j] = src[r * K + k];
    }
    int32_t sum = 0;
#pragma unroll
    for (int j = 0; j < kRcChunk; ++j)
        sum += r0 + j < rows ? v[j] : 0;
    atomicAdd(y < M ? &w.as[y * K + k] : &w.bs[k], sum);
}

__device__ __forceinline__ int64_t rc_wave_sum(int64_t x)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1)
        x += __shfl_xor(x, off);
    return x;
}

// Signed byte j of a 32-bit word.
__device__ __forceinline__ int32_t rc_byte(uint32_t w, int j)
{
    return (int32_t)(w << (24 - 8 * j)) >> 24;
}

// One wavefront per row R = m n + i of the stacked product.  VEC: rows of
// d, c and the row sums of G are 16-byte aligned (N % 4 == 0, K % 16 == 0),
// read in 16-byte loads.
template <bool VEC>
__global__ __launch_bounds__(256) void k_rc_rows(const int8_t *c, const int32_t *d, RcWs w,
                                                 uint32_t *row_flags, unsigned long long *n_bad,
                                                 int64_t M, int64_t n, int64_t K, int64_t N)
{
    const int64_t R = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (R >= M * n)
        return; // uniform over the wavefront
    const int8_t *a = c + R * K;
    const int32_t *dr = d + R * N;
    int64_t got = 0, ref = 0;
    if constexpr (VEC) {
        for (int64_t q = lane; q < N / 4; q += 64) {
            const int4 x = ((const int4 *)dr)[q];
            got += (int64_t)x.x + x.y + (int64_t)x.z + x.w;
        }
        for (int64_t q = lane; q < K / 16; q += 64) {
            const uint4 av = ((const uint4 *)a)[q];
            const int4 *b4 = (const int4 *)(w.bs + 16 * q);
            const int4 b0 = b4[0], b1 = b4[1], b2 = b4[2], b3 = b4[3];
            const uint32_t aw[4] = {av.x, av.y, av.z, av.w};
            const int32_t bv[16] = {b0.x, b0.y, b0.z, b0.w, b1.x, b1.y, b1.z, b1.w,
                                    b2.x, b2.y, b2.z, b2.w, b3.x, b3.y, b3.z, b3.w};
#pragma unroll
            for (int j = 0; j < 16; ++j)
                ref += (int64_t)rc_byte(aw[j >> 2], j & 3) * bv[j];
        }
    } else {
        for (int64_t p = lane; p < N; p += 64)
            got += dr[p];
        for (int64_t k = lane; k < K; k += 64)
            ref += (int64_t)a[k] * w.bs[k];
    }
    got = rc_wave_sum(got);
    ref = rc_wave_sum(ref);
    if (lane == 0 && got != ref) {
        const int64_t m = R / n, i = R - m * n;
        if (row_flags)
            atomicOr(&row_flags[m * ((n + 31) / 32) + i / 32], 1u << (i & 31));
        if (n_bad)
            atomicAdd(n_bad, 1ull);
    }
}

// Block (x, m, z): columns p = 256 x + tid, rows [32 z, 32 z + 32) of
// subblock m of d, added into csum.
__global__ __launch_bounds__(256) void k_rc_cols(const int32_t *d, RcWs w, int64_t n, int64_t N)
{
    const int64_t p = (int64_t)blockIdx.x * 256 + threadIdx.x;
    const int64_t m = blockIdx.y;
    const int64_t r0 = (int64_t)blockIdx.z * kRcChunk;
    if (p >= N || r0 >= n)
        return;
    const int32_t *dm = d + m * n * N;
    int32_t v[kRcChunk];
#pragma unroll
    for (int j = 0; j < kRcChunk; ++j) {
        const int64_t r = r0 + j < n ? r0 + j : r0;
        v[j] = dm[r * N + p];
    }
    int64_t sum = 0;
#pragma unroll
    for (int j = 0; j < kRcChunk; ++j)
        sum += r0 + j < n ? (int64_t)v[j] : 0;
    atomicAdd((unsigned long long *)&w.csum[m * N + p], (unsigned long long)sum);
}

// One workgroup per column p of G (row p of G^T), after k_rc_cols: the
// reference sum_k (e^T c_m)[k] G[k][p] of every subblock m (eight per pass
// over the row; each thread a stride of k, then a workgroup sum) against
// the column sum of d in csum[m][p].  A differing column sets its flag bit
// (the flag words were cleared by k_rc_zero).
__global__ __launch_bounds__(256) void k_rc_colref(const int8_t *Gt, RcWs w,
                                                   uint32_t *col_flags, unsigned long long *n_bad,
                                                   int64_t M, int64_t K, int64_t N)
{
    __shared__ int64_t part[4][8];
    const int64_t p = blockIdx.x;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int8_t *g = Gt + p * K;
    for (int64_t m0 = 0; m0 < M; m0 += 8) {
        int64_t acc[8] = {0, 0, 0, 0, 0, 0, 0, 0};
#pragma unroll 4
        for (int64_t k = tid; k < K; k += 256) {
            const int64_t gv = g[k];
#pragma unroll
            for (int j = 0; j < 8; ++j)
                if (m0 + j < M)
                    acc[j] += (int64_t)w.as[(m0 + j) * K + k] * gv;
        }
#pragma unroll
        for (int j = 0; j < 8; ++j)
            acc[j] = rc_wave_sum(acc[j]);
        if (lane == 0)
#pragma unroll
            for (int j = 0; j < 8; ++j)
                part[wave][j] = acc[j];
        __syncthreads();
        if (tid < 8 && m0 + tid < M) {
            const int64_t m = m0 + tid;
            const int64_t ref = part[0][tid] + part[1][tid] + part[2][tid] + part[3][tid];
            if (w.csum[m * N + p] != ref) {
                if (col_flags)
                    atomicOr(&col_flags[m * ((N + 31) / 32) + p / 32], 1u << (p & 31));
                if (n_bad)
                    atomicAdd(n_bad, 1ull);
            }
        }
        __syncthreads();
    }
}

unsigned rc_blocks(int64_t threads)
{
    return (unsigned)std::max<int64_t>(1, (threads + 255) / 256);
}

} // namespace

int64_t rc_workspace_bytes(int64_t M, int64_t K, int64_t N)
{
    return rc_align16((M * K + K) * 4) + M * N * 8;
}

int launch_abft_rc(const int8_t *c, const int8_t *Gt, int32_t *d, uint32_t *row_flags,
                   uint32_t *col_flags, unsigned long long *n_bad, int64_t M, int64_t n, int64_t K,
                   int64_t N, void *ws, bool gemm, hipStream_t s)
{
    const RcWs w = rc_ws(ws, M, K);
    const int64_t nrf = row_flags ? M * ((n + 31) / 32) : 0;
    const int64_t ncf = col_flags ? M * ((N + 31) / 32) : 0;
    const int64_t zmax = std::max({(M + 1) * K, M * N, nrf, ncf});
    k_rc_zero<<<std::min<unsigned>(2048, rc_blocks(zmax)), 256, 0, s>>>(w, (M + 1) * K, M * N,
                                                                         row_flags, nrf, col_flags,
                                                                         ncf);
    const unsigned chunks = (unsigned)((std::max(n, N) + kRcChunk - 1) / kRcChunk);
    k_rc_colsums<<<dim3(rc_blocks(K), (unsigned)(M + 1), chunks), 256, 0, s>>>(c, Gt, w, M, n, K,
                                                                                 N);
    if (gemm) {
        const int rc = launch_gemm_plain(c, Gt, d, M * n, K, N, s);
        if (rc != NE_OK)
            return rc;
    }
    const bool vec = N % 4 == 0 && K % 16 == 0 && ((uintptr_t)c & 15) == 0 &&
                     ((uintptr_t)d & 15) == 0 && ((uintptr_t)w.bs & 15) == 0;
    if (vec)
        k_rc_rows<true><<<rc_blocks(M * n * 64), 256, 0, s>>>(c, d, w, row_flags, n_bad, M, n, K, N);
    else
        k_rc_rows<false><<<rc_blocks(M * n * 64), 256, 0, s>>>(c, d, w, row_flags, n_bad, M, n, K,
                                                               N);
    k_rc_cols<<<dim3(rc_blocks(N), (unsigned)M, (unsigned)((n + kRcChunk - 1) / kRcChunk)), 256, 0,
                s>>>(d, w, n, N);
    k_rc_colref<<<(unsigned)N, 256, 0, s>>>(Gt, w, col_flags, n_bad, M, K, N);
    return launch_status();
}

} // namespace ne
