// ne_internal.h -- declarations shared by the library's translation units
// (launchers called by the C-ABI layer in ne_api.hip).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "ne.h"

namespace ne {

// Maximum number of streams handled by the element-wise kernels.
constexpr int kMaxStreamsElementwise = 16;
// Maximum number of streams handled by the fused GEMM.
constexpr int kMaxStreamsFused = 8;
// Largest K (or convolution length) whose int8 x int8 digit products,
// summed, always fit an int32 accumulator: K * 128 * 128 <= 2^31 - 1.
constexpr int64_t kMaxK = 131071;

struct StreamPtrs {
    const int64_t *p[kMaxStreamsElementwise];
};

// ---- element-wise kernels (ne_elementwise.hip) ----
// w = 64: words (eps, delta, d_hat, scale, add) are int64; w = 32: int32.
int launch_entangle(const void *c, int c_dtype, void *eps, int64_t N, int M, int l, int w,
                    hipStream_t s);
int launch_disentangle_check(const void *delta, void *dhat, uint32_t *flags,
                             unsigned long long *n_bad, int64_t N, int M, int l, int r, int w,
                             hipStream_t s);
int launch_recover(const StreamPtrs &delta, int lost, void *dhat, void *rebuilt, int64_t N, int M,
                   int l, int w, hipStream_t s);
int launch_permute_scale(const void *eps, const int32_t *perm, const void *scale, const void *add,
                         void *delta, int64_t N, int M, int l, int w, hipStream_t s);

// Bytes of the row copy (M inputs per position, 64-bit padded) that the
// fused permutation gathers from when given a workspace.
int64_t permute_rows_bytes(int64_t N, int M, int c_dtype);
int launch_permute_scale_fused(const void *c, int c_dtype, const int32_t *perm, const void *scale,
                               const void *add, void *dhat, int out64, uint32_t *flags,
                               unsigned long long *n_bad, int64_t N, int M, int l, int r, int w,
                               void *rows, hipStream_t s);

// Gather of position-major entangled rows [N][M] (no entangle), then
// disentangle and check.
int launch_permute_rows_check(const int64_t *rows, const int32_t *perm, void *dhat, int out64,
                              uint32_t *flags, unsigned long long *n_bad, int64_t N, int M, int l,
                              int r, hipStream_t s);

// ---- matrix-core GEMMs (ne_gemm.hip) ----
int launch_gemm_plain(const int8_t *A, const int8_t *Bt, int32_t *C, int64_t R, int64_t K,
                      int64_t N, hipStream_t s);
int launch_gemm_eps(const int64_t *eps, int digits, const int8_t *Bt, int64_t *delta, int64_t R,
                    int64_t K, int64_t N, hipStream_t s);
int launch_gemm_fused(const int8_t *c, const int8_t *Bt, void *dhat, int out64, uint32_t *flags,
                      unsigned long long *n_bad, int64_t n, int64_t K, int64_t N, int M, int l,
                      int r, const ne_inject_t *inj, hipStream_t s);
// GEMM head of a series: entangled products, scale / add, position-major
// rows [n * N][M] out.
int launch_series_gemm(const int8_t *c, const int8_t *Bt, const int64_t *scale, const int64_t *add,
                       int64_t *rows, int64_t n, int64_t K, int64_t N, int M, int l, int r,
                       hipStream_t s);
// ws: 2 n K bytes for the checksum digit planes (DMA pipeline), or NULL
// (the checksum built in the prologue).
int launch_gemm_abft(const int8_t *c, const int8_t *Bt, int32_t *d, uint32_t *flags,
                     unsigned long long *n_bad, int64_t n, int64_t K, int64_t N, int M, void *ws,
                     hipStream_t s);

// ---- circular convolution (ne_conv.hip) ----
// Split of the taps over workgroups when a workspace is given: S splits of
// KC taps each, bytes of 64-bit partial sums (S <= 1: no split).
struct ConvSplit {
    int S, KC;
    int64_t bytes;
};
ConvSplit conv_split(int64_t N, int M, bool fused);
int launch_circconv_eps(const int64_t *eps, int digits, const int8_t *g, int64_t *delta,
                        int64_t N, int M, void *ws, hipStream_t s);
int launch_circconv_fused(const void *c, int c_dtype, int c_bits, const int8_t *g, void *dhat,
                          int out64, uint32_t *flags, unsigned long long *n_bad, int64_t N, int M,
                          int l, int r, void *ws, hipStream_t s);
// Linear convolution of N samples with L taps (N + L - 1 outputs per stream).
// ws: linconv_workspace_bytes(N, L, M, digits) bytes (plane-staged) or NULL
int64_t linconv_workspace_bytes(int64_t N, int64_t L, int M, int digits);
int launch_linconv_eps(const int64_t *eps, int digits, const int8_t *g, int64_t L, int64_t *delta,
                       int64_t N, int M, void *ws, hipStream_t s);
int launch_linconv_fused(const void *c, int c_dtype, int c_bits, const int8_t *g, int64_t L,
                         void *dhat, int out64, uint32_t *flags, unsigned long long *n_bad,
                         int64_t N, int M, int l, int r, void *ws, hipStream_t s);

// Grid size for grid-stride element-wise kernels.
inline unsigned grid_for(int64_t work, int threads)
{
    int64_t blocks = (work + threads - 1) / threads;
    if (blocks > 8192)
        blocks = 8192;
    if (blocks < 1)
        blocks = 1;
    return (unsigned)blocks;
}

inline int launch_status()
{
    return hipGetLastError() == hipSuccess ? NE_OK : NE_ELAUNCH;
}

} // namespace ne
