// ne_conv.hip -- circular convolution of entangled streams with a shared
// kernel g (section II, the star operator), on 64-bit words:
//     delta[m][t] = sum_j eps[m][(t - j) mod N] * g[j]   (mod 2^64).
//
// Direct evaluation on the vector ALUs.  A workgroup owns 256 consecutive
// output positions and walks the kernel in 256-tap tiles; each tile stages
// the 256 taps and the 511 input words they touch in LDS, so every global
// word is read once per tile and each thread does 256 multiply-adds per
// stream from LDS.
//
//   k_circconv_direct   staged: one stream per workgroup row, eps given
//   k_circconv_fused<M> fused (device code in ne_conv_impl.h)
#include "ne_conv_impl.h"

namespace ne {
namespace {

constexpr int kT = 256;

__global__ __launch_bounds__(kT) void k_circconv_direct(const int64_t *__restrict__ eps,
                                                        const int8_t *__restrict__ g,
                                                        int64_t *__restrict__ delta, int64_t N)
{
    __shared__ int64_t xs[2 * kT];
    __shared__ int32_t gs[kT];
    const int tid = threadIdx.x;
    const int64_t m = blockIdx.y;
    const int64_t t0 = (int64_t)blockIdx.x * kT;
    const int64_t *x = eps + m * N;
    uint64_t acc = 0;
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
                xs[i] = x[idx];
            }
        }
        __syncthreads();
        const int taps = (N - j0 < kT) ? (int)(N - j0) : kT;
        for (int jj = 0; jj < taps; ++jj)
            acc += (uint64_t)xs[tid - jj + kT - 1] * (uint64_t)(int64_t)gs[jj];
        __syncthreads();
    }
    if (t0 + tid < N)
        delta[m * N + t0 + tid] = (int64_t)acc;
}

template <int M>
int launch_fused_m(const void *c, int c_dtype, const int8_t *g, void *dhat, int out64,
                   uint32_t *flags, unsigned long long *n_bad, int64_t N, int l, int r,
                   hipStream_t s)
{
    const dim3 grid((unsigned)((N + kT - 1) / kT));
    if (c_dtype == NE_I8)
        k_circconv_fused<M, int8_t><<<grid, kT, 0, s>>>((const int8_t *)c, g, dhat, out64, flags,
                                                         n_bad, N, l, r);
    else if (c_dtype == NE_I32)
        k_circconv_fused<M, int32_t><<<grid, kT, 0, s>>>((const int32_t *)c, g, dhat, out64,
                                                          flags, n_bad, N, l, r);
    else
        k_circconv_fused<M, int64_t><<<grid, kT, 0, s>>>((const int64_t *)c, g, dhat, out64,
                                                          flags, n_bad, N, l, r);
    return launch_status();
}

} // namespace

int launch_circconv_eps(const int64_t *eps, int digits, const int8_t *g, int64_t *delta,
                        int64_t N, int M, hipStream_t s)
{
    (void)digits;
    const dim3 grid((unsigned)((N + kT - 1) / kT), (unsigned)M);
    k_circconv_direct<<<grid, kT, 0, s>>>(eps, g, delta, N);
    return launch_status();
}

int launch_circconv_fused(const void *c, int c_dtype, const int8_t *g, void *dhat, int out64,
                          uint32_t *flags, unsigned long long *n_bad, int64_t N, int M, int l,
                          int r, hipStream_t s)
{
    switch (M) {
    case 3: return launch_fused_m<3>(c, c_dtype, g, dhat, out64, flags, n_bad, N, l, r, s);
    case 4: return launch_fused_m<4>(c, c_dtype, g, dhat, out64, flags, n_bad, N, l, r, s);
    case 5: return launch_fused_m<5>(c, c_dtype, g, dhat, out64, flags, n_bad, N, l, r, s);
    case 6: return launch_fused_m<6>(c, c_dtype, g, dhat, out64, flags, n_bad, N, l, r, s);
    case 7: return launch_fused_m<7>(c, c_dtype, g, dhat, out64, flags, n_bad, N, l, r, s);
    case 8: return launch_fused_m<8>(c, c_dtype, g, dhat, out64, flags, n_bad, N, l, r, s);
    default: return NE_EUNSUP;
    }
}

} // namespace ne
