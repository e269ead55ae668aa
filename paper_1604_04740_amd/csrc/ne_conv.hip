// ne_conv.hip -- launchers of the circular-convolution entry points
// (device code in ne_conv_impl.h: Toeplitz x Hankel blocks on the int8
// matrix cores).  One workgroup per block of 1024 outputs; the staged form
// takes up to eight streams per workgroup (grid y covers the rest).
#include "ne_conv_impl.h"

namespace ne {
namespace {

template <int M>
int launch_fused_m(const ConvJob &J, unsigned blocks, hipStream_t s)
{
    k_conv_fused<M><<<blocks, kCvThreads, 0, s>>>(J);
    return launch_status();
}

template <int G>
int launch_staged_g(const ConvJob &J, unsigned blocks, unsigned groups, hipStream_t s)
{
    k_conv_staged<G><<<dim3(blocks, groups), kCvThreads, 0, s>>>(J);
    return launch_status();
}

} // namespace

int launch_circconv_eps(const int64_t *eps, int digits, const int8_t *g, int64_t *delta,
                        int64_t N, int M, hipStream_t s)
{
    ConvJob J{};
    J.x = eps;
    J.x_dtype = NE_I64;
    J.digits = digits;
    J.g = g;
    J.out = delta;
    J.out64 = 1;
    J.N = N;
    J.M = M;
    const unsigned blocks = (unsigned)((N + kCvBlock - 1) / kCvBlock);
    switch (M) {
    case 3: return launch_staged_g<3>(J, blocks, 1, s);
    case 4: return launch_staged_g<4>(J, blocks, 1, s);
    case 5: return launch_staged_g<5>(J, blocks, 1, s);
    case 6: return launch_staged_g<6>(J, blocks, 1, s);
    case 7: return launch_staged_g<7>(J, blocks, 1, s);
    case 8: return launch_staged_g<8>(J, blocks, 1, s);
    default:
        if (M > 8 && M <= kMaxStreamsElementwise)
            return launch_staged_g<kCvMaxSlots>(J, blocks,
                                                (unsigned)((M + kCvMaxSlots - 1) / kCvMaxSlots), s);
        return NE_EUNSUP;
    }
}

int launch_circconv_fused(const void *c, int c_dtype, int c_bits, const int8_t *g, void *dhat,
                          int out64, uint32_t *flags, unsigned long long *n_bad, int64_t N, int M,
                          int l, int r, hipStream_t s)
{
    ConvJob J{};
    J.x = c;
    J.x_dtype = c_dtype;
    J.digits = cv_digits(c_bits);
    J.g = g;
    J.out = dhat;
    J.out64 = out64;
    J.flags = flags;
    J.n_bad = n_bad;
    J.N = N;
    J.M = M;
    J.l = l;
    J.r = r;
    const unsigned blocks = (unsigned)((N + kCvBlock - 1) / kCvBlock);
    switch (M) {
    case 3: return launch_fused_m<3>(J, blocks, s);
    case 4: return launch_fused_m<4>(J, blocks, s);
    case 5: return launch_fused_m<5>(J, blocks, s);
    case 6: return launch_fused_m<6>(J, blocks, s);
    case 7: return launch_fused_m<7>(J, blocks, s);
    case 8: return launch_fused_m<8>(J, blocks, s);
    default: return NE_EUNSUP;
    }
}

} // namespace ne
