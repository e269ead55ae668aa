// ne_conv.hip -- launchers of the circular-convolution entry points
// (device code in ne_conv_impl.h: Toeplitz x Hankel blocks on the int8
// matrix cores).  Without a workspace: one workgroup per block of 1024
// outputs (the staged form takes up to eight streams per workgroup, grid z
// covers the rest).  With a workspace: the taps of every block are split
// over several workgroups so that the launch fills the chip, each writes
// 64-bit partial sums, and a second kernel adds them and finishes.
#include "ne_conv_impl.h"

#ifndef NE_CONV_TARGET_WGS
#define NE_CONV_TARGET_WGS 256 // about one workgroup per compute unit
#endif

namespace ne {

ConvSplit conv_split(int64_t N, int M, bool fused)
{
    ConvSplit c{};
    const int64_t blocks = (N + kCvBlock - 1) / kCvBlock;
    const int64_t groups = fused ? 1 : (M + kCvMaxSlots - 1) / kCvMaxSlots;
    const int64_t steps = (N + kCvStep - 1) / kCvStep;
    const int64_t target = NE_CONV_TARGET_WGS; // workgroups in total
    int64_t S = (target + blocks * groups - 1) / (blocks * groups);
    if (S > steps)
        S = steps;
    if (S <= 1 || N <= 0)
        return c;
    const int64_t per = (steps + S - 1) / S; // steps per split
    c.KC = (int)(per * kCvStep);
    c.S = (int)((steps + per - 1) / per);
    c.bytes = (int64_t)c.S * M * blocks * kCvBlock * 8;
    return c;
}

namespace {

template <int M>
int launch_fused_m(const ConvJob &J, unsigned blocks, const ConvSplit &sp, uint64_t *ws,
                   hipStream_t s)
{
    if (sp.S > 1) {
        k_conv_part<M, true><<<dim3(blocks, sp.S, 1), kCvThreads, 0, s>>>(J, ws, sp.KC, M);
        if (launch_status())
            return NE_ELAUNCH;
        k_conv_reduce<M, true><<<(unsigned)((J.N + 255) / 256), 256, 0, s>>>(
            J, ws, sp.S, (int64_t)blocks * kCvBlock);
        return launch_status();
    }
    k_conv_fused<M><<<blocks, kCvThreads, 0, s>>>(J);
    return launch_status();
}

template <int G>
int launch_staged_g(const ConvJob &J, unsigned blocks, unsigned groups, const ConvSplit &sp,
                    uint64_t *ws, hipStream_t s)
{
    if (sp.S > 1) {
        k_conv_part<G, false><<<dim3(blocks, sp.S, groups), kCvThreads, 0, s>>>(J, ws, sp.KC,
                                                                                J.M);
        if (launch_status())
            return NE_ELAUNCH;
        k_conv_reduce<1, false><<<(unsigned)((J.N + 255) / 256), 256, 0, s>>>(
            J, ws, sp.S, (int64_t)blocks * kCvBlock);
        return launch_status();
    }
    k_conv_staged<G><<<dim3(blocks, groups), kCvThreads, 0, s>>>(J);
    return launch_status();
}

} // namespace

int launch_circconv_eps(const int64_t *eps, int digits, const int8_t *g, int64_t *delta,
                        int64_t N, int M, void *ws, hipStream_t s)
{
    const ConvSplit sp = ws ? conv_split(N, M, false) : ConvSplit{};
    ConvJob J{};
    J.x = eps;
    J.x_dtype = NE_I64;
    J.digits = digits;
    J.g = g;
    J.out = delta;
    J.out64 = 1;
    J.N = N;
    J.L = N;
    J.Nout = N;
    J.M = M;
    const unsigned blocks = (unsigned)((N + kCvBlock - 1) / kCvBlock);
    uint64_t *w = (uint64_t *)ws;
    switch (M) {
    case 3: return launch_staged_g<3>(J, blocks, 1, sp, w, s);
    case 4: return launch_staged_g<4>(J, blocks, 1, sp, w, s);
    case 5: return launch_staged_g<5>(J, blocks, 1, sp, w, s);
    case 6: return launch_staged_g<6>(J, blocks, 1, sp, w, s);
    case 7: return launch_staged_g<7>(J, blocks, 1, sp, w, s);
    case 8: return launch_staged_g<8>(J, blocks, 1, sp, w, s);
    default:
        if (M > 8 && M <= kMaxStreamsElementwise)
            return launch_staged_g<kCvMaxSlots>(
                J, blocks, (unsigned)((M + kCvMaxSlots - 1) / kCvMaxSlots), sp, w, s);
        return NE_EUNSUP;
    }
}

int launch_circconv_fused(const void *c, int c_dtype, int c_bits, const int8_t *g, void *dhat,
                          int out64, uint32_t *flags, unsigned long long *n_bad, int64_t N, int M,
                          int l, int r, void *ws, hipStream_t s)
{
    const ConvSplit sp = ws ? conv_split(N, M, true) : ConvSplit{};
    uint64_t *w = (uint64_t *)ws;
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
    J.L = N;
    J.Nout = N;
    J.M = M;
    J.l = l;
    J.r = r;
    const unsigned blocks = (unsigned)((N + kCvBlock - 1) / kCvBlock);
    switch (M) {
    case 3: return launch_fused_m<3>(J, blocks, sp, w, s);
    case 4: return launch_fused_m<4>(J, blocks, sp, w, s);
    case 5: return launch_fused_m<5>(J, blocks, sp, w, s);
    case 6: return launch_fused_m<6>(J, blocks, sp, w, s);
    case 7: return launch_fused_m<7>(J, blocks, sp, w, s);
    case 8: return launch_fused_m<8>(J, blocks, sp, w, s);
    default: return NE_EUNSUP;
    }
}

// ---------------------------------------------------- linear convolution

// Workspace of the plane-staged linear form: the digit planes of M streams
// and the padded copy of g.
int64_t linconv_workspace_bytes(int64_t N, int64_t L, int M, int digits)
{
    return (int64_t)M * digits * cv_plane_bytes(N, L) + ((L + 2 * kCvGPad + 15) / 16) * 16;
}

namespace {
// Planes and gpad in ws (linconv_workspace_bytes bytes): run the pre-pass
// and point J at them.
void linconv_planes(ConvJob &J, void *ws, hipStream_t s)
{
    J.P = cv_plane_bytes(J.N, J.L);
    J.pad = cv_plane_pad(J.L);
    int8_t *planes = (int8_t *)ws;
    int8_t *gpad = planes + (int64_t)J.M * J.digits * J.P;
    J.planes = planes;
    J.gpad = gpad;
    const int64_t dw = std::max(J.P, J.L + 2 * kCvGPad + 3) / 4;
    k_cv_planes<<<dim3((unsigned)((dw + 255) / 256), (unsigned)(J.M + 1)), 256, 0, s>>>(J, planes,
                                                                                         gpad);
}
} // namespace

int launch_linconv_eps(const int64_t *eps, int digits, const int8_t *g, int64_t L, int64_t *delta,
                       int64_t N, int M, void *ws, hipStream_t s)
{
    ConvJob J{};
    J.x = eps;
    J.x_dtype = NE_I64;
    J.digits = digits;
    J.g = g;
    J.out = delta;
    J.out64 = 1;
    J.N = N;
    J.L = L;
    J.Nout = N + L - 1;
    J.M = M;
    const unsigned blocks = (unsigned)((J.Nout + kCvBlock - 1) / kCvBlock);
    const unsigned groups = (unsigned)((M + kCvMaxSlots - 1) / kCvMaxSlots);
    if (M < 3 || M > kMaxStreamsElementwise)
        return NE_EUNSUP;
    if (ws) {
        linconv_planes(J, ws, s);
        switch (M) {
        case 3: k_linconv_staged_pl<3><<<dim3(blocks, 1), kCvThreads, 0, s>>>(J); break;
        case 4: k_linconv_staged_pl<4><<<dim3(blocks, 1), kCvThreads, 0, s>>>(J); break;
        case 5: k_linconv_staged_pl<5><<<dim3(blocks, 1), kCvThreads, 0, s>>>(J); break;
        case 6: k_linconv_staged_pl<6><<<dim3(blocks, 1), kCvThreads, 0, s>>>(J); break;
        case 7: k_linconv_staged_pl<7><<<dim3(blocks, 1), kCvThreads, 0, s>>>(J); break;
        default:
            k_linconv_staged_pl<kCvMaxSlots><<<dim3(blocks, groups), kCvThreads, 0, s>>>(J);
        }
        return launch_status();
    }
    switch (M) {
    case 3: k_linconv_staged<3><<<dim3(blocks, 1), kCvThreads, 0, s>>>(J); break;
    case 4: k_linconv_staged<4><<<dim3(blocks, 1), kCvThreads, 0, s>>>(J); break;
    case 5: k_linconv_staged<5><<<dim3(blocks, 1), kCvThreads, 0, s>>>(J); break;
    case 6: k_linconv_staged<6><<<dim3(blocks, 1), kCvThreads, 0, s>>>(J); break;
    case 7: k_linconv_staged<7><<<dim3(blocks, 1), kCvThreads, 0, s>>>(J); break;
    default:
        k_linconv_staged<kCvMaxSlots><<<dim3(blocks, groups), kCvThreads, 0, s>>>(J);
    }
    return launch_status();
}

int launch_linconv_fused(const void *c, int c_dtype, int c_bits, const int8_t *g, int64_t L,
                         void *dhat, int out64, uint32_t *flags, unsigned long long *n_bad,
                         int64_t N, int M, int l, int r, void *ws, hipStream_t s)
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
    J.L = L;
    J.Nout = N + L - 1;
    J.M = M;
    J.l = l;
    J.r = r;
    const unsigned blocks = (unsigned)((J.Nout + kCvBlock - 1) / kCvBlock);
    if (M < 3 || M > 8)
        return NE_EUNSUP;
    if (ws) {
        linconv_planes(J, ws, s);
        switch (M) {
        case 3: k_linconv_fused_pl<3><<<blocks, kCvThreads, 0, s>>>(J); break;
        case 4: k_linconv_fused_pl<4><<<blocks, kCvThreads, 0, s>>>(J); break;
        case 5: k_linconv_fused_pl<5><<<blocks, kCvThreads, 0, s>>>(J); break;
        case 6: k_linconv_fused_pl<6><<<blocks, kCvThreads, 0, s>>>(J); break;
        case 7: k_linconv_fused_pl<7><<<blocks, kCvThreads, 0, s>>>(J); break;
        default: k_linconv_fused_pl<8><<<blocks, kCvThreads, 0, s>>>(J); break;
        }
        return launch_status();
    }
    switch (M) {
    case 3: k_linconv_fused<3><<<blocks, kCvThreads, 0, s>>>(J); break;
    case 4: k_linconv_fused<4><<<blocks, kCvThreads, 0, s>>>(J); break;
    case 5: k_linconv_fused<5><<<blocks, kCvThreads, 0, s>>>(J); break;
    case 6: k_linconv_fused<6><<<blocks, kCvThreads, 0, s>>>(J); break;
    case 7: k_linconv_fused<7><<<blocks, kCvThreads, 0, s>>>(J); break;
    case 8: k_linconv_fused<8><<<blocks, kCvThreads, 0, s>>>(J); break;
    default: return NE_EUNSUP;
    }
    return launch_status();
}

} // namespace ne
