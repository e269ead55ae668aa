// ne_gemm.hip -- launchers of the int8 matrix-core GEMM entry points
// (device code in ne_gemm_impl.h).
#include "ne_gemm_impl.h"

namespace ne {
namespace {

// --------------------------------------------------------------- launchers

inline bool aligned16(const void *p) { return ((uintptr_t)p & 15) == 0; }

template <class V>
int launch(typename V::Args &args, int64_t rows, bool al, hipStream_t s)
{
    const int64_t tm = (rows + V::BMS - 1) / V::BMS, tn = (args.N + V::BN - 1) / V::BN;
    if (tm * tn > 0x7fffffff)
        return NE_EINVAL;
    args.tiles_m = (int)tm;
    args.tiles_n = (int)tn;
    const dim3 grid((unsigned)(tm * tn));
    if constexpr (V::kDma) {
        if (al) {
            k_gemm_dma<V, V::kBK, V::kStages><<<grid, kThreads, 0, s>>>(args);
            return launch_status();
        }
    }
    if (al)
        k_gemm<V, true><<<grid, kThreads, 0, s>>>(args);
    else
        k_gemm<V, false><<<grid, kThreads, 0, s>>>(args);
    return launch_status();
}

template <int L>
int launch_eps_l(const int64_t *eps, const int8_t *Bt, int64_t *delta, int64_t R, int64_t K,
                 int64_t N, hipStream_t s)
{
    typename EpsV<L>::Args a{};
    a.Bt = Bt;
    a.K = K;
    a.N = N;
    a.eps = eps;
    a.delta = delta;
    a.R = R;
    return launch<EpsV<L>>(a, R, (K % 16 == 0) && aligned16(Bt), s);
}

template <int M, bool INJ>
int launch_fused_v(const int8_t *c, const int8_t *Bt, void *dhat, int out64, uint32_t *flags,
                   unsigned long long *n_bad, int64_t n, int64_t K, int64_t N, int l, int r,
                   const ne_inject_t *inj, hipStream_t s)
{
    using V = FusedV<M, FusedV<M>::BN, INJ>; // same tile as the default variant
    typename V::Args a{};
    a.Bt = Bt;
    a.K = K;
    a.N = N;
    a.c = c;
    a.dhat = dhat;
    a.flags = flags;
    a.n_bad = n_bad;
    a.n = n;
    a.l = l;
    a.r = r;
    a.out64 = out64;
    if (INJ) {
        a.inj_pos = inj->position;
        a.inj_stream = inj->stream;
        a.inj_mask = inj->xor_mask;
        a.inj_count = inj->count;
    }
    return launch<V>(a, n, (K % 16 == 0) && aligned16(c) && aligned16(Bt), s);
}

template <int M>
int launch_fused_m(const int8_t *c, const int8_t *Bt, void *dhat, int out64, uint32_t *flags,
                   unsigned long long *n_bad, int64_t n, int64_t K, int64_t N, int l, int r,
                   const ne_inject_t *inj, hipStream_t s)
{
    if (inj && inj->count > 0)
        return launch_fused_v<M, true>(c, Bt, dhat, out64, flags, n_bad, n, K, N, l, r, inj, s);
    return launch_fused_v<M, false>(c, Bt, dhat, out64, flags, n_bad, n, K, N, l, r, inj, s);
}

template <int M>
int launch_series_m(const int8_t *c, const int8_t *Bt, const int64_t *scale, const int64_t *add,
                    int64_t *rows, int64_t n, int64_t K, int64_t N, int l, int r, hipStream_t s)
{
    using V = SeriesV<M>;
    typename V::Args a{};
    a.Bt = Bt;
    a.K = K;
    a.N = N;
    a.c = c;
    a.n = n;
    a.l = l;
    a.r = r;
    a.scale = scale;
    a.add = add;
    a.rows = rows;
    return launch<V>(a, n, (K % 16 == 0) && aligned16(c) && aligned16(Bt), s);
}

template <int M>
int launch_abft_m(const int8_t *c, const int8_t *Bt, int32_t *d, uint32_t *flags,
                  unsigned long long *n_bad, int64_t n, int64_t K, int64_t N, hipStream_t s)
{
    typename AbftV<M>::Args a{};
    a.Bt = Bt;
    a.K = K;
    a.N = N;
    a.c = c;
    a.d = d;
    a.flags = flags;
    a.n_bad = n_bad;
    a.n = n;
    return launch<AbftV<M>>(a, n, (K % 16 == 0) && aligned16(c) && aligned16(Bt), s);
}

} // namespace

int launch_gemm_plain(const int8_t *A, const int8_t *Bt, int32_t *C, int64_t R, int64_t K,
                      int64_t N, hipStream_t s)
{
    PlainV::Args a{};
    a.Bt = Bt;
    a.K = K;
    a.N = N;
    a.A = A;
    a.C = C;
    a.R = R;
    return launch<PlainV>(a, R, (K % 16 == 0) && aligned16(A) && aligned16(Bt), s);
}

int launch_gemm_eps(const int64_t *eps, int digits, const int8_t *Bt, int64_t *delta, int64_t R,
                    int64_t K, int64_t N, hipStream_t s)
{
    switch (digits) {
    case 1: return launch_eps_l<1>(eps, Bt, delta, R, K, N, s);
    case 2: return launch_eps_l<2>(eps, Bt, delta, R, K, N, s);
    case 3: return launch_eps_l<3>(eps, Bt, delta, R, K, N, s);
    case 4: return launch_eps_l<4>(eps, Bt, delta, R, K, N, s);
    case 5: return launch_eps_l<5>(eps, Bt, delta, R, K, N, s);
    case 6: return launch_eps_l<6>(eps, Bt, delta, R, K, N, s);
    case 7: return launch_eps_l<7>(eps, Bt, delta, R, K, N, s);
    case 8: return launch_eps_l<8>(eps, Bt, delta, R, K, N, s);
    default: return NE_EINVAL;
    }
}

int launch_gemm_fused(const int8_t *c, const int8_t *Bt, void *dhat, int out64, uint32_t *flags,
                      unsigned long long *n_bad, int64_t n, int64_t K, int64_t N, int M, int l,
                      int r, const ne_inject_t *inj, hipStream_t s)
{
    switch (M) {
    case 3: return launch_fused_m<3>(c, Bt, dhat, out64, flags, n_bad, n, K, N, l, r, inj, s);
    case 4: return launch_fused_m<4>(c, Bt, dhat, out64, flags, n_bad, n, K, N, l, r, inj, s);
    case 5: return launch_fused_m<5>(c, Bt, dhat, out64, flags, n_bad, n, K, N, l, r, inj, s);
    case 6: return launch_fused_m<6>(c, Bt, dhat, out64, flags, n_bad, n, K, N, l, r, inj, s);
    case 7: return launch_fused_m<7>(c, Bt, dhat, out64, flags, n_bad, n, K, N, l, r, inj, s);
    case 8: return launch_fused_m<8>(c, Bt, dhat, out64, flags, n_bad, n, K, N, l, r, inj, s);
    default: return NE_EUNSUP;
    }
}

int launch_series_gemm(const int8_t *c, const int8_t *Bt, const int64_t *scale, const int64_t *add,
                       int64_t *rows, int64_t n, int64_t K, int64_t N, int M, int l, int r,
                       hipStream_t s)
{
    switch (M) {
    case 3: return launch_series_m<3>(c, Bt, scale, add, rows, n, K, N, l, r, s);
    case 4: return launch_series_m<4>(c, Bt, scale, add, rows, n, K, N, l, r, s);
    case 5: return launch_series_m<5>(c, Bt, scale, add, rows, n, K, N, l, r, s);
    case 6: return launch_series_m<6>(c, Bt, scale, add, rows, n, K, N, l, r, s);
    case 7: return launch_series_m<7>(c, Bt, scale, add, rows, n, K, N, l, r, s);
    case 8: return launch_series_m<8>(c, Bt, scale, add, rows, n, K, N, l, r, s);
    default: return NE_EUNSUP;
    }
}

template <int M>
int launch_abft_dma_m(const int8_t *c, const int8_t *Bt, int32_t *d, uint32_t *flags,
                      unsigned long long *n_bad, int64_t n, int64_t K, int64_t N, int8_t *planes,
                      hipStream_t s)
{
    using V = AbftDmaV<M>;
    const int64_t count = n * K;
    int8_t *lo = planes, *hi = planes + count;
    const int64_t blocks = (count / 16 + kThreads - 1) / kThreads;
    k_abft_checksum<M><<<(unsigned)(blocks < 8192 ? (blocks < 1 ? 1 : blocks) : 8192), kThreads, 0,
                         s>>>(c, lo, hi, count);
    if (launch_status())
        return NE_ELAUNCH;
    typename V::Args a{};
    a.Bt = Bt;
    a.K = K;
    a.N = N;
    a.c = c;
    a.rlo = lo;
    a.rhi = hi;
    a.d = d;
    a.flags = flags;
    a.n_bad = n_bad;
    a.n = n;
    const int64_t tm = (n + V::BMS - 1) / V::BMS, tn = (N + V::BN - 1) / V::BN;
    if (tm * tn > 0x7fffffff)
        return NE_EINVAL;
    a.tiles_m = (int)tm;
    a.tiles_n = (int)tn;
    k_gemm_dma<V, V::kBK, V::kStages><<<dim3((unsigned)(tm * tn)), kThreads, 0, s>>>(a);
    return launch_status();
}

int launch_gemm_abft(const int8_t *c, const int8_t *Bt, int32_t *d, uint32_t *flags,
                     unsigned long long *n_bad, int64_t n, int64_t K, int64_t N, int M,
                     void *ws, hipStream_t s)
{
    if (ws && K > 0 && K % 16 == 0 && aligned16(c) && aligned16(Bt)) {
        int8_t *pl = (int8_t *)ws;
        switch (M) {
        case 1: return launch_abft_dma_m<1>(c, Bt, d, flags, n_bad, n, K, N, pl, s);
        case 2: return launch_abft_dma_m<2>(c, Bt, d, flags, n_bad, n, K, N, pl, s);
        case 3: return launch_abft_dma_m<3>(c, Bt, d, flags, n_bad, n, K, N, pl, s);
        case 4: return launch_abft_dma_m<4>(c, Bt, d, flags, n_bad, n, K, N, pl, s);
        case 5: return launch_abft_dma_m<5>(c, Bt, d, flags, n_bad, n, K, N, pl, s);
        case 6: return launch_abft_dma_m<6>(c, Bt, d, flags, n_bad, n, K, N, pl, s);
        case 7: return launch_abft_dma_m<7>(c, Bt, d, flags, n_bad, n, K, N, pl, s);
        case 8: return launch_abft_dma_m<8>(c, Bt, d, flags, n_bad, n, K, N, pl, s);
        default: return NE_EUNSUP;
        }
    }
    switch (M) {
    case 1: return launch_abft_m<1>(c, Bt, d, flags, n_bad, n, K, N, s);
    case 2: return launch_abft_m<2>(c, Bt, d, flags, n_bad, n, K, N, s);
    case 3: return launch_abft_m<3>(c, Bt, d, flags, n_bad, n, K, N, s);
    case 4: return launch_abft_m<4>(c, Bt, d, flags, n_bad, n, K, N, s);
    case 5: return launch_abft_m<5>(c, Bt, d, flags, n_bad, n, K, N, s);
    case 6: return launch_abft_m<6>(c, Bt, d, flags, n_bad, n, K, N, s);
    case 7: return launch_abft_m<7>(c, Bt, d, flags, n_bad, n, K, N, s);
    case 8: return launch_abft_m<8>(c, Bt, d, flags, n_bad, n, K, N, s);
    default: return NE_EUNSUP;
    }
}

} // namespace ne
