// ne_elementwise.hip -- HBM-bound kernels of the staged path: entanglement,
// disentanglement + reliability check, fail-stop recovery, and the
// permute/scale/add operation.  One thread per stream position, all M
// streams of that position in registers; loads and stores of every stream
// are coalesced across the wavefront.
#include "ne_arith.h"
#include "ne_internal.h"
#include "ne_perm_impl.h"

namespace ne {
namespace {

constexpr int kThreads = 256;

// Words W: int64_t (w = 64) or int32_t (w = 32); every word operation
// wraps modulo 2^w.

// Section III-C (operator E): eps[m] = c[m] + 2^l c[m-1 mod M].
// c and eps may be the same buffer (in place when T is W): each thread reads
// all M words of its position before writing any.
template <int M, typename T, typename W>
__global__ __launch_bounds__(kThreads) void k_entangle(const T *c, W *eps, int64_t N, int l)
{
    const int64_t stride = (int64_t)gridDim.x * kThreads;
    for (int64_t n = (int64_t)blockIdx.x * kThreads + threadIdx.x; n < N; n += stride) {
        W v[M];
#pragma unroll
        for (int m = 0; m < M; ++m)
            v[m] = (W)c[(int64_t)m * N + n];
#pragma unroll
        for (int m = 0; m < M; ++m)
            eps[(int64_t)m * N + n] = entangle_word(v[m], v[(m + M - 1) % M], l);
    }
}

// Disentanglement without stream r and the check against stream r.  Each
// wavefront covers 64 consecutive positions, i.e. whole 32-bit words of the
// flag mask, so mask words are written without atomics.
template <int M, typename W>
__global__ __launch_bounds__(kThreads) void k_disentangle_check(const W *delta, W *dhat,
                                                                uint32_t *flags,
                                                                unsigned long long *n_bad,
                                                                int64_t N, int l, int r)
{
    const int lane = threadIdx.x & 63;
    const int64_t stride = (int64_t)gridDim.x * kThreads;
    const int64_t words = (N + 31) / 32;
    unsigned long long count = 0;
    for (int64_t base = (int64_t)blockIdx.x * kThreads + (threadIdx.x & ~63); base < N;
         base += stride) {
        const int64_t n = base + lane;
        bool f = false;
        if (n < N) {
            W d[M], o[M];
#pragma unroll
            for (int j = 0; j < M; ++j)
                d[j] = delta[(int64_t)((r + j) % M) * N + n];
            f = disentangle_rot<M>(d, l, o);
#pragma unroll
            for (int j = 0; j < M; ++j)
                dhat[(int64_t)((r + j) % M) * N + n] = o[j];
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

// Fail-stop recovery: the same extraction with r = lost; stream `lost` is
// never read.  Optionally re-creates the lost entangled stream.
template <int M, typename W>
__global__ __launch_bounds__(kThreads) void k_recover(StreamPtrs delta, int lost, W *dhat,
                                                      W *rebuilt, int64_t N, int l)
{
    const int64_t stride = (int64_t)gridDim.x * kThreads;
    for (int64_t n = (int64_t)blockIdx.x * kThreads + threadIdx.x; n < N; n += stride) {
        W d[M], o[M];
        d[0] = 0;
#pragma unroll
        for (int j = 1; j < M; ++j)
            d[j] = ((const W *)delta.p[(lost + j) % M])[n];
        (void)disentangle_rot<M>(d, l, o);
#pragma unroll
        for (int j = 0; j < M; ++j)
            dhat[(int64_t)((lost + j) % M) * N + n] = o[j];
        if (rebuilt)
            rebuilt[n] = reentangle(o[0], o[M - 1], l);
    }
}

// delta[m][n] = scale[n] * eps[m][perm[n]] + (2^l + 1) add[n]   (mod 2^w).
template <int M, typename W>
__global__ __launch_bounds__(kThreads) void k_permute_scale(const W *__restrict__ eps,
                                                            const int32_t *__restrict__ perm,
                                                            const W *__restrict__ scale,
                                                            const W *__restrict__ add,
                                                            W *__restrict__ delta, int64_t N, int l)
{
    typedef typename UWord<W>::type U;
    const int64_t stride = (int64_t)gridDim.x * kThreads;
    for (int64_t n = (int64_t)blockIdx.x * kThreads + threadIdx.x; n < N; n += stride) {
        int64_t src = perm[n];
        src = src < 0 ? 0 : (src >= N ? N - 1 : src);
        const U s = scale ? (U)scale[n] : (U)1;
        const U a = add ? (U)entangle_word(add[n], add[n], l) : (U)0;
#pragma unroll
        for (int m = 0; m < M; ++m)
            delta[(int64_t)m * N + n] = (W)(s * (U)eps[(int64_t)m * N + src] + a);
    }
}

template <template <int> class F, typename... A>
int dispatch_m(int M, A... args)
{
    switch (M) {
    case 3: return F<3>::run(args...);
    case 4: return F<4>::run(args...);
    case 5: return F<5>::run(args...);
    case 6: return F<6>::run(args...);
    case 7: return F<7>::run(args...);
    case 8: return F<8>::run(args...);
    case 9: return F<9>::run(args...);
    case 10: return F<10>::run(args...);
    case 11: return F<11>::run(args...);
    case 12: return F<12>::run(args...);
    case 13: return F<13>::run(args...);
    case 14: return F<14>::run(args...);
    case 15: return F<15>::run(args...);
    case 16: return F<16>::run(args...);
    default: return NE_EUNSUP;
    }
}

template <int M> struct EntangleL {
    template <typename W>
    static void go(const void *c, int dt, W *eps, int64_t N, int l, hipStream_t s)
    {
        const unsigned g = grid_for(N, kThreads);
        if (dt == NE_I8)
            k_entangle<M, int8_t, W><<<g, kThreads, 0, s>>>((const int8_t *)c, eps, N, l);
        else if (dt == NE_I32)
            k_entangle<M, int32_t, W><<<g, kThreads, 0, s>>>((const int32_t *)c, eps, N, l);
        else
            k_entangle<M, int64_t, W><<<g, kThreads, 0, s>>>((const int64_t *)c, eps, N, l);
    }
    static int run(const void *c, int dt, void *eps, int64_t N, int l, int w, hipStream_t s)
    {
        if (w == 32)
            go<int32_t>(c, dt, (int32_t *)eps, N, l, s);
        else
            go<int64_t>(c, dt, (int64_t *)eps, N, l, s);
        return launch_status();
    }
};

template <int M> struct CheckL {
    template <typename W>
    static void go(const void *delta, void *dhat, uint32_t *flags, unsigned long long *nb,
                   int64_t N, int l, int r, hipStream_t s)
    {
        k_disentangle_check<M, W><<<grid_for(N, kThreads), kThreads, 0, s>>>(
            (const W *)delta, (W *)dhat, flags, nb, N, l, r);
    }
    static int run(const void *delta, void *dhat, uint32_t *flags, unsigned long long *nb,
                   int64_t N, int l, int r, int w, hipStream_t s)
    {
        if (w == 32)
            go<int32_t>(delta, dhat, flags, nb, N, l, r, s);
        else
            go<int64_t>(delta, dhat, flags, nb, N, l, r, s);
        return launch_status();
    }
};

template <int M> struct RecoverL {
    static int run(const StreamPtrs *d, int lost, void *dhat, void *rb, int64_t N, int l, int w,
                   hipStream_t s)
    {
        const unsigned g = grid_for(N, kThreads);
        if (w == 32)
            k_recover<M, int32_t><<<g, kThreads, 0, s>>>(*d, lost, (int32_t *)dhat, (int32_t *)rb,
                                                         N, l);
        else
            k_recover<M, int64_t><<<g, kThreads, 0, s>>>(*d, lost, (int64_t *)dhat, (int64_t *)rb,
                                                         N, l);
        return launch_status();
    }
};

template <int M> struct PermL {
    static int run(const void *eps, const int32_t *perm, const void *scale, const void *add,
                   void *delta, int64_t N, int l, int w, hipStream_t s)
    {
        const unsigned g = grid_for(N, kThreads);
        if (w == 32)
            k_permute_scale<M, int32_t><<<g, kThreads, 0, s>>>(
                (const int32_t *)eps, perm, (const int32_t *)scale, (const int32_t *)add,
                (int32_t *)delta, N, l);
        else
            k_permute_scale<M, int64_t><<<g, kThreads, 0, s>>>(
                (const int64_t *)eps, perm, (const int64_t *)scale, (const int64_t *)add,
                (int64_t *)delta, N, l);
        return launch_status();
    }
};

template <int M> struct PermFusedL {
    template <typename T, typename W>
    static int go(const T *c, uint64_t *rows, const int32_t *perm, const W *scale, const W *add,
                  void *dhat, int out64, uint32_t *flags, unsigned long long *nb, int64_t N, int l,
                  int r, hipStream_t s)
    {
        const unsigned g = grid_for(N, kThreads);
        if (rows) {
            k_perm_pack<M, T><<<g, kThreads, 0, s>>>(c, rows, N, r);
            if (launch_status())
                return NE_ELAUNCH;
        }
        k_permute_scale_fused<M, T, false, W><<<g, kThreads, 0, s>>>(
            c, rows, perm, scale, add, dhat, out64, flags, nb, N, l, r);
        return launch_status();
    }
    template <typename W>
    static int go_w(const void *c, int dt, uint64_t *rows, const int32_t *perm, const void *scale,
                    const void *add, void *dhat, int out64, uint32_t *flags,
                    unsigned long long *nb, int64_t N, int l, int r, hipStream_t s)
    {
        const W *sc = (const W *)scale, *ad = (const W *)add;
        if (dt == NE_I8)
            return go<int8_t, W>((const int8_t *)c, rows, perm, sc, ad, dhat, out64, flags, nb, N,
                                 l, r, s);
        if (dt == NE_I32)
            return go<int32_t, W>((const int32_t *)c, rows, perm, sc, ad, dhat, out64, flags, nb,
                                  N, l, r, s);
        return go<int64_t, W>((const int64_t *)c, rows, perm, sc, ad, dhat, out64, flags, nb, N,
                              l, r, s);
    }
    static int run(const void *c, int dt, uint64_t *rows, const int32_t *perm, const void *scale,
                   const void *add, void *dhat, int out64, uint32_t *flags,
                   unsigned long long *nb, int64_t N, int l, int r, int w, hipStream_t s)
    {
        if (w == 32)
            return go_w<int32_t>(c, dt, rows, perm, scale, add, dhat, out64, flags, nb, N, l, r,
                                 s);
        return go_w<int64_t>(c, dt, rows, perm, scale, add, dhat, out64, flags, nb, N, l, r, s);
    }
};

// Gather of entangled rows (the position-major output of a series' GEMM
// head), then disentangle and check.
template <int M> struct PermRowsL {
    static int run(const int64_t *rows, const int32_t *perm, void *dhat, int out64,
                   uint32_t *flags, unsigned long long *nb, int64_t N, int l, int r,
                   hipStream_t s)
    {
        k_permute_scale_fused<M, int64_t, true, int64_t><<<grid_for(N, kThreads), kThreads, 0, s>>>(
            nullptr, (const uint64_t *)rows, perm, nullptr, nullptr, dhat, out64, flags, nb, N, l,
            r);
        return launch_status();
    }
};

} // namespace

int launch_permute_rows_check(const int64_t *rows, const int32_t *perm, void *dhat, int out64,
                              uint32_t *flags, unsigned long long *n_bad, int64_t N, int M, int l,
                              int r, hipStream_t s)
{
    return dispatch_m<PermRowsL>(M, rows, perm, dhat, out64, flags, n_bad, N, l, r, s);
}

int64_t permute_rows_bytes(int64_t N, int M, int c_dtype)
{
    return N * ((M * c_dtype + 7) / 8) * 8;
}

int launch_permute_scale_fused(const void *c, int c_dtype, const int32_t *perm, const void *scale,
                               const void *add, void *dhat, int out64, uint32_t *flags,
                               unsigned long long *n_bad, int64_t N, int M, int l, int r, int w,
                               void *rows, hipStream_t s)
{
    return dispatch_m<PermFusedL>(M, c, c_dtype, (uint64_t *)rows, perm, scale, add, dhat, out64,
                                  flags, n_bad, N, l, r, w, s);
}

int launch_entangle(const void *c, int c_dtype, void *eps, int64_t N, int M, int l, int w,
                    hipStream_t s)
{
    return dispatch_m<EntangleL>(M, c, c_dtype, eps, N, l, w, s);
}

int launch_disentangle_check(const void *delta, void *dhat, uint32_t *flags,
                             unsigned long long *n_bad, int64_t N, int M, int l, int r, int w,
                             hipStream_t s)
{
    return dispatch_m<CheckL>(M, delta, dhat, flags, n_bad, N, l, r, w, s);
}

int launch_recover(const StreamPtrs &delta, int lost, void *dhat, void *rebuilt, int64_t N, int M,
                   int l, int w, hipStream_t s)
{
    return dispatch_m<RecoverL>(M, &delta, lost, dhat, rebuilt, N, l, w, s);
}

int launch_permute_scale(const void *eps, const int32_t *perm, const void *scale, const void *add,
                         void *delta, int64_t N, int M, int l, int w, hipStream_t s)
{
    return dispatch_m<PermL>(M, eps, perm, scale, add, delta, N, l, w, s);
}

} // namespace ne
