// ne_selftest_host.hip -- host-side entry points that run the library's
// device word arithmetic (ne_arith.h) on the CPU.  Built into a separate
// library used only by the CPU test-suite; the product library does not
// contain or call it.
#include "ne_arith.h"

namespace {

template <int M>
int64_t run(const int64_t *delta, int64_t *dhat, uint8_t *flags, int64_t N, int l, int r)
{
    int64_t bad = 0;
    for (int64_t n = 0; n < N; ++n) {
        int64_t d[M], o[M];
        for (int j = 0; j < M; ++j)
            d[j] = delta[(int64_t)((r + j) % M) * N + n];
        const bool f = ne::disentangle_rot<M>(d, l, o);
        for (int j = 0; j < M; ++j)
            dhat[(int64_t)((r + j) % M) * N + n] = o[j];
        if (flags)
            flags[n] = f;
        bad += f;
    }
    return bad;
}

template <int M>
int64_t run32(const int32_t *delta, int32_t *dhat, uint8_t *flags, int64_t N, int l, int r)
{
    int64_t bad = 0;
    for (int64_t n = 0; n < N; ++n) {
        int32_t d[M], o[M];
        for (int j = 0; j < M; ++j)
            d[j] = delta[(int64_t)((r + j) % M) * N + n];
        const bool f = ne::disentangle_rot<M>(d, l, o);
        for (int j = 0; j < M; ++j)
            dhat[(int64_t)((r + j) % M) * N + n] = o[j];
        if (flags)
            flags[n] = f;
        bad += f;
    }
    return bad;
}

} // namespace

// w = 32 words
extern "C" int64_t ne_selftest_disentangle32(const int32_t *delta, int32_t *dhat, uint8_t *flags,
                                             int M, int64_t N, int l, int r)
{
    switch (M) {
    case 3: return run32<3>(delta, dhat, flags, N, l, r);
    case 4: return run32<4>(delta, dhat, flags, N, l, r);
    case 5: return run32<5>(delta, dhat, flags, N, l, r);
    case 6: return run32<6>(delta, dhat, flags, N, l, r);
    case 7: return run32<7>(delta, dhat, flags, N, l, r);
    case 8: return run32<8>(delta, dhat, flags, N, l, r);
    case 9: return run32<9>(delta, dhat, flags, N, l, r);
    case 10: return run32<10>(delta, dhat, flags, N, l, r);
    case 11: return run32<11>(delta, dhat, flags, N, l, r);
    case 12: return run32<12>(delta, dhat, flags, N, l, r);
    case 13: return run32<13>(delta, dhat, flags, N, l, r);
    case 14: return run32<14>(delta, dhat, flags, N, l, r);
    case 15: return run32<15>(delta, dhat, flags, N, l, r);
    case 16: return run32<16>(delta, dhat, flags, N, l, r);
    default: return -1;
    }
}

extern "C" int64_t ne_selftest_disentangle(const int64_t *delta, int64_t *dhat, uint8_t *flags,
                                           int M, int64_t N, int l, int r)
{
    switch (M) {
    case 3: return run<3>(delta, dhat, flags, N, l, r);
    case 4: return run<4>(delta, dhat, flags, N, l, r);
    case 5: return run<5>(delta, dhat, flags, N, l, r);
    case 6: return run<6>(delta, dhat, flags, N, l, r);
    case 7: return run<7>(delta, dhat, flags, N, l, r);
    case 8: return run<8>(delta, dhat, flags, N, l, r);
    case 9: return run<9>(delta, dhat, flags, N, l, r);
    case 10: return run<10>(delta, dhat, flags, N, l, r);
    case 11: return run<11>(delta, dhat, flags, N, l, r);
    case 12: return run<12>(delta, dhat, flags, N, l, r);
    case 13: return run<13>(delta, dhat, flags, N, l, r);
    case 14: return run<14>(delta, dhat, flags, N, l, r);
    case 15: return run<15>(delta, dhat, flags, N, l, r);
    case 16: return run<16>(delta, dhat, flags, N, l, r);
    default: return -1;
    }
}

extern "C" void ne_selftest_digits(const int64_t *v, int8_t *digits, int64_t N, int L)
{
    for (int64_t n = 0; n < N; ++n) {
        int64_t x = v[n];
        for (int j = 0; j < L; ++j)
            digits[n * L + j] = ne::digit(x);
    }
}
