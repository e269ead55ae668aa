// ne_arith.h -- word arithmetic of numerical entanglement shared by every
// kernel (host-callable too, so the exact same code can be exercised on the
// CPU by the self-test library).
//
// Anam & Andreopoulos, "Reliable Linear, Sesquilinear and Bijective
// Operations on Integer Data Streams via Numerical Entanglement".
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#define NE_HD __host__ __device__ __forceinline__

namespace ne {

// Entangled word of section III-C (operator E):  c + 2^l * c_prev  (mod 2^64).
NE_HD int64_t entangle_word(int64_t c, int64_t c_prev, int l)
{
    return (int64_t)((uint64_t)c + ((uint64_t)c_prev << l));
}

// Next signed int8 digit of a 64-bit word (least significant first):
// v = sum_j 2^(8j) e_j with e_j in [-128, 127].  digits_for_bits(b) digits
// leave a zero remainder for every word in [-2^(b-1), 2^(b-1)); eight digits
// reproduce every word modulo 2^64 (the ninth digit's weight is 2^64).
NE_HD int8_t digit(int64_t &v)
{
    const int8_t e = (int8_t)(v & 0xFF);
    v = (v - (int64_t)e) >> 8;
    return e;
}

// Number of signed int8 digits needed for words in [-2^(b-1), 2^(b-1)).
NE_HD int digits_for_bits(int bits)
{
    const int L = bits / 8 + 1;
    return L > 8 ? 8 : L;
}

// ---------------------------------------------------------------------------
// Disentanglement and reliability check, section III-C (with the readings
// used throughout this library: d_temp carries a leading (-1)^M, and the
// chain runs for 1 <= m <= M-2).  Inputs are rotated so that the stream that
// is NOT used for extraction (r) sits in slot 0:
//     d[j] = delta of stream (r + j) mod M,   out[j] = d_hat of that stream.
// d[0] is read only by the check.
//
// The paper evaluates d_temp in 2w = 128 bits.  Here the same integers are
// obtained with 64-bit operations only:
//   * the low (M-1) l bits of d_temp (all that the sign extension for
//     d_hat[r-1] needs) come from a Horner evaluation modulo 2^64;
//   * d_hat[r] = (-1)^M (d_temp - d_hat[r-1]) / 2^((M-1) l) is an exact
//     division, carried out as M-1 exact divisions by 2^l.  At each step the
//     running value plus (or minus) the next delta is divisible by 2^l, so
//     floor(a/2^l) + floor(b/2^l) plus a carry that is 1 exactly when the low
//     l bits of b are non-zero gives the quotient without forming a+b
//     (which could overflow 64 bits).  Every intermediate stays below
//     2^(64-l) in magnitude.
//   * the chain keeps the low 64 bits, as a 128-bit chain truncated to 64.
//   * the check delta_r == d_hat_r + 2^l d_hat_(r-1), exact over the
//     integers, holds iff the low l bits of delta_r and d_hat_r agree and
//     floor(delta_r/2^l) - floor(d_hat_r/2^l) == d_hat_(r-1).
// Requires 2 <= l and (M-1) l < 64.  Returns the check flag.
// ---------------------------------------------------------------------------
template <int M>
NE_HD bool disentangle_rot(const int64_t (&d)[M], int l, int64_t (&out)[M])
{
    const int L = (M - 1) * l;
    uint64_t U = 0;
#pragma unroll
    for (int m = 0; m <= M - 2; ++m) {
        const uint64_t v = (uint64_t)d[1 + m];
        U = (U << l) + (((M + m) & 1) ? (uint64_t)0 - v : v);
    }
    const int64_t lo = (int64_t)(U << (64 - L)) >> (64 - L);
    const uint64_t mask = ((uint64_t)1 << l) - 1;
    int64_t q = (d[M - 1] >> l) - (lo >> l);
#pragma unroll
    for (int m = M - 3; m >= 0; --m) {
        const int64_t v = d[1 + m];
        if (((M + m) & 1) == 0)
            q = (q >> l) + (v >> l) + (int64_t)(((uint64_t)v & mask) != 0);
        else
            q = (q >> l) - (v >> l);
    }
    const int64_t dr = (M & 1) ? -q : q;
    out[0] = dr;
    out[M - 1] = lo;
    int64_t prev = dr;
#pragma unroll
    for (int m = 1; m <= M - 2; ++m) {
        prev = (int64_t)((uint64_t)d[m] - ((uint64_t)prev << l));
        out[m] = prev;
    }
    const int64_t d0 = d[0];
    return ((((uint64_t)(d0 ^ dr)) & mask) != 0) || (((d0 >> l) - (dr >> l)) != lo);
}

// Re-created entangled word of a stream from its own output and that of the
// previous stream: d + 2^l d_prev (mod 2^64).
NE_HD int64_t reentangle(int64_t d, int64_t d_prev, int l)
{
    return entangle_word(d, d_prev, l);
}

// ---------------------------------------------------------------------------
// w = 32 (the word width of the paper's Table II and its experiments): words
// wrap modulo 2^32 and the disentanglement's 2w-bit interim is a 64-bit
// integer, so d_temp is formed directly: |d_temp| < 2^((M-2) l + 32) <= 2^62
// because (M-1) l + k <= 32.  Outputs keep the low 32 bits, and the check
// rebuilds delta_r from those stored outputs in 64-bit arithmetic:
//     flag = delta_r != d_hat_r + 2^l d_hat_(r-1)   (64-bit, exact).
// ---------------------------------------------------------------------------
// Unsigned type of a word, for wrapping arithmetic.
template <typename W> struct UWord;
template <> struct UWord<int64_t> { typedef uint64_t type; };
template <> struct UWord<int32_t> { typedef uint32_t type; };

NE_HD int32_t entangle_word(int32_t c, int32_t c_prev, int l)
{
    return (int32_t)((uint32_t)c + ((uint32_t)c_prev << l));
}

NE_HD int32_t reentangle(int32_t d, int32_t d_prev, int l)
{
    return entangle_word(d, d_prev, l);
}

template <int M>
NE_HD bool disentangle_rot(const int32_t (&d)[M], int l, int32_t (&out)[M])
{
    const int L = (M - 1) * l;
    uint64_t t = 0; // d_temp, exact (two's complement in 64 bits)
#pragma unroll
    for (int m = 0; m <= M - 2; ++m) {
        const uint64_t term = (uint64_t)(int64_t)d[1 + m] << ((M - 2 - m) * l);
        t = (m & 1) ? t - term : t + term;
    }
    if (M & 1)
        t = (uint64_t)0 - t;
    const int64_t lo = (int64_t)(t << (64 - L)) >> (64 - L);
    uint64_t diff = t - (uint64_t)lo;
    if (M & 1)
        diff = (uint64_t)0 - diff;
    const int64_t dr = (int64_t)diff >> L;
    out[0] = (int32_t)dr;
    out[M - 1] = (int32_t)lo;
    uint64_t prev = (uint64_t)dr;
#pragma unroll
    for (int m = 1; m <= M - 2; ++m) {
        prev = (uint64_t)(int64_t)d[m] - (prev << l);
        out[m] = (int32_t)prev;
    }
    const uint64_t rebuilt = (uint64_t)(int64_t)out[0] + ((uint64_t)(int64_t)out[M - 1] << l);
    return (uint64_t)(int64_t)d[0] != rebuilt;
}

} // namespace ne
