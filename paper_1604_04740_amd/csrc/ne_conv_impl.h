// ne_conv_impl.h -- circular convolution on the int8 matrix cores (device
// code shared by the convolution entry points and the batched kernel).
//
// The star operator of section II, y[t] = sum_j x[(t - j) mod N] g[j], for
// the 1024 outputs t = t0 + 32 a + p (a, p in 0..31) of one block is a
// 32 x 32 matrix product over the tap index i in [0, N):
//     Y[a][p] = sum_i A[a][i] B[i][p],
//     A[a][i] = x[(t0 + 32 a - i) mod N]     (Toeplitz in a, i)
//     B[i][p] = g[(p + i) mod N]             (Hankel in i, p; 0 for i >= N)
// (substitute j = (p + i) mod N).  Both operands are built in LDS from x
// and g, one 32-tap k-step at a time feeds v_mfma_i32_32x32x32_i8.
//
// Words wider than a byte are split into signed int8 digits (balanced, base
// 256): x = sum_d 256^d x_d.  Each digit is its own pass over the taps; the
// int32 accumulators are exact (|sum| <= N * 128 * 128 < 2^31 for
// N <= 131071) and are folded into 64-bit words (mod 2^64) after the pass.
//
// Fused (section III-C): the sources are the plain streams c; slot s holds
// stream (r + s) mod M, and the entangled output of slot s is
//     delta_s = conv(c_s, g) + 2^l conv(c_{s-1}, g),
// two independent accumulator sets per slot, so that a fault in one
// stream's computation reaches only that stream's delta.  The epilogue
// disentangles and checks (delta never reaches memory).
// Staged: the sources are given 64-bit words (entangled streams) and delta
// is written out.
//
// Linear convolution (LIN) of a stream of Nx samples with L taps,
// y[t] = sum_{j<L} x[t - j] g[j] for 0 <= t < Nx + L - 1 (x zero outside):
// the same block product over i in [0, L + 32) with
//     A[a][i] = x[t0 + 32 + 32 a - i],   B[i][p] = g[p + i - 32]
// (zero outside the stream or the kernel); the shift by 32 keeps the tap
// index of every column non-negative.  Only the taps of the kernel are
// visited, so the work per block is proportional to L, not to Nx.
//
// LDS, per workgroup (4 wavefronts):
//   A rings   one 2048-byte ring per slot: byte v holds digit d of
//             x[(t0 - v) mod N], so the 16 bytes a lane needs for row a at
//             taps i0 + 16h .. +15 start at v = i0 + 16h - 32a (aligned).
//             Chunks are XOR-swizzled (bit 0 ^= bit 4) so that the 16 rows
//             a lane group reads hit 16 different bank groups.
//   g copies  32 rings of 1024 bytes (stride 1040 for the banks): copy p
//             holds B[i][p] at byte i mod 1024, so column p's 16 taps are
//             one aligned read.
//   red       [slots][1024] uint64: the folded delta of the block.
// A workgroup with at most four 256-tap steps (a split of the taps) stages
// all of them at once: one wait for memory, one barrier, then only MFMAs.
// Longer tap ranges slide: each step is staged while the previous one is
// multiplied (256 new bytes per ring per step), one barrier per step.  The
// four wavefronts take two k-steps of each 256-tap step and add their
// folded partial sums into red with LDS atomics.
#pragma once

#include "ne_arith.h"
#include "ne_internal.h"

namespace ne {
namespace {

typedef int cv4i __attribute__((ext_vector_type(4)));
typedef int cv16i __attribute__((ext_vector_type(16)));

constexpr int kCvThreads = 256;
constexpr int kCvBlock = 1024;    // outputs per block
constexpr int kCvStep = 256;      // taps staged per step
constexpr int kCvRing = 2048;     // bytes per A ring (>= 992 + 4 * 256)
constexpr int kCvGRing = 1024;    // bytes per g copy (>= 4 * 256)
constexpr int kCvGStride = 1040;  // bytes between g copies (16 mod 256: bank spread)
constexpr int kCvOneShot = 4;     // steps a workgroup stages at once
constexpr int kCvMaxSlots = 8;
constexpr int kCvGPad = 512;     // zero bytes around g in the plane-staged form (>= 290)

// A rings allocated for G slots: at least eight, so that a one-shot
// workgroup can hold every digit of up to eight (slot, digit) sources.
__host__ __device__ constexpr int cv_rings(int slots)
{
    return slots < 8 ? 8 : slots;
}

__host__ __device__ constexpr int cv_lds_bytes(int slots)
{
    return cv_rings(slots) * kCvRing + 32 * kCvGStride + slots * kCvBlock * 8;
}

__device__ __forceinline__ unsigned long long *cv_red(int8_t *lds, int slots)
{
    return (unsigned long long *)(lds + cv_rings(slots) * kCvRing + 32 * kCvGStride);
}

// Number of balanced int8 digits for values with |x| < 2^(bits-1).
__host__ __device__ inline int cv_digits(int bits)
{
    return bits <= 8 ? 1 : (bits / 8 + 1 > 8 ? 8 : bits / 8 + 1);
}

struct ConvJob {
    const void *x;              // fused: c [M][N]; staged: eps [M][N] int64
    int x_dtype;                // NE_I8 / NE_I32 / NE_I64
    int digits;                 // balanced int8 digits per value
    const int8_t *g;            // [N]
    void *out;                  // fused: d_hat (int32 or int64); staged: delta int64
    int out64;
    uint32_t *flags;            // fused: [ceil(N/32)] or NULL
    unsigned long long *n_bad;  // fused: counter or NULL
    int64_t N;                  // samples per input stream
    int64_t L;                  // taps (circular: N)
    int64_t Nout;               // outputs per stream (circular: N; linear: N + L - 1)
    // linear form with digit planes (k_cv_planes), or NULL:
    const int8_t *planes;       // [M][digits][P]: digit d of sample j - pad at byte j
    const int8_t *gpad;         // g with kCvGPad zero bytes on both sides
    int64_t P;                  // bytes per plane (a multiple of 4)
    int pad;                    // 3 mod 4
    int M, l, r;
    int s0;                     // staged: first stream of this workgroup
};

__device__ __forceinline__ int8_t cv_digit(int64_t v, int d)
{
    int8_t e = digit(v);
    for (int j = 0; j < d; ++j)
        e = digit(v);
    return e;
}

// Byte offset of ring coordinate v (any integer) inside an A ring.
__device__ __forceinline__ int cv_ring_off(int64_t v)
{
    const int c = (int)((v & (kCvRing - 1)) >> 4);
    return ((c ^ ((c >> 4) & 1)) << 4) | (int)(v & 15);
}

// a mod N in [0, N) for |a| < 2^31 (N <= 131071, so every index here fits).
__device__ __forceinline__ int cv_mod(int a, int N)
{
    const int m = a % N;
    return m < 0 ? m + N : m;
}

// One thread's share of an A-ring step: ring coordinate v of every slot.
// The samples are kept as loaded (int8 and int32 sign-extended in lo,
// int64 in hi:lo) and widened only when stored: an instruction that uses a
// load's result right after it makes the wavefront wait for that load
// alone, so the loads of a step would be served one after another.
template <int G>
struct CvA {
    uint32_t lo[G], hi[G];
    uint32_t valid; // bit s: slot s holds a sample (else it counts as 0)
    int v;
    // ok == false: the coordinate lies outside the stream (linear form).
    // Every lane loads (from index 0 where it has no sample) and the dtype
    // test is uniform, so no load result is overwritten while in flight.
    __device__ __forceinline__ void load(const ConvJob &J, const int (&stream)[G], int idx, int v_,
                                         bool ok = true)
    {
        v = v_;
        const int ic = ok ? idx : 0;
        valid = 0;
#pragma unroll
        for (int s = 0; s < G; ++s)
            if (ok && stream[s] >= 0)
                valid |= 1u << s;
        if (J.x_dtype == NE_I64) {
#pragma unroll
            for (int s = 0; s < G; ++s) {
                const int64_t i = (int64_t)(stream[s] < 0 ? 0 : stream[s]) * J.N + ic;
                const uint2 w = ((const uint2 *)J.x)[i];
                lo[s] = w.x;
                hi[s] = w.y;
            }
        } else if (J.x_dtype == NE_I32) {
#pragma unroll
            for (int s = 0; s < G; ++s) {
                lo[s] = ((const uint32_t *)J.x)[(int64_t)(stream[s] < 0 ? 0 : stream[s]) * J.N + ic];
                hi[s] = 0;
            }
        } else {
#pragma unroll
            for (int s = 0; s < G; ++s) {
                lo[s] = (uint32_t)(int32_t)(
                    (const int8_t *)J.x)[(int64_t)(stream[s] < 0 ? 0 : stream[s]) * J.N + ic];
                hi[s] = 0;
            }
        }
    }
    __device__ __forceinline__ int64_t value(int s, int dt) const
    {
        const int64_t x =
            dt == NE_I64 ? (int64_t)(((uint64_t)hi[s] << 32) | lo[s]) : (int64_t)(int32_t)lo[s];
        return (valid >> s) & 1 ? x : 0;
    }
    __device__ __forceinline__ void store(int8_t *rings, int d, int dt) const
    {
        const int off = cv_ring_off(v);
        if (dt == NE_I64) {
#pragma unroll
            for (int s = 0; s < G; ++s)
                rings[s * kCvRing + off] = cv_digit(value(s, dt), d);
        } else {
            // samples of at most 32 bits: the same balanced digits in 32-bit
            // arithmetic; (x - e) / 256 = floor(x / 256) + bit 7 of x, which
            // cannot overflow
#pragma unroll
            for (int s = 0; s < G; ++s) {
                int32_t x = (valid >> s) & 1 ? (int32_t)lo[s] : 0;
                for (int j = 0; j < d; ++j)
                    x = (x >> 8) + ((x >> 7) & 1);
                rings[s * kCvRing + off] = (int8_t)(x & 0xFF);
            }
        }
    }
    // every digit: digit dd of slot s into ring s + G dd
    __device__ __forceinline__ void store_all(int8_t *rings, int digits, int dt) const
    {
        const int off = cv_ring_off(v);
#pragma unroll
        for (int s = 0; s < G; ++s) {
            int64_t x = value(s, dt);
            for (int dd = 0; dd < digits; ++dd)
                rings[(s + G * dd) * kCvRing + off] = digit(x);
        }
    }
};

// One thread's share of a g-copy step: 32 taps [i0, i0 + 32) of copy p.
// w holds nine dwords and sh a byte shift; tap word k is
// alignbyte(w[k + 1], w[k], sh), formed only when stored (as for CvA).
struct CvG {
    uint32_t w[9];
    uint32_t sh;
    int p;
    int i0;
    template <bool LIN = false>
    __device__ __forceinline__ void load(const ConvJob &J, int I, int tid)
    {
        p = tid >> 3;
        i0 = I + 32 * (tid & 7);
        sh = 0;
        w[8] = 0;
        if constexpr (LIN) {
            // B[i][p] = g[p + i - 32], zero outside the L taps
            const int L = (int)J.L, s = i0 + p - 32;
            if (J.gpad && s >= -kCvGPad && s + 36 <= L + kCvGPad) {
                gather_aligned(J.gpad + kCvGPad + s); // zero-padded copy of g
                return;
            }
            if (s >= 0 && s + 36 <= L) {
                gather_aligned(J.g + s);
            } else {
                // byte by byte; every byte load is issued (from tap 0 where
                // there is no tap) before any is used
                uint32_t b[32];
#pragma unroll
                for (int q = 0; q < 32; ++q) {
                    const int j = s + q;
                    b[q] = (uint32_t)(uint8_t)J.g[(j >= 0 && j < L) ? j : 0];
                }
#pragma unroll
                for (int k = 0; k < 8; ++k) {
                    uint32_t x = 0;
#pragma unroll
                    for (int q = 0; q < 4; ++q) {
                        const int j = s + 4 * k + q;
                        x |= ((j >= 0 && j < L) ? b[4 * k + q] : 0u) << (8 * q);
                    }
                    w[k] = x;
                }
            }
            return;
        }
        const int N = (int)J.N, s = i0 + p;
        if (i0 + 32 <= N && s + 36 <= N) {
            gather_aligned(J.g + s);
        } else {
            // wrap-around or past the last tap: byte by byte, every load
            // issued before any is used
            uint32_t b[32];
            int j = cv_mod(s, N);
#pragma unroll
            for (int q = 0; q < 32; ++q) {
                b[q] = (uint32_t)(uint8_t)J.g[j];
                j = j + 1 == N ? 0 : j + 1;
            }
#pragma unroll
            for (int k = 0; k < 8; ++k) {
                uint32_t x = 0;
#pragma unroll
                for (int q = 0; q < 4; ++q)
                    x |= (i0 + 4 * k + q < N ? b[4 * k + q] : 0u) << (8 * q);
                w[k] = x;
            }
        }
    }
    // src[0 .. 31] as nine aligned dwords and a shift (all inside the
    // kernel: the caller checks that src + 36 does not pass its end)
    __device__ __forceinline__ void gather_aligned(const int8_t *src)
    {
        const uintptr_t a = (uintptr_t)src;
        const uint32_t *q = (const uint32_t *)(a & ~(uintptr_t)3);
        sh = (uint32_t)(a & 3);
#pragma unroll
        for (int k = 0; k < 9; ++k)
            w[k] = q[k];
    }
    __device__ __forceinline__ void store(int8_t *gc) const
    {
        int8_t *dst = gc + p * kCvGStride + (int)(i0 & (kCvGRing - 1));
        uint32_t t[8];
#pragma unroll
        for (int k = 0; k < 8; ++k)
            t[k] = __builtin_amdgcn_alignbyte(w[k + 1], w[k], sh);
        *(cv4i *)dst = cv4i{(int)t[0], (int)t[1], (int)t[2], (int)t[3]};
        *(cv4i *)(dst + 16) = cv4i{(int)t[4], (int)t[5], (int)t[6], (int)t[7]};
    }
};

// ---------------------------------------------------------------------------
// Linear form from digit planes.  A pre-pass (k_cv_planes) writes digit d
// of every sample of stream m into plane (m, d) at byte j = index + pad,
// zeros around the stream, and g with kCvGPad zero bytes on both sides.
// Ring bytes v .. v + 3 (v a multiple of 4) hold samples t0 + 32 - v - k,
// k = 0..3, which are the plane bytes o + 3 - k for o = t0 + 29 - v + pad,
// a multiple of 4 since pad = 3 mod 4: one aligned dword, bytes reversed.
// No bounds tests and no digit arithmetic remain in the staging.
// ---------------------------------------------------------------------------

__host__ __device__ constexpr int cv_plane_pad(int64_t L)
{
    return (int)(((L + 2048 + 3) / 4) * 4 + 3);
}

__host__ __device__ constexpr int64_t cv_plane_bytes(int64_t N, int64_t L)
{
    return ((N + 2 * (int64_t)cv_plane_pad(L) + 8 + 3) / 4) * 4;
}

// One thread's share of a round of A-ring dwords: NW plane dwords and the
// ring byte offset each goes to (-1: none).
template <int NW>
struct CvP {
    uint32_t w[NW];
    int dst[NW];
    // Dwords u0 + k * 256 + tid of the range: nrings rings of nd dwords from
    // ring byte vb; ring rr is slot rr mod G of digit rr / G (alld) or of
    // digit d.  Every lane loads (from the range's last dword past its end).
    template <int G, bool FUSED>
    __device__ __forceinline__ void load(const ConvJob &J, int t0i, int vb, int nd, int nrings,
                                         bool alld, int d, int u0, int tid)
    {
        const int T = nrings * nd;
#pragma unroll
        for (int k = 0; k < NW; ++k) {
            const int u = u0 + k * kCvThreads + tid;
            const int uc = u < T ? u : T - 1;
            const int rr = uc / nd, q = uc - rr * nd;
            const int s = rr % G, dig = alld ? rr / G : d;
            const int v = vb + 4 * q;
            int m;
            if constexpr (FUSED)
                m = (J.r + s) % J.M;
            else
                m = J.s0 + s < J.M ? J.s0 + s : 0; // slots past M: any valid plane
            const int64_t o = (int64_t)(m * J.digits + dig) * J.P + (t0i + 29 - v + J.pad);
            w[k] = *(const uint32_t *)(J.planes + o);
            dst[k] = u < T ? (alld ? rr : s) * kCvRing + cv_ring_off(v) : -1;
        }
    }
    __device__ __forceinline__ void store(int8_t *rings) const
    {
#pragma unroll
        for (int k = 0; k < NW; ++k)
            if (dst[k] >= 0)
                *(uint32_t *)(rings + dst[k]) = __builtin_amdgcn_perm(w[k], w[k], 0x00010203u);
    }
};

// Stream held by slot s: fused, stream (r + s) mod M (slot 0 is the one the
// check rebuilds); staged, stream s0 + s, or -1 past the last stream.
template <int G, bool FUSED>
__device__ __forceinline__ void cv_streams(const ConvJob &J, int (&stream)[G])
{
#pragma unroll
    for (int s = 0; s < G; ++s)
        stream[s] = FUSED ? (J.r + s) % J.M : (J.s0 + s < J.M ? J.s0 + s : -1);
}

// Taps [Ia, Ib) (multiples of 256, Ib <= the tap count rounded up to 256)
// of the block of 1024 outputs starting at t0, every digit pass, folded
// into red[slot][position] (uint64, mod 2^64).  Ends after a barrier, with
// red complete.  lds: cv_lds_bytes(G) bytes, 16-byte aligned.
// SPLIT (fused only): the own-stream and previous-stream products of every
// slot are accumulated in two passes of G accumulator sets each instead of
// one pass of 2G (half the accumulator registers, twice the staging).
template <int G, bool FUSED, bool SPLIT = false, bool LIN = false>
__device__ __forceinline__ void conv_accumulate(const ConvJob &J, int64_t t0, int Ia, int Ib,
                                                const int (&stream)[G], int8_t *lds)
{
    static_assert(FUSED || !SPLIT, "split passes are for the fused form");
    constexpr int CH = (FUSED && !SPLIT) ? 2 * G : G; // accumulator sets
    constexpr int HALVES = SPLIT ? 2 : 1;
    int8_t *rings = lds;
    int8_t *gc = lds + cv_rings(G) * kCvRing;
    auto *red = cv_red(lds, G);

    const int tid = threadIdx.x, lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int Ni = (int)J.N, t0i = (int)t0, step_mod = LIN ? kCvStep : kCvStep % Ni;
    // taps with a nonzero column of B, rounded to whole k-steps
    const int Np = LIN ? ((int)J.L + 32 + 31) & ~31 : (Ni + 31) & ~31;
    const int steps = (Ib - Ia) / kCvStep;
    const int a = lane & 31, h = lane >> 5;

    for (int i = tid; i < G * kCvBlock; i += kCvThreads)
        red[i] = 0;

    for (int pass = 0; pass < J.digits * HALVES; ++pass) {
        const int d = pass / HALVES;
        const bool prev = SPLIT && (pass & 1); // this pass: previous-stream products
        cv16i acc[CH];
#pragma unroll
        for (int q = 0; q < CH; ++q)
#pragma unroll
            for (int e = 0; e < 16; ++e)
                acc[q][e] = 0;

        // prologue: ring bytes v in [Ia - 992, Ia + span) and g taps
        // [Ia, Ia + span), span = every step (one shot) or the first one.
        // One shot: the g copies are staged once, and when every digit's
        // rings fit, the rings too (later passes only multiply).  Each round
        // issues all its loads before its stores.
        const bool oneshot = steps <= kCvOneShot;
        const int span = oneshot ? steps * kCvStep : kCvStep;
        const bool alld = oneshot && G * J.digits <= cv_rings(G);
        const bool stage_a = !alld || pass == 0;
        const bool stage_g = !oneshot || pass == 0;
        const int dsel = alld ? d : 0; // ring group of this pass's digit
        constexpr int RA = G <= 4 ? 4 : 2; // ring bytes in flight per thread and round
        const int a_bytes = stage_a ? 992 + span : 0, g_steps = stage_g ? span / kCvStep : 0;
#pragma unroll 1
        for (int r = 0; r * RA * kCvThreads < a_bytes || 2 * r < g_steps; ++r) {
            CvA<G> st[RA];
            CvG sg[2];
            const int k0 = r * RA * kCvThreads;
#pragma unroll
            for (int u = 0; u < RA; ++u) {
                const int v = Ia - 992 + k0 + u * kCvThreads + tid;
                if (k0 + u * kCvThreads + tid < a_bytes) {
                    if constexpr (LIN) {
                        const int idx = t0i + 32 - v;
                        st[u].load(J, stream, idx, v, idx >= 0 && idx < Ni);
                    } else {
                        st[u].load(J, stream, cv_mod(t0i - v, Ni), v);
                    }
                }
            }
#pragma unroll
            for (int u = 0; u < 2; ++u)
                if (2 * r + u < g_steps)
                    sg[u].template load<LIN>(J, Ia + (2 * r + u) * kCvStep, tid);
#pragma unroll
            for (int u = 0; u < RA; ++u)
                if (k0 + u * kCvThreads + tid < a_bytes) {
                    if (alld)
                        st[u].store_all(rings, J.digits, J.x_dtype);
                    else
                        st[u].store(rings, d, J.x_dtype);
                }
#pragma unroll
            for (int u = 0; u < 2; ++u)
                if (2 * r + u < g_steps)
                    sg[u].store(gc);
        }
        // ring coordinate v = Ia + 256 (j + 1) + tid of step j's prefetch,
        // and its input index (t0 - v) mod N, advanced by -256 mod N per step
        // (linear: t0 + 32 - v, advanced by -256, in range or not)
        int pidx = LIN ? t0i + 32 - Ia - kCvStep - tid : cv_mod(t0i - Ia - kCvStep - tid, Ni);
        __syncthreads();

        for (int j = 0; j < steps; ++j) {
            const int I = Ia + j * kCvStep;
            const bool more = !oneshot && j + 1 < steps;
            CvA<G> na;
            CvG ng;
            if (more) {
                na.load(J, stream, pidx, I + kCvStep + tid, !LIN || (pidx >= 0 && pidx < Ni));
                ng.template load<LIN>(J, I + kCvStep, tid);
                pidx -= step_mod;
                if (!LIN && pidx < 0)
                    pidx += Ni;
            }
#pragma unroll
            for (int kk = 0; kk < 2; ++kk) {
                const int i0 = I + 64 * wave + 32 * kk;
                if (i0 < Np) {
                    const cv4i B = *(const cv4i *)(gc + a * kCvGStride +
                                                   ((i0 + 16 * h) & (kCvGRing - 1)));
                    cv4i A[G];
#pragma unroll
                    for (int s = 0; s < G; ++s)
                        A[s] = *(const cv4i *)(rings + (s + G * dsel) * kCvRing +
                                               cv_ring_off(i0 + 16 * h - 32 * a));
#pragma unroll
                    for (int s = 0; s < G; ++s) {
                        if constexpr (SPLIT) {
                            acc[s] = __builtin_amdgcn_mfma_i32_32x32x32_i8(
                                prev ? A[(s + G - 1) % G] : A[s], B, acc[s], 0, 0, 0);
                        } else {
                            acc[s] = __builtin_amdgcn_mfma_i32_32x32x32_i8(A[s], B, acc[s], 0, 0,
                                                                           0);
                            if constexpr (FUSED)
                                acc[G + s] = __builtin_amdgcn_mfma_i32_32x32x32_i8(
                                    A[(s + G - 1) % G], B, acc[G + s], 0, 0, 0);
                        }
                    }
                }
            }
            if (more) {
                na.store(rings, d, J.x_dtype);
                ng.store(gc);
            }
            if (!oneshot)
                __syncthreads();
        }
        if (oneshot)
            __syncthreads(); // every wavefront's reads are done before the fold's next pass

        // fold this digit's products into red (mod 2^64)
#pragma unroll
        for (int s = 0; s < G; ++s)
#pragma unroll
            for (int e = 0; e < 16; ++e) {
                const int row = 8 * (e >> 2) + 4 * h + (e & 3);
                int lo, hi = 0;
                asm volatile("v_accvgpr_read_b32 %0, %1" : "=v"(lo) : "a"(acc[s][e]));
                if constexpr (FUSED && !SPLIT)
                    asm volatile("v_accvgpr_read_b32 %0, %1" : "=v"(hi) : "a"(acc[G + s][e]));
                uint64_t v = (uint64_t)(int64_t)lo;
                if constexpr (FUSED && !SPLIT)
                    v += (uint64_t)(int64_t)hi << J.l;
                if constexpr (SPLIT)
                    v = prev ? v << J.l : v;
                atomicAdd(&red[s * kCvBlock + 32 * row + a], v << (8 * d));
            }
        __syncthreads();
    }
}

// conv_accumulate for the linear form from digit planes (J.planes): the
// same tap loop, with each step's ring bytes staged as plane dwords and two
// steps in flight (the registers of a step are a few dwords per thread).
template <int G, bool FUSED, bool SPLIT = false>
__device__ __forceinline__ void conv_accumulate_pl(const ConvJob &J, int64_t t0, int Ia, int Ib,
                                                   int8_t *lds)
{
    static_assert(FUSED || !SPLIT, "split passes are for the fused form");
    constexpr int CH = (FUSED && !SPLIT) ? 2 * G : G; // accumulator sets
    constexpr int HALVES = SPLIT ? 2 : 1;
    constexpr int NWS = (G * 64 + kCvThreads - 1) / kCvThreads; // ring dwords per thread and step
    int8_t *rings = lds;
    int8_t *gc = lds + cv_rings(G) * kCvRing;
    auto *red = cv_red(lds, G);

    const int tid = threadIdx.x, lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int t0i = (int)t0;
    const int Np = ((int)J.L + 32 + 31) & ~31;
    const int steps = (Ib - Ia) / kCvStep;
    const int a = lane & 31, h = lane >> 5;

    for (int i = tid; i < G * kCvBlock; i += kCvThreads)
        red[i] = 0;

    for (int pass = 0; pass < J.digits * HALVES; ++pass) {
        const int d = pass / HALVES;
        const bool prev = SPLIT && (pass & 1); // this pass: previous-stream products
        cv16i acc[CH];
#pragma unroll
        for (int q = 0; q < CH; ++q)
#pragma unroll
            for (int e = 0; e < 16; ++e)
                acc[q][e] = 0;

        // prologue: ring bytes [Ia - 992, Ia + span) and g taps
        // [Ia, Ia + span) as in conv_accumulate
        const bool oneshot = steps <= kCvOneShot;
        const int span = oneshot ? steps * kCvStep : kCvStep;
        const bool alld = oneshot && G * J.digits <= cv_rings(G);
        const bool stage_a = !alld || pass == 0;
        const bool stage_g = !oneshot || pass == 0;
        const int dsel = alld ? d : 0; // ring group of this pass's digit
        if (stage_a) {
            const int nd = (992 + span) / 4, nr = alld ? G * J.digits : G;
#pragma unroll 1
            for (int u0 = 0; u0 < nr * nd; u0 += 4 * kCvThreads) {
                CvP<4> b;
                b.template load<G, FUSED>(J, t0i, Ia - 992, nd, nr, alld, d, u0, tid);
                b.store(rings);
            }
        }
        if (stage_g) {
#pragma unroll 1
            for (int j = 0; j < span / kCvStep; j += 2) {
                CvG sg[2];
#pragma unroll
                for (int u = 0; u < 2; ++u)
                    if (j + u < span / kCvStep)
                        sg[u].template load<true>(J, Ia + (j + u) * kCvStep, tid);
#pragma unroll
                for (int u = 0; u < 2; ++u)
                    if (j + u < span / kCvStep)
                        sg[u].store(gc);
            }
        }
        // Two steps in flight: while step j is multiplied, step j + 2 is
        // loaded and step j + 1 (loaded one step earlier) is stored; the loop
        // is unrolled by two so that the register sets swap roles.
        auto fetch = [&](CvP<NWS> &pp, CvG &gg, int jj) {
            pp.template load<G, FUSED>(J, t0i, Ia + jj * kCvStep, kCvStep / 4, G, false, d, 0, tid);
            gg.template load<true>(J, Ia + jj * kCvStep, tid);
        };
        CvP<NWS> pa, pb;
        CvG ga, gb;
        if (!oneshot && steps > 1)
            fetch(pa, ga, 1);
        __syncthreads();
        auto step = [&](int j, CvP<NWS> &cur, CvG &gcur, CvP<NWS> &nxt, CvG &gnxt) {
            const int I = Ia + j * kCvStep;
            if (!oneshot && j + 2 < steps)
                fetch(nxt, gnxt, j + 2);
#pragma unroll
            for (int kk = 0; kk < 2; ++kk) {
                const int i0 = I + 64 * wave + 32 * kk;
                if (i0 < Np) {
                    const cv4i B = *(const cv4i *)(gc + a * kCvGStride +
                                                   ((i0 + 16 * h) & (kCvGRing - 1)));
                    cv4i A[G];
#pragma unroll
                    for (int s = 0; s < G; ++s)
                        A[s] = *(const cv4i *)(rings + (s + G * dsel) * kCvRing +
                                               cv_ring_off(i0 + 16 * h - 32 * a));
#pragma unroll
                    for (int s = 0; s < G; ++s) {
                        if constexpr (SPLIT) {
                            acc[s] = __builtin_amdgcn_mfma_i32_32x32x32_i8(
                                prev ? A[(s + G - 1) % G] : A[s], B, acc[s], 0, 0, 0);
                        } else {
                            acc[s] = __builtin_amdgcn_mfma_i32_32x32x32_i8(A[s], B, acc[s], 0, 0,
                                                                           0);
                            if constexpr (FUSED)
                                acc[G + s] = __builtin_amdgcn_mfma_i32_32x32x32_i8(
                                    A[(s + G - 1) % G], B, acc[G + s], 0, 0, 0);
                        }
                    }
                }
            }
            if (!oneshot && j + 1 < steps) {
                cur.store(rings);
                gcur.store(gc);
            }
            if (!oneshot)
                __syncthreads();
        };
        for (int j = 0; j < steps; j += 2) {
            step(j, pa, ga, pb, gb);
            if (j + 1 < steps)
                step(j + 1, pb, gb, pa, ga);
        }
        if (oneshot)
            __syncthreads(); // every wavefront's reads are done before the fold

        // fold this digit's products into red (mod 2^64)
#pragma unroll
        for (int s = 0; s < G; ++s)
#pragma unroll
            for (int e = 0; e < 16; ++e) {
                const int row = 8 * (e >> 2) + 4 * h + (e & 3);
                int lo, hi = 0;
                asm volatile("v_accvgpr_read_b32 %0, %1" : "=v"(lo) : "a"(acc[s][e]));
                if constexpr (FUSED && !SPLIT)
                    asm volatile("v_accvgpr_read_b32 %0, %1" : "=v"(hi) : "a"(acc[G + s][e]));
                uint64_t v = (uint64_t)(int64_t)lo;
                if constexpr (FUSED && !SPLIT)
                    v += (uint64_t)(int64_t)hi << J.l;
                if constexpr (SPLIT)
                    v = prev ? v << J.l : v;
                atomicAdd(&red[s * kCvBlock + 32 * row + a], v << (8 * d));
            }
        __syncthreads();
    }
}

// Finish one output position t of the fused form from the M delta words
// of its slots: disentangle, check, store, and the wavefront's flag words
// (the 64 lanes of a wavefront hold 64 consecutive positions starting at a
// multiple of 64).
template <int M>
__device__ __forceinline__ void conv_finish(const ConvJob &J, const int (&stream)[M], int64_t t,
                                            int64_t (&dd)[M])
{
    const int lane = threadIdx.x & 63;
    const int64_t N = J.Nout;
    const bool valid = t < N;
    int64_t o[M];
    const bool flag = disentangle_rot<M>(dd, J.l, o) && valid;
    if (valid) {
#pragma unroll
        for (int s = 0; s < M; ++s) {
            const int64_t idx = (int64_t)stream[s] * N + t;
            if (J.out64)
                ((int64_t *)J.out)[idx] = o[s];
            else
                ((int32_t *)J.out)[idx] = (int32_t)o[s];
        }
    }
    const uint64_t mask = __ballot(flag);
    const int64_t words = (N + 31) / 32, w0 = (t - lane) / 32;
    if (J.flags) {
        if (lane == 0 && w0 < words)
            J.flags[w0] = (uint32_t)mask;
        if (lane == 32 && w0 + 1 < words)
            J.flags[w0 + 1] = (uint32_t)(mask >> 32);
    }
    if (J.n_bad && lane == 0 && mask)
        atomicAdd(J.n_bad, (unsigned long long)__popcll(mask));
}

// One whole block of 1024 outputs (all taps) in one workgroup.  FUSED:
// G == M, disentangle and check; staged: write delta.
// PL (linear form only): ring bytes from the digit planes of J.planes.
template <int G, bool FUSED, bool SPLIT = false, bool LIN = false, bool PL = false>
__device__ __forceinline__ void conv_block(const ConvJob &J, int64_t block, int8_t *lds)
{
    static_assert(LIN || !PL, "digit planes are for the linear form");
    int stream[G];
    cv_streams<G, FUSED>(J, stream);
    const int64_t t0 = block * kCvBlock;
    const int64_t span = LIN ? J.L + 32 : J.N;
    const int taps = (int)((span + kCvStep - 1) / kCvStep) * kCvStep;
    if constexpr (PL)
        conv_accumulate_pl<G, FUSED, SPLIT>(J, t0, 0, taps, lds);
    else
        conv_accumulate<G, FUSED, SPLIT, LIN>(J, t0, 0, taps, stream, lds);
    const auto *red = cv_red(lds, G);
    const int tid = threadIdx.x;
#pragma unroll 1
    for (int q = 0; q < kCvBlock / kCvThreads; ++q) {
        const int pos = q * kCvThreads + tid;
        const int64_t t = t0 + pos;
        if constexpr (FUSED) {
            int64_t dd[G];
#pragma unroll
            for (int s = 0; s < G; ++s)
                dd[s] = (int64_t)red[s * kCvBlock + pos];
            conv_finish<G>(J, stream, t, dd);
        } else if (t < J.Nout) {
#pragma unroll
            for (int s = 0; s < G; ++s)
                if (stream[s] >= 0)
                    ((int64_t *)J.out)[(int64_t)stream[s] * J.Nout + t] =
                        (int64_t)red[s * kCvBlock + pos];
        }
    }
}

template <int M>
__global__ __launch_bounds__(kCvThreads) void k_conv_fused(const ConvJob J)
{
    __shared__ __attribute__((aligned(16))) int8_t lds[cv_lds_bytes(M)];
    conv_block<M, true>(J, blockIdx.x, lds);
}

template <int G>
__global__ __launch_bounds__(kCvThreads) void k_conv_staged(ConvJob J)
{
    __shared__ __attribute__((aligned(16))) int8_t lds[cv_lds_bytes(G)];
    J.s0 = (int)blockIdx.y * G;
    conv_block<G, false>(J, blockIdx.x, lds);
}

// Linear convolution, one block of 1024 outputs per workgroup: fused
// (entangle, convolve, disentangle, check) and staged (delta out).
template <int M>
__global__ __launch_bounds__(kCvThreads) void k_linconv_fused(const ConvJob J)
{
    __shared__ __attribute__((aligned(16))) int8_t lds[cv_lds_bytes(M)];
    conv_block<M, true, false, true>(J, blockIdx.x, lds);
}

template <int G>
__global__ __launch_bounds__(kCvThreads) void k_linconv_staged(ConvJob J)
{
    __shared__ __attribute__((aligned(16))) int8_t lds[cv_lds_bytes(G)];
    J.s0 = (int)blockIdx.y * G;
    conv_block<G, false, false, true>(J, blockIdx.x, lds);
}

template <int M>
__global__ __launch_bounds__(kCvThreads) void k_linconv_fused_pl(const ConvJob J)
{
    __shared__ __attribute__((aligned(16))) int8_t lds[cv_lds_bytes(M)];
    conv_block<M, true, false, true, true>(J, blockIdx.x, lds);
}

template <int G>
__global__ __launch_bounds__(kCvThreads) void k_linconv_staged_pl(ConvJob J)
{
    __shared__ __attribute__((aligned(16))) int8_t lds[cv_lds_bytes(G)];
    J.s0 = (int)blockIdx.y * G;
    conv_block<G, false, false, true, true>(J, blockIdx.x, lds);
}

// Pre-pass of the plane-staged linear form.  Row m < M of the grid writes
// the digit planes of stream m (one dword of every plane per thread: plane
// bytes 4q .. 4q + 3 hold digits of samples 4q - pad .. 4q - pad + 3, zero
// outside the stream); row M writes g with kCvGPad zero bytes on both sides.
__global__ __launch_bounds__(256) void k_cv_planes(const ConvJob J, int8_t *planes, int8_t *gpad)
{
    const int64_t q = (int64_t)blockIdx.x * 256 + threadIdx.x;
    const int m = blockIdx.y;
    if (m == J.M) {
        const int64_t gbytes = J.L + 2 * kCvGPad;
        if (4 * q >= gbytes)
            return;
        uint32_t w = 0;
#pragma unroll
        for (int b = 0; b < 4; ++b) {
            const int64_t i = 4 * q + b - kCvGPad;
            if (i >= 0 && i < J.L)
                w |= (uint32_t)(uint8_t)J.g[i] << (8 * b);
        }
        *(uint32_t *)(gpad + 4 * q) = w;
        return;
    }
    if (4 * q >= J.P)
        return;
    int64_t v[4];
#pragma unroll
    for (int b = 0; b < 4; ++b) {
        const int64_t i = 4 * q + b - J.pad;
        const bool in = i >= 0 && i < J.N;
        const int64_t ic = (int64_t)m * J.N + (in ? i : 0);
        const int64_t x = J.x_dtype == NE_I64   ? ((const int64_t *)J.x)[ic]
                          : J.x_dtype == NE_I32 ? ((const int32_t *)J.x)[ic]
                                                : ((const int8_t *)J.x)[ic];
        v[b] = in ? x : 0;
    }
    for (int d = 0; d < J.digits; ++d) {
        uint32_t w = 0;
#pragma unroll
        for (int b = 0; b < 4; ++b)
            w |= (uint32_t)(uint8_t)digit(v[b]) << (8 * b);
        *(uint32_t *)(planes + ((int64_t)m * J.digits + d) * J.P + 4 * q) = w;
    }
}

// Split taps: workgroup (block, z, group) accumulates taps [z KC, (z+1) KC)
// and writes its 64-bit partial sums to ws[z][stream or slot][position]
// (positions padded to whole blocks: Nb = blocks * 1024).
template <int G, bool FUSED>
__global__ __launch_bounds__(kCvThreads) void k_conv_part(ConvJob J, uint64_t *ws, int KC,
                                                          int slots)
{
    __shared__ __attribute__((aligned(16))) int8_t lds[cv_lds_bytes(G)];
    J.s0 = (int)blockIdx.z * G;
    int stream[G];
    cv_streams<G, FUSED>(J, stream);
    const int64_t t0 = (int64_t)blockIdx.x * kCvBlock;
    const int taps = (int)((J.N + kCvStep - 1) / kCvStep) * kCvStep;
    const int z = blockIdx.y, Ia = z * KC, Ib = Ia + KC < taps ? Ia + KC : taps;
    conv_accumulate<G, FUSED>(J, t0, Ia, Ib, stream, lds);
    const auto *red = cv_red(lds, G);
    const int64_t Nb = (int64_t)gridDim.x * kCvBlock;
    for (int i = threadIdx.x; i < G * kCvBlock; i += kCvThreads) {
        const int s = i / kCvBlock, pos = i % kCvBlock;
        const int row = FUSED ? s : stream[s];
        if (row >= 0)
            ws[((int64_t)z * slots + row) * Nb + t0 + pos] = red[i];
    }
}

// Sum the partials of every split and finish: fused, disentangle and check
// (M == slots); staged, write delta.  One thread per position.
template <int M, bool FUSED>
__global__ __launch_bounds__(256) void k_conv_reduce(const ConvJob J, const uint64_t *ws, int S,
                                                     int64_t Nb)
{
    const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if constexpr (FUSED) {
        int stream[M];
        cv_streams<M, true>(J, stream);
        int64_t dd[M];
        const int64_t tc = t < Nb ? t : 0;
#pragma unroll
        for (int s = 0; s < M; ++s)
            dd[s] = 0;
        // four splits per round, all loads of a round in flight together
        for (int z0 = 0; z0 < S; z0 += 4) {
            uint64_t v[4][M];
#pragma unroll
            for (int u = 0; u < 4; ++u)
#pragma unroll
                for (int s = 0; s < M; ++s)
                    v[u][s] = z0 + u < S ? ws[((int64_t)(z0 + u) * M + s) * Nb + tc] : 0;
#pragma unroll
            for (int u = 0; u < 4; ++u)
#pragma unroll
                for (int s = 0; s < M; ++s)
                    dd[s] = (int64_t)((uint64_t)dd[s] + v[u][s]);
        }
        conv_finish<M>(J, stream, t, dd);
    } else {
        if (t >= J.N)
            return;
        for (int m = 0; m < J.M; ++m) {
            uint64_t v = 0;
            for (int z = 0; z < S; ++z)
                v += ws[((int64_t)z * J.M + m) * Nb + t];
            ((int64_t *)J.out)[(int64_t)m * J.N + t] = (int64_t)v;
        }
    }
}

} // namespace
} // namespace ne
