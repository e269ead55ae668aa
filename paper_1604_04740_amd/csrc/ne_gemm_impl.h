// ne_gemm_impl.h -- int8 matrix-core GEMM device code for gfx950 (shared by
// the GEMM entry points and the batched persistent kernel).
//
// One kernel template, six variants:
//   PlainV     C = A * B, int8 -> int32 (the fault-intolerant baseline)
//   EpsV<L>    delta = eps * G on generic int64 words: each word is split
//              into L signed int8 digits in the prologue, one exact int32
//              accumulator per digit, recombined modulo 2^64 (the LSB
//              routine, unaware of entanglement, of section III-A)
//   FusedV<M>  the hot path: entangle in the prologue (the digits of
//              eps_m = c_m + 2^l c_{m-1} at bit offsets 0 and l are c_m and
//              c_{m-1}), two independent int32 products per stream,
//              delta_m = P_lo + 2^l P_hi, then disentangle and check in the
//              epilogue (section III-C); delta never leaves registers
//   SeriesV<M> the GEMM at the head of an operation series (section II):
//              FusedV's prologue and products, then scale and add on the
//              entangled words in the epilogue, stored position-major for
//              the operation that follows; no disentangle
//   AbftDmaV<M> the same ABFT with the checksum stream built beforehand as
//              two int8 digit planes, so every source goes through the DMA
//              pipeline of FusedV
//   AbftV<M>   checksum-stream ABFT of section II-A: the checksum row
//              sum_m c_m (two int8 digits) is built in the prologue and
//              multiplied alongside the M streams; the epilogue checks
//              sum_m d_m == e
//
// Structure (all variants): 256 threads = 4 wavefronts; a workgroup tile
// holds NSRC source row-blocks of BMS rows and BN columns of Bt in LDS, with
// BK = 64 bytes of K per stage, double-buffered.  Rows are stored as four
// 16-byte chunks whose position is XOR-swizzled by the row so that the
// 64-lane ds_read_b128 fragment reads and the ds_write_b128 stores hit
// distinct banks.  Each wavefront reads, per 32-wide k-step, one 32x32 A
// fragment per source and one B fragment per column block and issues
// v_mfma_i32_32x32x32_i8 for every (accumulator set, row block, column
// block); an A fragment feeds every accumulator set that uses its source
// (in FusedV each c_m fragment feeds stream m's low digit and stream m+1's
// high digit).  Tiles are ordered so that the tiles resident on one XCD
// (workgroups are dealt round-robin over the 8 XCDs) are neighbours in
// groups of 8 row tiles, sharing A rows and B columns in that XCD's L2.
#pragma once

#include "ne_arith.h"
#include "ne_internal.h"

namespace ne {
namespace {

typedef int v4i __attribute__((ext_vector_type(4)));
typedef int v16i __attribute__((ext_vector_type(16)));

#ifndef NE_GEMM_BK
#define NE_GEMM_BK 64
#endif
#ifndef NE_GEMM_STAGES
#define NE_GEMM_STAGES 4
#endif

constexpr int kThreads = 256;
constexpr int BK = 64;
constexpr int kChunks = BK / 16;

__device__ __forceinline__ int lds_off(int row, int chunk)
{
    return row * BK + ((chunk ^ ((row >> 2) & (kChunks - 1))) << 4);
}

__device__ __forceinline__ v16i mfma(v4i a, v4i b, v16i c)
{
    return __builtin_amdgcn_mfma_i32_32x32x32_i8(a, b, c, 0, 0, 0);
}

// 16 bytes of a row starting at element k (zero outside [0, K) or invalid row).
template <bool AL>
__device__ __forceinline__ v4i load_chunk(const int8_t *row_ptr, int64_t k, int64_t K, bool row_ok)
{
    v4i v = {0, 0, 0, 0};
    if (!row_ok || k >= K)
        return v;
    if (AL) {
        v = *(const v4i *)(row_ptr + k);
        return v;
    }
    // Rows that are not 16-byte aligned: the widest aligned loads the
    // address allows for a whole chunk (rows of K = 8j or 4j bytes), else
    // bytes.  Every load of a chunk is issued before any result is used (a
    // value consumed right after its load would serialise the loads).
    const int8_t *src = row_ptr + k;
    const uintptr_t a = (uintptr_t)src;
    if (k + 16 <= K && (a & 7) == 0) {
        const uint2 x = *(const uint2 *)src, y = *(const uint2 *)(src + 8);
        v[0] = (int)x.x;
        v[1] = (int)x.y;
        v[2] = (int)y.x;
        v[3] = (int)y.y;
    } else if (k + 16 <= K && (a & 3) == 0) {
        const uint32_t *q = (const uint32_t *)src;
        const uint32_t x0 = q[0], x1 = q[1], x2 = q[2], x3 = q[3];
        v[0] = (int)x0;
        v[1] = (int)x1;
        v[2] = (int)x2;
        v[3] = (int)x3;
    } else {
        // bytes past the end of the row are read from its last byte and
        // masked off after every load has been issued
        uint32_t b[16];
#pragma unroll
        for (int j = 0; j < 16; ++j)
            b[j] = (uint32_t)(uint8_t)src[k + j < K ? j : K - 1 - k];
        uint32_t w[4] = {0, 0, 0, 0};
#pragma unroll
        for (int j = 0; j < 16; ++j)
            w[j >> 2] |= (k + j < K ? b[j] : 0u) << (8 * (j & 3));
        v[0] = (int)w[0];
        v[1] = (int)w[1];
        v[2] = (int)w[2];
        v[3] = (int)w[3];
    }
    return v;
}

__device__ __forceinline__ void tile_coords(int tiles_m, int tiles_n, int &tm, int &tn)
{
    int b = blockIdx.x;
    const int nb = gridDim.x;
    if ((nb & 7) == 0)
        b = (b & 7) * (nb >> 3) + (b >> 3);
    constexpr int GM = 8;
    const int per_group = GM * tiles_n;
    const int g = b / per_group;
    const int first = g * GM;
    const int gm = min(GM, tiles_m - first);
    const int in = b - g * per_group;
    tm = first + in % gm;
    tn = in / gm;
}

// Row (within a 32-row block) and column (within a 32-column block) of
// accumulator register r of lane `lane` for v_mfma_i32_32x32x32_i8.
__device__ __forceinline__ int acc_row(int r, int lane) { return 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3); }
__device__ __forceinline__ int acc_col(int lane) { return lane & 31; }

// Shared B-operand (Bt, [N][K] int8) staging: BN rows x 4 chunks.
template <int BN, bool AL>
struct BStage {
    static constexpr int CH = BN * kChunks;
    static constexpr int NB = (CH + kThreads - 1) / kThreads;
    v4i b[NB];
    __device__ __forceinline__ void load(const int8_t *Bt, int64_t N, int64_t K, int64_t col0,
                                         int64_t k0, int tid)
    {
#pragma unroll
        for (int i = 0; i < NB; ++i) {
            const int q = tid + i * kThreads;
            const int row = q / kChunks, ch = q % kChunks;
            const int64_t col = col0 + row;
            b[i] = (q < CH) ? load_chunk<AL>(Bt + col * K, k0 + ch * 16, K, col < N)
                            : v4i{0, 0, 0, 0};
        }
    }
    __device__ __forceinline__ void store(int8_t *lds_b, int tid) const
    {
#pragma unroll
        for (int i = 0; i < NB; ++i) {
            const int q = tid + i * kThreads;
            if (q < CH)
                *(v4i *)(lds_b + lds_off(q / kChunks, q % kChunks)) = b[i];
        }
    }
};

// ----------------------------------------------------------------- kernel

template <class V, bool AL>
__global__ __launch_bounds__(kThreads, V::kOcc) void k_gemm(const typename V::Args args)
{
    constexpr int NSRC = V::NSRC, P = V::P, BMS = V::BMS, BN = V::BN, WM = V::WM, WN = V::WN;
    constexpr int RB = BMS / (32 * WM), CB = BN / (32 * WN);
    constexpr int A_BYTES = NSRC * BMS * BK;
    constexpr int STAGE = A_BYTES + BN * BK;
    static_assert(WM * WN == 4, "four wavefronts");
    static_assert(RB >= 1 && CB >= 1, "tile too small");

    __shared__ __attribute__((aligned(16))) int8_t lds[2 * STAGE];

    const int tid = threadIdx.x, lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6); // uniform per wavefront
    const int wm = wave / WN, wn = wave % WN;
    int tm, tn;
    tile_coords(args.tiles_m, args.tiles_n, tm, tn);
    const int64_t row0 = (int64_t)tm * BMS, col0 = (int64_t)tn * BN;

    v16i acc[P][RB][CB];
#pragma unroll
    for (int p = 0; p < P; ++p)
#pragma unroll
        for (int i = 0; i < RB; ++i)
#pragma unroll
            for (int j = 0; j < CB; ++j)
#pragma unroll
                for (int r = 0; r < 16; ++r)
                    acc[p][i][j][r] = 0;

    typename V::template AStage<AL> sa;
    BStage<BN, AL> sb;
    const int nk = (int)((args.K + BK - 1) / BK);

    sa.load(args, row0, 0, tid);
    sb.load(args.Bt, args.N, args.K, col0, 0, tid);
    sa.store(lds, tid);
    sb.store(lds + A_BYTES, tid);
    __syncthreads();

    for (int kt = 0; kt < nk; ++kt) {
        const int8_t *cur = lds + (kt & 1) * STAGE;
        const bool more = kt + 1 < nk;
        if (more) {
            sa.load(args, row0, (int64_t)(kt + 1) * BK, tid);
            sb.load(args.Bt, args.N, args.K, col0, (int64_t)(kt + 1) * BK, tid);
        }
#pragma unroll
        for (int ks = 0; ks < BK / 32; ++ks) {
            const int chunk = ks * 2 + (lane >> 5);
            v4i a[NSRC][RB], b[CB];
#pragma unroll
            for (int s = 0; s < NSRC; ++s)
#pragma unroll
                for (int i = 0; i < RB; ++i) {
                    const int row = (wm * RB + i) * 32 + (lane & 31);
                    a[s][i] = *(const v4i *)(cur + s * BMS * BK + lds_off(row, chunk));
                }
#pragma unroll
            for (int j = 0; j < CB; ++j) {
                const int row = (wn * CB + j) * 32 + (lane & 31);
                b[j] = *(const v4i *)(cur + A_BYTES + lds_off(row, chunk));
            }
#pragma unroll
            for (int p = 0; p < P; ++p)
#pragma unroll
                for (int i = 0; i < RB; ++i)
#pragma unroll
                    for (int j = 0; j < CB; ++j)
                        acc[p][i][j] = mfma(a[V::src(p)][i], b[j], acc[p][i][j]);
        }
        if (more) {
            int8_t *nxt = lds + ((kt + 1) & 1) * STAGE;
            sa.store(nxt, tid);
            sb.store(nxt + A_BYTES, tid);
        }
        __syncthreads();
    }

    V::epilogue(args, acc, row0, col0, wm, wn, lane);
}

// ------------------------------------------------- DMA-fed kernel (gfx950)
//
// Variants whose A sources are raw int8 rows (PlainV, FusedV) use a ring of
// S LDS stages filled by buffer_load_dwordx4 ... lds: each instruction moves
// 64 x 16 bytes from global memory straight into 1 KB of LDS, so no VGPRs are
// spent on staging and S-1 tiles are in flight.  Each lane picks the global
// chunk that belongs at its LDS slot under the XOR swizzle.  Out-of-range
// rows, columns and k read as zero through the buffer descriptor's range
// check (per-source descriptors start at the tile's first row).  Waits are
// explicit: before computing tile kt a wavefront waits until only the loads
// of the tiles after kt are outstanding, then the workgroup barrier makes
// every wavefront's share of tile kt visible and frees the stage that the
// next tile is loaded into.

typedef __amdgpu_buffer_rsrc_t rsrc_t;
constexpr unsigned kOOB = 0x80000000u;   // beyond every descriptor's range
constexpr int kRsrcWord3 = 0x00020000;   // raw buffer, 32-bit data format

__device__ __forceinline__ rsrc_t make_rsrc(const void *base, int64_t bytes)
{
    return __builtin_amdgcn_make_buffer_rsrc((void *)base, (short)0, (int)bytes, kRsrcWord3);
}

template <int BK_>
__device__ __forceinline__ int swz_off(int row, int chunk)
{
    constexpr int C = BK_ / 16;                 // chunks per row
    constexpr int SH = (C == 4) ? 2 : (C == 8 ? 1 : 0);
    return row * BK_ + ((chunk ^ ((row >> SH) & (C - 1))) << 4);
}

// vmcnt-only wait followed by the workgroup barrier (no memory fence: the
// only outstanding memory operations are this wavefront's LDS DMA loads).
template <int N>
__device__ __forceinline__ void wait_vm_barrier()
{
    static_assert(N >= 0 && N < 64, "vmcnt range");
    asm volatile("s_waitcnt vmcnt(%0)\n\ts_barrier" ::"n"(N) : "memory");
}

// Issue this wavefront's share of the DMA loads of k-tile kt into LDS stage
// `stage`: regions g = wave, wave + 4, ... of 1 KB; A regions first (source
// by source), then B.
template <int NSRC, int BMS, int BN, int BK_, int PART = 0, int NPARTS = 1>
__device__ __forceinline__ void dma_tile(int8_t *stage, const rsrc_t *ra, rsrc_t rb,
                                         int64_t k0, int64_t K, int wave, int lane)
{
    constexpr int C = BK_ / 16, RPR = 1024 / BK_, RPS = BMS / RPR; // regions per source
    constexpr int A_REG = NSRC * RPS, REG = A_REG + BN / RPR;
    // Region g = 4 * round + wave: with these multiples of four every round is
    // all-A or all-B and reads one source, so the descriptor is a constant
    // and the issue has no branches (it can then be interleaved with MFMAs).
    static_assert(A_REG % 4 == 0 && REG % 4 == 0 && (RPS % 4 == 0 || 4 % RPS == 0),
                  "DMA region layout");
    constexpr int ROUNDS = REG / 4;
    constexpr int PER = (ROUNDS + NPARTS - 1) / NPARTS;
    const int r_in = lane / C, pc = lane % C;
#pragma unroll
    for (int rd = PART * PER; rd < ROUNDS && rd < (PART + 1) * PER; ++rd) {
        const int g = rd * 4 + wave;
        const bool isA = rd * 4 < A_REG;                       // same for all waves
        const int gg = isA ? g : g - A_REG;
        const int row = (isA ? gg % RPS : gg) * RPR + r_in;
        const int lc = pc ^ ((row >> (C == 4 ? 2 : 1)) & (C - 1));
        const int64_t k = k0 + lc * 16;
        const unsigned off = (k < K) ? (unsigned)(row * K + k) : kOOB;
        auto *dst = (__attribute__((address_space(3))) void *)(stage + g * 1024);
        if (isA) {
            constexpr int dummy = 0;
            (void)dummy;
            // source of this round: rd * 4 / RPS when RPS is a multiple of 4,
            // else every wave of the round reads a different source row-block
            if constexpr (RPS % 4 == 0) {
#pragma unroll
                for (int s2 = 0; s2 < NSRC; ++s2)
                    if (s2 == rd * 4 / RPS)
                        __builtin_amdgcn_raw_ptr_buffer_load_lds(ra[s2], dst, 16, off, 0, 0, 0);
            } else {
#pragma unroll
                for (int s2 = 0; s2 < NSRC; ++s2)
                    if (s2 == g / RPS)
                        __builtin_amdgcn_raw_ptr_buffer_load_lds(ra[s2], dst, 16, off, 0, 0, 0);
            }
        } else {
            __builtin_amdgcn_raw_ptr_buffer_load_lds(rb, dst, 16, off, 0, 0, 0);
        }
    }
}

// Fragments of one 32-wide k-step: an A fragment per (source, row block)
// and a B fragment per column block (ds_read_b128 each).
template <int NSRC, int RB, int CB, int BMS, int BK_, int A_BYTES>
__device__ __forceinline__ void load_frags(const int8_t *cur, int ks, int wm, int wn, int lane,
                                           v4i (&a)[NSRC][RB], v4i (&b)[CB])
{
    const int chunk = ks * 2 + (lane >> 5);
#pragma unroll
    for (int s = 0; s < NSRC; ++s)
#pragma unroll
        for (int i = 0; i < RB; ++i) {
            const int row = (wm * RB + i) * 32 + (lane & 31);
            a[s][i] = *(const v4i *)(cur + s * BMS * BK_ + swz_off<BK_>(row, chunk));
        }
#pragma unroll
    for (int j = 0; j < CB; ++j) {
        const int row = (wn * CB + j) * 32 + (lane & 31);
        b[j] = *(const v4i *)(cur + A_BYTES + swz_off<BK_>(row, chunk));
    }
}

// Scheduling hint for one k-step: alternate MFMA and LDS read so that the
// reads of the next k-step are issued in the shadow of this step's MFMAs.
template <int NMFMA, int NREAD, int NDMA>
__device__ __forceinline__ void interleave()
{
#pragma unroll
    for (int i = 0; i < NMFMA; ++i) {
        __builtin_amdgcn_sched_group_barrier(0x008, 1, 0); // one MFMA
        if (i < NREAD)
            __builtin_amdgcn_sched_group_barrier(0x100, 1, 0); // one LDS read
        if (i >= NMFMA - NDMA)
            __builtin_amdgcn_sched_group_barrier(0x020, 1, 0); // one global->LDS copy
    }
    if (NREAD > NMFMA)
        __builtin_amdgcn_sched_group_barrier(0x100, NREAD - NMFMA, 0);
}

// k-step ks issues part ks of the next tile's DMA (KS parts in total).
template <int NSRC, int BMS, int BN, int BK_, int KS>
__device__ __forceinline__ void dma_part(int ks, int8_t *stage, const rsrc_t *ra,
                                         rsrc_t rb, int64_t k0, int64_t K, int wave, int lane)
{
    if (ks == 0) dma_tile<NSRC, BMS, BN, BK_, 0, KS>(stage, ra, rb, k0, K, wave, lane);
    if constexpr (KS > 1) if (ks == 1) dma_tile<NSRC, BMS, BN, BK_, 1, KS>(stage, ra, rb, k0, K, wave, lane);
    if constexpr (KS > 2) if (ks == 2) dma_tile<NSRC, BMS, BN, BK_, 2, KS>(stage, ra, rb, k0, K, wave, lane);
    if constexpr (KS > 3) if (ks == 3) dma_tile<NSRC, BMS, BN, BK_, 3, KS>(stage, ra, rb, k0, K, wave, lane);
}

// Workgroups per CU for the DMA kernel: the variant's register-based target,
// capped by what its LDS ring leaves room for (160 KB per CU).
template <class V, int BK_, int S>
constexpr int dma_occ()
{
    constexpr int bytes = S * (V::NSRC * V::BMS * BK_ + V::BN * BK_);
    constexpr int by_lds = (160 * 1024) / bytes;
    return V::kOcc < by_lds ? V::kOcc : (by_lds < 1 ? 1 : by_lds);
}

// One output tile (tm, tn) of variant V with an S-stage LDS ring at `lds`
// (S * stage bytes, 1 KB aligned).  Called by k_gemm_dma (one tile per
// workgroup) and by the batched persistent kernel.
template <class V, int BK_, int S>
constexpr int dma_lds_bytes()
{
    return S * (V::NSRC * V::BMS * BK_ + V::BN * BK_);
}

template <class V, int BK_, int S>
__device__ __forceinline__ void gemm_tile_dma(const typename V::Args &args, int tm, int tn,
                                              int8_t *lds)
{
    constexpr int NSRC = V::NSRC, P = V::P, BMS = V::BMS, BN = V::BN, WM = V::WM, WN = V::WN;
    constexpr int RB = BMS / (32 * WM), CB = BN / (32 * WN);
    constexpr int RPR = 1024 / BK_;                // rows per 1 KB DMA region
    constexpr int A_BYTES = NSRC * BMS * BK_;
    constexpr int STAGE = A_BYTES + BN * BK_;
    constexpr int A_REG = NSRC * BMS / RPR, B_REG = BN / RPR, REG = A_REG + B_REG;
    constexpr int LOADS_MIN = REG / 4;             // DMA instructions per tile, fewest over waves
    static_assert(WM * WN == 4, "four wavefronts");
    static_assert(BMS % RPR == 0 && BN % RPR == 0, "regions must not straddle sources");
    static_assert(S >= 2 && S <= 8, "stages");

    const int tid = threadIdx.x, lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6); // uniform per wavefront
    const int wm = wave / WN, wn = wave % WN;
    const int64_t row0 = (int64_t)tm * BMS, col0 = (int64_t)tn * BN;
    const int64_t K = args.K;

    // One descriptor per A source and one for B, each starting at the tile.
    rsrc_t ra[NSRC];
#pragma unroll
    for (int s = 0; s < NSRC; ++s) {
        const int64_t rows = V::source_rows(args, s, row0);
        ra[s] = make_rsrc(V::source_base(args, s, row0), (rows < BMS ? rows : BMS) * K);
    }
    const int64_t bcols = args.N - col0;
    const rsrc_t rb = make_rsrc(args.Bt + col0 * K, (bcols < BN ? bcols : BN) * K);


    v16i acc[P][RB][CB];
#pragma unroll
    for (int p = 0; p < P; ++p)
#pragma unroll
        for (int i = 0; i < RB; ++i)
#pragma unroll
            for (int j = 0; j < CB; ++j)
#pragma unroll
                for (int r = 0; r < 16; ++r)
                    acc[p][i][j][r] = 0;

    const int nk = (int)((K + BK_ - 1) / BK_);
    // Prologue: tiles 0 .. S-2.  Every iteration then issues exactly one
    // tile's loads (past the last tile, range-checked dummies that fill the
    // free stage with zeros without touching memory), so the number of loads
    // allowed in flight at each wait is the same constant.
#pragma unroll
    for (int t = 0; t < S - 1; ++t)
        dma_tile<NSRC, BMS, BN, BK_>(lds + t * STAGE, ra, rb, t < nk ? (int64_t)t * BK_ : K, K,
                                     wave, lane);

    constexpr int KS = BK_ / 32;
    constexpr int DMA_PER_KS = ((REG + 3) / 4 + KS - 1) / KS; // per wave, per k-step
    for (int kt = 0; kt < nk; ++kt) {
        wait_vm_barrier<(S - 2) * LOADS_MIN>();
        const int tn = kt + S - 1;
        int8_t *nxt = lds + (tn % S) * STAGE;
        const int64_t nk0 = tn < nk ? (int64_t)tn * BK_ : K;

        const int8_t *cur = lds + (kt % S) * STAGE;
        // Fragments of k-step ks+1 are read while the MFMAs of k-step ks
        // issue (two register sets), one LDS read in the shadow of each MFMA.
        v4i fa[2][NSRC][RB], fb[2][CB];
        load_frags<NSRC, RB, CB, BMS, BK_, A_BYTES>(cur, 0, wm, wn, lane, fa[0], fb[0]);
#pragma unroll
        for (int ks = 0; ks < KS; ++ks) {
            __builtin_amdgcn_sched_barrier(0); // each k-step is its own scheduling region
            const int c = ks & 1;
            if (ks + 1 < KS)
                load_frags<NSRC, RB, CB, BMS, BK_, A_BYTES>(cur, ks + 1, wm, wn, lane, fa[c ^ 1],
                                                            fb[c ^ 1]);
            // this k-step's share of the next tile's global -> LDS copies
            dma_part<NSRC, BMS, BN, BK_, KS>(ks, nxt, ra, rb, nk0, K, wave, lane);
#pragma unroll
            for (int p = 0; p < P; ++p)
#pragma unroll
                for (int i = 0; i < RB; ++i)
#pragma unroll
                    for (int j = 0; j < CB; ++j)
                        acc[p][i][j] = mfma(fa[c][V::src(p)][i], fb[c][j], acc[p][i][j]);
            if (ks + 1 < KS)
                interleave<P * RB * CB, NSRC * RB + CB, DMA_PER_KS>();
            else
                interleave<P * RB * CB, 0, DMA_PER_KS>();
        }
    }
    // The dummy loads of the last iterations still target the LDS ring: let
    // them land before the caller (the batch kernel) reuses that memory.
    asm volatile("s_waitcnt vmcnt(0)" ::: "memory");

    V::epilogue(args, acc, row0, col0, wm, wn, lane);
}

template <class V, int BK_, int S>
__global__ __launch_bounds__(kThreads, (dma_occ<V, BK_, S>())) void k_gemm_dma(const typename V::Args args)
{
    __shared__ __attribute__((aligned(1024))) int8_t lds[dma_lds_bytes<V, BK_, S>()];
    int tm, tn;
    tile_coords(args.tiles_m, args.tiles_n, tm, tn);
    gemm_tile_dma<V, BK_, S>(args, tm, tn, lds);
}
// Common argument block.
struct ArgsBase {
    const int8_t *Bt;
    int64_t K, N;
    int tiles_m, tiles_n;
};

// ------------------------------------------------------------------ plain

#ifndef NE_PLAIN_BK
#define NE_PLAIN_BK 128
#endif
#ifndef NE_PLAIN_STAGES
#define NE_PLAIN_STAGES 2
#endif

// 256 x 256 workgroup tile, each wavefront 128 x 128 (16 accumulator blocks,
// 256 accumulator registers): half the LDS fragment traffic per MFMA of a
// 128 x 64 wavefront tile, which is what bounds this loop on gfx950.
struct PlainV {
    static constexpr int NSRC = 1, P = 1, BMS = 256, BN = 256, WM = 2, WN = 2;
    static constexpr int kOcc = 1;
    static constexpr bool kDma = true;
    static constexpr int kBK = NE_PLAIN_BK, kStages = NE_PLAIN_STAGES;
    static constexpr int RB = BMS / (32 * WM), CB = BN / (32 * WN);
    __host__ __device__ static constexpr int src(int) { return 0; }
    struct Args : ArgsBase {
        const int8_t *A;
        int32_t *C;
        int64_t R;
    };
    __device__ __forceinline__ static const int8_t *source_base(const Args &g, int, int64_t row0)
    {
        return g.A + row0 * g.K;
    }
    __device__ __forceinline__ static int64_t source_rows(const Args &g, int, int64_t row0)
    {
        return g.R - row0;
    }
    template <bool AL> struct AStage {
        static constexpr int CH = BMS * kChunks;
        static constexpr int NA = CH / kThreads;
        v4i a[NA];
        __device__ __forceinline__ void load(const Args &g, int64_t row0, int64_t k0, int tid)
        {
#pragma unroll
            for (int i = 0; i < NA; ++i) {
                const int q = tid + i * kThreads;
                const int64_t row = row0 + q / kChunks;
                a[i] = load_chunk<AL>(g.A + row * g.K, k0 + (q % kChunks) * 16, g.K, row < g.R);
            }
        }
        __device__ __forceinline__ void store(int8_t *lds_a, int tid) const
        {
#pragma unroll
            for (int i = 0; i < NA; ++i) {
                const int q = tid + i * kThreads;
                *(v4i *)(lds_a + lds_off(q / kChunks, q % kChunks)) = a[i];
            }
        }
    };
    __device__ __forceinline__ static void epilogue(const Args &g, v16i (&acc)[P][RB][CB],
                                                    int64_t row0, int64_t col0, int wm, int wn,
                                                    int lane)
    {
#pragma unroll
        for (int i = 0; i < RB; ++i)
#pragma unroll
            for (int j = 0; j < CB; ++j) {
                const int64_t col = col0 + (wn * CB + j) * 32 + acc_col(lane);
#pragma unroll
                for (int r = 0; r < 16; ++r) {
                    const int64_t row = row0 + (wm * RB + i) * 32 + acc_row(r, lane);
                    if (row < g.R && col < g.N)
                        g.C[row * g.N + col] = acc[0][i][j][r];
                }
            }
    }
};

// ---------------------------------------------------- staged GEMM on eps

template <int L>
struct EpsV {
    static constexpr int NSRC = L, P = L, BMS = 32, BN = 128, WM = 1, WN = 4;
    static constexpr int kOcc = (L <= 6) ? 2 : 1;
    static constexpr bool kDma = false;
    static constexpr int RB = 1, CB = 1;
    __host__ __device__ static constexpr int src(int p) { return p; }
    struct Args : ArgsBase {
        const int64_t *eps;
        int64_t *delta;
        int64_t R;
    };
    template <bool AL> struct AStage {
        static constexpr int UNITS = BMS * kChunks; // (row, 16-element chunk)
        static_assert(UNITS <= kThreads, "one unit per thread");
        int64_t x[16];
        __device__ __forceinline__ void load(const Args &g, int64_t row0, int64_t k0, int tid)
        {
            if (tid < UNITS) {
                const int64_t row = row0 + tid / kChunks;
                const int64_t k = k0 + (tid % kChunks) * 16;
                const int64_t *p = g.eps + row * g.K;
#pragma unroll
                for (int e = 0; e < 16; ++e)
                    x[e] = (row < g.R && k + e < g.K) ? p[k + e] : 0;
            }
        }
        __device__ __forceinline__ void store(int8_t *lds_a, int tid) const
        {
            if (tid < UNITS) {
                const int row = tid / kChunks, ch = tid % kChunks;
                uint32_t w[L][4];
#pragma unroll
                for (int j = 0; j < L; ++j)
#pragma unroll
                    for (int q = 0; q < 4; ++q)
                        w[j][q] = 0;
#pragma unroll
                for (int e = 0; e < 16; ++e) {
                    int64_t v = x[e];
#pragma unroll
                    for (int j = 0; j < L; ++j)
                        w[j][e >> 2] |= (uint32_t)(uint8_t)digit(v) << (8 * (e & 3));
                }
#pragma unroll
                for (int j = 0; j < L; ++j)
                    *(v4i *)(lds_a + j * BMS * BK + lds_off(row, ch)) =
                        v4i{(int)w[j][0], (int)w[j][1], (int)w[j][2], (int)w[j][3]};
            }
        }
    };
    __device__ __forceinline__ static void epilogue(const Args &g, v16i (&acc)[P][RB][CB],
                                                    int64_t row0, int64_t col0, int wm, int wn,
                                                    int lane)
    {
        const int64_t col = col0 + wn * 32 + acc_col(lane);
#pragma unroll
        for (int r = 0; r < 16; ++r) {
            const int64_t row = row0 + wm * 32 + acc_row(r, lane);
            uint64_t d = 0;
#pragma unroll
            for (int j = 0; j < L; ++j)
                d += (uint64_t)(int64_t)acc[j][0][0][r] << (8 * j);
            if (row < g.R && col < g.N)
                g.delta[row * g.N + col] = (int64_t)d;
        }
    }
};

// ------------------------------------------------------- fused hot path

#ifndef NE_FUSED_BK
#define NE_FUSED_BK 128
#endif
#ifndef NE_FUSED_STAGES
#define NE_FUSED_STAGES 3
#endif

// Workgroup tile: 32 rows of every stream x BN columns; each wavefront owns
// BN/4 columns of those rows for all M streams and both digits, i.e.
// 2 * M * (BN / 128) accumulator blocks (at most 256 registers).
// INJ: the variant that XORs a device list of faults into the entangled
// words before the check (fault-injection runs); a separate kernel, so the
// production kernel carries none of it.
template <int M, int BN_ = (M <= 4) ? 256 : 128, bool INJ = false>
struct FusedV {
    static constexpr int NSRC = M, P = 2 * M, BMS = 32, BN = BN_, WM = 1, WN = 4;
    static constexpr int kOcc = 1;
    static constexpr bool kDma = true;
    static constexpr int kBK = NE_FUSED_BK, kStages = NE_FUSED_STAGES;
    static constexpr int RB = 1, CB = BN / 128;
    // accumulator set p < M: low digit (c_p) of stream p; p >= M: high digit
    // (c_{p-M-1 mod M}) of stream p - M.
    __host__ __device__ static constexpr int src(int p) { return p < M ? p : (p - 1) % M; }
    struct Args : ArgsBase {
        const int8_t *c;
        void *dhat;
        uint32_t *flags;
        unsigned long long *n_bad;
        const int64_t *inj_pos;
        const int32_t *inj_stream;
        const uint64_t *inj_mask;
        int64_t inj_count;
        int64_t n;
        int l, r, out64;
    };
    // Slot s holds stream (r + s) mod M, so that the stream the check
    // rebuilds (r) sits in slot 0 and the epilogue arithmetic is the same for
    // every r.
    __device__ __forceinline__ static int stream_of(const Args &g, int s) { return (g.r + s) % M; }
    __device__ __forceinline__ static const int8_t *source_base(const Args &g, int s, int64_t row0)
    {
        return g.c + ((int64_t)stream_of(g, s) * g.n + row0) * g.K;
    }
    __device__ __forceinline__ static int64_t source_rows(const Args &g, int, int64_t row0)
    {
        return g.n - row0;
    }
    template <bool AL> struct AStage {
        static constexpr int CH = M * BMS * kChunks;
        static constexpr int NA = (CH + kThreads - 1) / kThreads;
        v4i a[NA];
        __device__ __forceinline__ void load(const Args &g, int64_t row0, int64_t k0, int tid)
        {
#pragma unroll
            for (int i = 0; i < NA; ++i) {
                const int q = tid + i * kThreads;
                const int s = q / (BMS * kChunks), rem = q % (BMS * kChunks);
                const int64_t row = row0 + rem / kChunks;
                a[i] = (q < CH) ? load_chunk<AL>(g.c + ((int64_t)stream_of(g, s) * g.n + row) * g.K,
                                                 k0 + (rem % kChunks) * 16, g.K, row < g.n)
                                : v4i{0, 0, 0, 0};
            }
        }
        __device__ __forceinline__ void store(int8_t *lds_a, int tid) const
        {
#pragma unroll
            for (int i = 0; i < NA; ++i) {
                const int q = tid + i * kThreads;
                if (q < CH) {
                    const int s = q / (BMS * kChunks), rem = q % (BMS * kChunks);
                    *(v4i *)(lds_a + s * BMS * BK + lds_off(rem / kChunks, rem % kChunks)) = a[i];
                }
            }
        }
    };

    __device__ __forceinline__ static void epi(const Args &g, v16i (&acc)[P][RB][CB],
                                               int64_t row0, int64_t col0, int wm, int wn,
                                               int lane, int64_t f_beg, int64_t f_end)
    {
        const int64_t W = (g.N + 31) / 32;
        unsigned long long cnt = 0;
#pragma unroll
        for (int j = 0; j < CB; ++j) {
            const int64_t cblk = col0 + (wn * CB + j) * 32;
            const int64_t col = cblk + acc_col(lane);
            const int64_t word = cblk / 32;
#pragma unroll
            for (int r = 0; r < 16; ++r) {
                const int64_t row = row0 + wm * 32 + acc_row(r, lane);
                const bool valid = row < g.n && col < g.N;
                int64_t d[M], o[M];
#pragma unroll
                for (int s = 0; s < M; ++s) {
                    // Copy the two accumulators out of the AGPRs here, at their
                    // use: left to itself the compiler moves all of them out
                    // right after the main loop and spills.
                    int lo, hi;
                    asm volatile("v_accvgpr_read_b32 %0, %1" : "=v"(lo) : "a"(acc[s][0][j][r]));
                    asm volatile("v_accvgpr_read_b32 %0, %1" : "=v"(hi) : "a"(acc[M + s][0][j][r]));
                    d[s] = (int64_t)((uint64_t)(int64_t)lo + ((uint64_t)(int64_t)hi << g.l));
                }
                if constexpr (INJ)
                for (int64_t f = f_beg; f < f_end; ++f) {
                    if (g.inj_pos[f] == row * g.N + col) {
                        const int st = (g.inj_stream[f] - g.r + M) % M; // its slot
                        const uint64_t msk = g.inj_mask[f];
#pragma unroll
                        for (int s = 0; s < M; ++s)
                            if (s == st)
                                d[s] = (int64_t)((uint64_t)d[s] ^ msk);
                    }
                }
                const bool flag = disentangle_rot<M>(d, g.l, o) && valid;
                if (valid) {
                    if (g.out64) {
#pragma unroll
                        for (int s = 0; s < M; ++s)
                            ((int64_t *)g.dhat)[((int64_t)stream_of(g, s) * g.n + row) * g.N + col] =
                                o[s];
                    } else {
#pragma unroll
                        for (int s = 0; s < M; ++s)
                            ((int32_t *)g.dhat)[((int64_t)stream_of(g, s) * g.n + row) * g.N + col] =
                                (int32_t)o[s];
                    }
                }
                const uint64_t mask = __ballot(flag);
                if (g.flags && word < W && row < g.n && (lane & 31) == 0)
                    g.flags[row * W + word] = (uint32_t)(lane ? (mask >> 32) : mask);
                cnt += (unsigned long long)__popcll(mask);
                // one output position at a time: keeps the 2M words of a
                // position, not of all positions, live in registers
                __builtin_amdgcn_sched_barrier(0);
            }
        }
        if (g.n_bad && lane == 0 && cnt)
            atomicAdd(g.n_bad, cnt);
    }

    __device__ __forceinline__ static void epilogue(const Args &g, v16i (&acc)[P][RB][CB],
                                                    int64_t row0, int64_t col0, int wm, int wn,
                                                    int lane)
    {
        // Injected faults of this tile: positions are sorted, so the tile's
        // rows form one contiguous range of the list.
        int64_t fb = 0, fe = 0;
        if (INJ && g.inj_count > 0) {
            const int64_t rows_end = row0 + BMS < g.n ? row0 + BMS : g.n;
            const int64_t lo_key = row0 * g.N, hi_key = rows_end * g.N;
            int64_t lo = 0, hi = g.inj_count;
            while (lo < hi) {
                const int64_t mid = (lo + hi) >> 1;
                if (g.inj_pos[mid] < lo_key) lo = mid + 1; else hi = mid;
            }
            fb = lo;
            hi = g.inj_count;
            while (lo < hi) {
                const int64_t mid = (lo + hi) >> 1;
                if (g.inj_pos[mid] < hi_key) lo = mid + 1; else hi = mid;
            }
            fe = lo;
        }
        epi(g, acc, row0, col0, wm, wn, lane, fb, fe);
    }
};

// GEMM head of a series: the entangled products of FusedV, then
//     delta[q] = scale[q] * delta[q] + (2^l + 1) * add[q]   (mod 2^64)
// on every stream, stored as rows[q][s] (slot s = stream (r + s) mod M): a
// lane holds every stream of its positions, so each store is M contiguous
// words and a half-wavefront writes 32 * M contiguous words.
template <int M>
struct SeriesV : FusedV<M> {
    using Base = FusedV<M>;
    using Base::BMS;
    using Base::CB;
    using Base::P;
    using Base::RB;
    struct Args : Base::Args {
        const int64_t *scale;
        const int64_t *add;
        int64_t *rows;
    };

    __device__ __forceinline__ static void epilogue(const Args &g, v16i (&acc)[P][RB][CB],
                                                    int64_t row0, int64_t col0, int wm, int wn,
                                                    int lane)
    {
#pragma unroll
        for (int j = 0; j < CB; ++j) {
            const int64_t col = col0 + (wn * CB + j) * 32 + acc_col(lane);
            // the scale and add words of the lane's 16 positions, all loaded
            // before the first is used (from position 0 where there is none)
            uint64_t sc[16], ad[16];
#pragma unroll
            for (int r = 0; r < 16; ++r) {
                const int64_t row = row0 + wm * 32 + acc_row(r, lane);
                const int64_t q = (row < g.n && col < g.N) ? row * g.N + col : 0;
                sc[r] = g.scale ? (uint64_t)g.scale[q] : 1u;
                ad[r] = g.add ? (uint64_t)g.add[q] : 0u;
            }
#pragma unroll
            for (int r = 0; r < 16; ++r) {
                const int64_t row = row0 + wm * 32 + acc_row(r, lane);
                uint64_t d[M];
#pragma unroll
                for (int s = 0; s < M; ++s) {
                    int lo, hi;
                    asm volatile("v_accvgpr_read_b32 %0, %1" : "=v"(lo) : "a"(acc[s][0][j][r]));
                    asm volatile("v_accvgpr_read_b32 %0, %1" : "=v"(hi) : "a"(acc[M + s][0][j][r]));
                    d[s] = (uint64_t)(int64_t)lo + ((uint64_t)(int64_t)hi << g.l);
                }
                if (row < g.n && col < g.N) {
                    const int64_t q = row * g.N + col;
                    const uint64_t a = (uint64_t)entangle_word((int64_t)ad[r], (int64_t)ad[r], g.l);
#pragma unroll
                    for (int s = 0; s < M; ++s)
                        g.rows[q * M + s] = (int64_t)(sc[r] * d[s] + a);
                }
                __builtin_amdgcn_sched_barrier(0);
            }
        }
    }
};

// ------------------------------------------------------------------- ABFT

template <int M>
struct AbftV {
    static constexpr int NSRC = M + 2, P = M + 2, BMS = 32, BN = 128, WM = 1, WN = 4;
    static constexpr int kOcc = (M <= 6) ? 2 : 1;
    static constexpr bool kDma = false;
    static constexpr int RB = 1, CB = 1;
    __host__ __device__ static constexpr int src(int p) { return p; }
    struct Args : ArgsBase {
        const int8_t *c;
        int32_t *d;
        uint32_t *flags;
        unsigned long long *n_bad;
        int64_t n;
    };
    template <bool AL> struct AStage {
        static constexpr int UNITS = BMS * kChunks;
        static_assert(UNITS <= kThreads, "one unit per thread");
        v4i a[M];
        __device__ __forceinline__ void load(const Args &g, int64_t row0, int64_t k0, int tid)
        {
            if (tid < UNITS) {
                const int64_t row = row0 + tid / kChunks;
                const int64_t k = k0 + (tid % kChunks) * 16;
#pragma unroll
                for (int s = 0; s < M; ++s)
                    a[s] = load_chunk<AL>(g.c + ((int64_t)s * g.n + row) * g.K, k, g.K, row < g.n);
            }
        }
        __device__ __forceinline__ void store(int8_t *lds_a, int tid) const
        {
            if (tid < UNITS) {
                const int row = tid / kChunks, ch = tid % kChunks;
                uint32_t lo[4] = {0, 0, 0, 0}, hi[4] = {0, 0, 0, 0};
#pragma unroll
                for (int e = 0; e < 16; ++e) {
                    int sum = 0;
#pragma unroll
                    for (int s = 0; s < M; ++s)
                        sum += (int)(int8_t)((uint32_t)a[s][e >> 2] >> (8 * (e & 3)));
                    const int d0 = (int)(int8_t)(sum & 0xFF);
                    const int d1 = (sum - d0) >> 8;
                    lo[e >> 2] |= (uint32_t)(uint8_t)d0 << (8 * (e & 3));
                    hi[e >> 2] |= (uint32_t)(uint8_t)d1 << (8 * (e & 3));
                }
#pragma unroll
                for (int s = 0; s < M; ++s)
                    *(v4i *)(lds_a + s * BMS * BK + lds_off(row, ch)) = a[s];
                *(v4i *)(lds_a + M * BMS * BK + lds_off(row, ch)) =
                    v4i{(int)lo[0], (int)lo[1], (int)lo[2], (int)lo[3]};
                *(v4i *)(lds_a + (M + 1) * BMS * BK + lds_off(row, ch)) =
                    v4i{(int)hi[0], (int)hi[1], (int)hi[2], (int)hi[3]};
            }
        }
    };
    __device__ __forceinline__ static void epilogue(const Args &g, v16i (&acc)[P][RB][CB],
                                                    int64_t row0, int64_t col0, int wm, int wn,
                                                    int lane)
    {
        const int64_t W = (g.N + 31) / 32;
        const int64_t col = col0 + wn * 32 + acc_col(lane);
        const int64_t word = (col0 + wn * 32) / 32;
        unsigned long long cnt = 0;
#pragma unroll
        for (int r = 0; r < 16; ++r) {
            const int64_t row = row0 + wm * 32 + acc_row(r, lane);
            const bool valid = row < g.n && col < g.N;
            int64_t sum = 0;
#pragma unroll
            for (int s = 0; s < M; ++s)
                sum += (int64_t)acc[s][0][0][r];
            const int64_t e = (int64_t)acc[M][0][0][r] + (int64_t)acc[M + 1][0][0][r] * 256;
            const bool flag = valid && sum != e;
            if (valid) {
#pragma unroll
                for (int s = 0; s < M; ++s)
                    g.d[((int64_t)s * g.n + row) * g.N + col] = acc[s][0][0][r];
            }
            const uint64_t mask = __ballot(flag);
            if (g.flags && word < W && row < g.n && (lane & 31) == 0)
                g.flags[row * W + word] = (uint32_t)(lane ? (mask >> 32) : mask);
            cnt += (unsigned long long)__popcll(mask);
        }
        if (g.n_bad && lane == 0 && cnt)
            atomicAdd(g.n_bad, cnt);
    }
};

// Checksum-stream ABFT through the DMA pipeline: the checksum stream
// r = sum_m c_m is built beforehand (k_abft_checksum) as two int8 digit
// planes, so that all M + 2 sources are plain int8 rows the DMA engine
// copies into LDS; one accumulator set per source.
template <int M>
struct AbftDmaV {
    static constexpr int NSRC = M + 2, P = M + 2, BMS = 32, BN = (M <= 4) ? 256 : 128, WM = 1,
                         WN = 4;
    static constexpr int kOcc = 1;
    static constexpr bool kDma = true;
    static constexpr int kBK = 128, kStages = 2;
    static constexpr int RB = 1, CB = BN / 128;
    __host__ __device__ static constexpr int src(int p) { return p; }
    struct Args : ArgsBase {
        const int8_t *c;
        const int8_t *rlo, *rhi; // checksum digit planes [n][K]
        int32_t *d;
        uint32_t *flags;
        unsigned long long *n_bad;
        int64_t n;
    };
    __device__ __forceinline__ static const int8_t *source_base(const Args &g, int s, int64_t row0)
    {
        if (s < M)
            return g.c + ((int64_t)s * g.n + row0) * g.K;
        return (s == M ? g.rlo : g.rhi) + row0 * g.K;
    }
    __device__ __forceinline__ static int64_t source_rows(const Args &g, int, int64_t row0)
    {
        return g.n - row0;
    }
    __device__ __forceinline__ static void epilogue(const Args &g, v16i (&acc)[P][RB][CB],
                                                    int64_t row0, int64_t col0, int wm, int wn,
                                                    int lane)
    {
        const int64_t W = (g.N + 31) / 32;
        unsigned long long cnt = 0;
#pragma unroll
        for (int j = 0; j < CB; ++j) {
            const int64_t cblk = col0 + (wn * CB + j) * 32;
            const int64_t col = cblk + acc_col(lane);
            const int64_t word = cblk / 32;
#pragma unroll
            for (int r = 0; r < 16; ++r) {
                const int64_t row = row0 + wm * 32 + acc_row(r, lane);
                const bool valid = row < g.n && col < g.N;
                int v[P];
#pragma unroll
                for (int s = 0; s < P; ++s)
                    asm volatile("v_accvgpr_read_b32 %0, %1" : "=v"(v[s]) : "a"(acc[s][0][j][r]));
                int64_t sum = 0;
#pragma unroll
                for (int s = 0; s < M; ++s)
                    sum += v[s];
                const int64_t e = (int64_t)v[M] + (int64_t)v[M + 1] * 256;
                const bool flag = valid && sum != e;
                if (valid) {
#pragma unroll
                    for (int s = 0; s < M; ++s)
                        g.d[((int64_t)s * g.n + row) * g.N + col] = v[s];
                }
                const uint64_t mask = __ballot(flag);
                if (g.flags && word < W && row < g.n && (lane & 31) == 0)
                    g.flags[row * W + word] = (uint32_t)(lane ? (mask >> 32) : mask);
                cnt += (unsigned long long)__popcll(mask);
                __builtin_amdgcn_sched_barrier(0);
            }
        }
        if (g.n_bad && lane == 0 && cnt)
            atomicAdd(g.n_bad, cnt);
    }
};

// The checksum stream of the ABFT baseline as two balanced int8 digit
// planes: r = sum_m c[m] = lo + 256 hi, 16 bytes per thread (count a
// multiple of 16, every row 16-byte aligned).
template <int M>
__global__ __launch_bounds__(kThreads) void k_abft_checksum(const int8_t *__restrict__ c,
                                                            int8_t *__restrict__ lo,
                                                            int8_t *__restrict__ hi,
                                                            int64_t count)
{
    const int64_t stride = (int64_t)gridDim.x * kThreads * 16;
    for (int64_t i = ((int64_t)blockIdx.x * kThreads + threadIdx.x) * 16; i < count; i += stride) {
        v4i x[M];
#pragma unroll
        for (int m = 0; m < M; ++m)
            x[m] = *(const v4i *)(c + (int64_t)m * count + i);
        uint32_t l[4] = {0, 0, 0, 0}, h[4] = {0, 0, 0, 0};
#pragma unroll
        for (int e = 0; e < 16; ++e) {
            int sum = 0;
#pragma unroll
            for (int m = 0; m < M; ++m)
                sum += (int)(int8_t)((uint32_t)x[m][e >> 2] >> (8 * (e & 3)));
            const int d0 = (int)(int8_t)(sum & 0xFF);
            const int d1 = (sum - d0) >> 8;
            l[e >> 2] |= (uint32_t)(uint8_t)d0 << (8 * (e & 3));
            h[e >> 2] |= (uint32_t)(uint8_t)d1 << (8 * (e & 3));
        }
        *(v4i *)(lo + i) = v4i{(int)l[0], (int)l[1], (int)l[2], (int)l[3]};
        *(v4i *)(hi + i) = v4i{(int)h[0], (int)h[1], (int)h[2], (int)h[3]};
    }
}

} // namespace
} // namespace ne
