// ne_gemm.hip -- int8 matrix-core GEMMs for gfx950.
//
// One kernel template, four variants:
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
#include "ne_arith.h"
#include "ne_internal.h"

namespace ne {
namespace {

typedef int v4i __attribute__((ext_vector_type(4)));
typedef int v16i __attribute__((ext_vector_type(16)));

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
    } else {
        uint32_t w[4] = {0, 0, 0, 0};
#pragma unroll
        for (int b = 0; b < 16; ++b)
            if (k + b < K)
                w[b >> 2] |= (uint32_t)(uint8_t)row_ptr[k + b] << (8 * (b & 3));
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

    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
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

// Common argument block.
struct ArgsBase {
    const int8_t *Bt;
    int64_t K, N;
    int tiles_m, tiles_n;
};

// ------------------------------------------------------------------ plain

struct PlainV {
    static constexpr int NSRC = 1, P = 1, BMS = 256, BN = 128, WM = 2, WN = 2, kOcc = 2;
    static constexpr int RB = BMS / (32 * WM), CB = BN / (32 * WN);
    __host__ __device__ static constexpr int src(int) { return 0; }
    struct Args : ArgsBase {
        const int8_t *A;
        int32_t *C;
        int64_t R;
    };
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

// Disentangle with a compile-time r: rotate into slot order, extract, rotate back.
template <int M, int R>
__device__ __forceinline__ bool extract_r(const int64_t (&d)[M], int l, int64_t (&o)[M])
{
    int64_t dr[M], orr[M];
#pragma unroll
    for (int j = 0; j < M; ++j)
        dr[j] = d[(R + j) % M];
    const bool f = disentangle_rot<M>(dr, l, orr);
#pragma unroll
    for (int j = 0; j < M; ++j)
        o[(R + j) % M] = orr[j];
    return f;
}

template <int M>
struct FusedV {
    static constexpr int NSRC = M, P = 2 * M, BMS = 32, BN = 128, WM = 1, WN = 4;
    static constexpr int kOcc = (M <= 4) ? 2 : 1;
    static constexpr int RB = 1, CB = 1;
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
                a[i] = (q < CH) ? load_chunk<AL>(g.c + ((int64_t)s * g.n + row) * g.K,
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

    template <int R>
    __device__ __forceinline__ static void epi(const Args &g, v16i (&acc)[P][RB][CB],
                                               int64_t row0, int64_t col0, int wm, int wn,
                                               int lane, int64_t f_beg, int64_t f_end)
    {
        const int64_t W = (g.N + 31) / 32;
        const int64_t col = col0 + wn * 32 + acc_col(lane);
        const int64_t word = (col0 + wn * 32) / 32;
        unsigned long long cnt = 0;
#pragma unroll
        for (int r = 0; r < 16; ++r) {
            const int64_t row = row0 + wm * 32 + acc_row(r, lane);
            const bool valid = row < g.n && col < g.N;
            int64_t d[M], o[M];
#pragma unroll
            for (int s = 0; s < M; ++s)
                d[s] = (int64_t)((uint64_t)(int64_t)acc[s][0][0][r] +
                                 ((uint64_t)(int64_t)acc[M + s][0][0][r] << g.l));
            for (int64_t f = f_beg; f < f_end; ++f) {
                if (g.inj_pos[f] == row * g.N + col) {
                    const int st = g.inj_stream[f];
                    const uint64_t msk = g.inj_mask[f];
#pragma unroll
                    for (int s = 0; s < M; ++s)
                        if (s == st)
                            d[s] = (int64_t)((uint64_t)d[s] ^ msk);
                }
            }
            const bool flag = extract_r<M, R>(d, g.l, o) && valid;
            if (valid) {
                if (g.out64) {
#pragma unroll
                    for (int s = 0; s < M; ++s)
                        ((int64_t *)g.dhat)[((int64_t)s * g.n + row) * g.N + col] = o[s];
                } else {
#pragma unroll
                    for (int s = 0; s < M; ++s)
                        ((int32_t *)g.dhat)[((int64_t)s * g.n + row) * g.N + col] = (int32_t)o[s];
                }
            }
            const uint64_t mask = __ballot(flag);
            if (g.flags && word < W && row < g.n && (lane & 31) == 0)
                g.flags[row * W + word] = (uint32_t)(lane ? (mask >> 32) : mask);
            cnt += (unsigned long long)__popcll(mask);
        }
        if (g.n_bad && lane == 0 && cnt)
            atomicAdd(g.n_bad, cnt);
    }

    template <int R>
    __device__ __forceinline__ static void epi_dispatch(int r, const Args &g,
                                                        v16i (&acc)[P][RB][CB], int64_t row0,
                                                        int64_t col0, int wm, int wn, int lane,
                                                        int64_t fb, int64_t fe)
    {
        if constexpr (R == M - 1) {
            epi<R>(g, acc, row0, col0, wm, wn, lane, fb, fe);
        } else {
            if (r == R)
                epi<R>(g, acc, row0, col0, wm, wn, lane, fb, fe);
            else
                epi_dispatch<R + 1>(r, g, acc, row0, col0, wm, wn, lane, fb, fe);
        }
    }

    __device__ __forceinline__ static void epilogue(const Args &g, v16i (&acc)[P][RB][CB],
                                                    int64_t row0, int64_t col0, int wm, int wn,
                                                    int lane)
    {
        // Injected faults of this tile: positions are sorted, so the tile's
        // rows form one contiguous range of the list.
        int64_t fb = 0, fe = 0;
        if (g.inj_count > 0) {
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
        epi_dispatch<0>(g.r, g, acc, row0, col0, wm, wn, lane, fb, fe);
    }
};

// ------------------------------------------------------------------- ABFT

template <int M>
struct AbftV {
    static constexpr int NSRC = M + 2, P = M + 2, BMS = 32, BN = 128, WM = 1, WN = 4;
    static constexpr int kOcc = (M <= 6) ? 2 : 1;
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

template <int M>
int launch_fused_m(const int8_t *c, const int8_t *Bt, void *dhat, int out64, uint32_t *flags,
                   unsigned long long *n_bad, int64_t n, int64_t K, int64_t N, int l, int r,
                   const ne_inject_t *inj, hipStream_t s)
{
    typename FusedV<M>::Args a{};
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
    if (inj && inj->count > 0) {
        a.inj_pos = inj->position;
        a.inj_stream = inj->stream;
        a.inj_mask = inj->xor_mask;
        a.inj_count = inj->count;
    }
    return launch<FusedV<M>>(a, n, (K % 16 == 0) && aligned16(c) && aligned16(Bt), s);
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

int launch_gemm_abft(const int8_t *c, const int8_t *Bt, int32_t *d, uint32_t *flags,
                     unsigned long long *n_bad, int64_t n, int64_t K, int64_t N, int M,
                     hipStream_t s)
{
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
