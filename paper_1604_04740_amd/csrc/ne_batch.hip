// ne_batch.hip -- many independent entangled problems (uneven M, size and
// operation) in one persistent launch.
//
// Host side (setup, not graph-capturable): ne_batch_plan turns a problem
// list into work items -- one per GEMM output tile, one per 1024-position
// convolution block, two per permute/scale chunk (copy of the inputs into
// rows, then the gather) -- deals them to the XCDs (a GEMM's tiles in eight
// runs of neighbouring tiles, the other items in turn), balances each XCD's
// items over its workgroups longest-first by a cost estimate (each item to
// the least loaded workgroup), and writes the problem table, the per-
// workgroup item lists and room for the row copies into a caller-provided
// device buffer.  ne_batch_autotune times the candidate
// tile choices of every (operation, M, size-class) bucket on the device and
// returns the fastest per bucket.
//
// Device side: ne_batch_run makes up to three launches.  Phase 0 copies
// the permutations' inputs into rows and phase 2 runs their gathers, both
// in a kernel without LDS whose workgroups split each list (many memory
// accesses in flight per CU); phase 1, the persistent kernel (grid = one
// workgroup per CU), runs every GEMM tile and convolution block.  Each
// workgroup runs its own list.  Every loop is bounded by the list bounds in
// the table, so the grid always drains.  The launches are plain kernels (no
// memset nodes), so ne_batch_run can be captured in a HIP graph and
// replayed.
#include <algorithm>
#include <cstdlib>
#include <cstring>
#include <vector>

#include "ne_conv_impl.h"
#include "ne_gemm_impl.h"
#include "ne_perm_impl.h"

namespace ne {
namespace {

constexpr int kBatchThreads = 256;
constexpr int kGemmBK = NE_FUSED_BK;
constexpr int kGemmStages = NE_FUSED_STAGES;

struct DevProblem {
    int32_t op, M, l, r;
    int32_t out64, bn, tiles_m, tiles_n;
    int64_t n, K, N, chunk;
    const void *c;
    const void *g;
    const int32_t *perm;
    const int64_t *scale;
    const int64_t *add;
    void *dhat;
    uint32_t *flags;
    unsigned long long *n_bad;
    uint64_t *rows; // permutation: row copy of the inputs (in the table)
};

// kind 0: the item of its operation; kind 1: a chunk of a permutation's
// row copy (phase 0; its gathers run in phase 2).
struct DevItem {
    int32_t problem, a, b, kind;
};

// Three phases, one launch each: row copies, GEMM tiles and convolution
// blocks, permutation gathers (which read the row copies).  Each phase
// keeps one item list per workgroup of the persistent grid: list w of
// phase p is items[wg[p][w] .. wg[p][w + 1]), wg an int32 array
// [3][grid + 1] at wg_off.
constexpr int kXcds = 8;
struct DevHeader {
    int32_t grid, n_problems;
    int64_t problems_off, items_off, wg_off;
};

constexpr int64_t kHeaderBytes = 256;

// The item and problem records are the same in every lane; passing every
// field through readfirstlane states it, which keeps the buffer descriptors
// built from them in SGPRs (no per-load waterfall loops).
__device__ __forceinline__ int32_t uni(int32_t v) { return __builtin_amdgcn_readfirstlane(v); }
__device__ __forceinline__ int64_t uni(int64_t v)
{
    const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)v);
    const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)((uint64_t)v >> 32));
    return (int64_t)(((uint64_t)hi << 32) | lo);
}
template <typename T> __device__ __forceinline__ T *uni(T *p)
{
    return (T *)(uintptr_t)uni((int64_t)(uintptr_t)p);
}

__device__ __forceinline__ DevProblem uniform(const DevProblem &x)
{
    DevProblem u;
    u.op = uni(x.op);
    u.M = uni(x.M);
    u.l = uni(x.l);
    u.r = uni(x.r);
    u.out64 = uni(x.out64);
    u.bn = uni(x.bn);
    u.tiles_m = uni(x.tiles_m);
    u.tiles_n = uni(x.tiles_n);
    u.n = uni(x.n);
    u.K = uni(x.K);
    u.N = uni(x.N);
    u.chunk = uni(x.chunk);
    u.c = uni(x.c);
    u.g = uni(x.g);
    u.perm = uni(x.perm);
    u.scale = uni(x.scale);
    u.add = uni(x.add);
    u.dhat = uni(x.dhat);
    u.flags = uni(x.flags);
    u.n_bad = uni(x.n_bad);
    u.rows = uni(x.rows);
    return u;
}

template <int M, int BN>
__device__ __forceinline__ void run_gemm_tile(const DevProblem &P, int tm, int tn, int8_t *lds)
{
    using V = FusedV<M, BN>;
    typename V::Args a{};
    a.Bt = (const int8_t *)P.g;
    a.K = P.K;
    a.N = P.N;
    a.tiles_m = P.tiles_m;
    a.tiles_n = P.tiles_n;
    a.c = (const int8_t *)P.c;
    a.dhat = P.dhat;
    a.flags = P.flags;
    a.n_bad = P.n_bad;
    a.n = P.n;
    a.l = P.l;
    a.r = P.r;
    a.out64 = P.out64;
    gemm_tile_dma<V, kGemmBK, kGemmStages>(a, tm, tn, lds);
}

__device__ __forceinline__ void run_gemm(const DevProblem &P, int tm, int tn, int8_t *lds)
{
    if (P.bn == 256) {
        switch (P.M) {
        case 3: run_gemm_tile<3, 256>(P, tm, tn, lds); return;
        case 4: run_gemm_tile<4, 256>(P, tm, tn, lds); return;
        default: return;
        }
    }
    switch (P.M) {
    case 3: run_gemm_tile<3, 128>(P, tm, tn, lds); return;
    case 4: run_gemm_tile<4, 128>(P, tm, tn, lds); return;
    case 5: run_gemm_tile<5, 128>(P, tm, tn, lds); return;
    case 6: run_gemm_tile<6, 128>(P, tm, tn, lds); return;
    case 7: run_gemm_tile<7, 128>(P, tm, tn, lds); return;
    case 8: run_gemm_tile<8, 128>(P, tm, tn, lds); return;
    default: return;
    }
}

template <int M>
__device__ __forceinline__ void run_conv_m(const DevProblem &P, int block, int8_t *lds)
{
    ConvJob J{};
    J.x = P.c;
    J.x_dtype = NE_I8;
    J.digits = 1;
    J.g = (const int8_t *)P.g;
    J.out = P.dhat;
    J.out64 = P.out64;
    J.flags = P.flags;
    J.n_bad = P.n_bad;
    J.N = P.N;
    J.L = P.N;
    J.Nout = P.N;
    J.M = M;
    J.l = P.l;
    J.r = P.r;
    // above four streams the two products of every slot take two passes:
    // this kernel also holds the GEMM tiles, and 2M accumulator sets for
    // M > 4 would push it into spilling
    conv_block<M, true, (M > 4)>(J, block, lds);
}

__device__ __forceinline__ void run_conv(const DevProblem &P, int block, int8_t *lds)
{
    switch (P.M) {
    case 3: run_conv_m<3>(P, block, lds); return;
    case 4: run_conv_m<4>(P, block, lds); return;
    case 5: run_conv_m<5>(P, block, lds); return;
    case 6: run_conv_m<6>(P, block, lds); return;
    case 7: run_conv_m<7>(P, block, lds); return;
    case 8: run_conv_m<8>(P, block, lds); return;
    default: return;
    }
}

template <int M>
// Positions first + start + tid, stepping by stride, of the chunk.
__device__ __forceinline__ void run_perm_m(const DevProblem &P, int chunk, bool pack,
                                           int64_t start, int64_t stride)
{
    const int64_t first = (int64_t)chunk * P.chunk;
    const int64_t last = first + P.chunk < P.N ? first + P.chunk : P.N;
    if (pack)
        perm_pack_range<M, int8_t>((const int8_t *)P.c, P.rows, P.N, P.r, first, last, start,
                                   stride);
    else
        perm_fused_range<M, int8_t>((const int8_t *)P.c, P.rows, P.perm, P.scale, P.add, P.dhat,
                                    P.out64, P.flags, P.n_bad, P.N, P.l, P.r, first, last, start,
                                    stride);
}

template <int M>
__device__ __forceinline__ void run_perm_m(const DevProblem &P, int chunk, bool pack)
{
    run_perm_m<M>(P, chunk, pack, 0, kBatchThreads);
}

__device__ __forceinline__ void run_perm(const DevProblem &P, int chunk, bool pack,
                                         int64_t start = 0, int64_t stride = kBatchThreads)
{
    switch (P.M) {
    case 3: run_perm_m<3>(P, chunk, pack, start, stride); return;
    case 4: run_perm_m<4>(P, chunk, pack, start, stride); return;
    case 5: run_perm_m<5>(P, chunk, pack, start, stride); return;
    case 6: run_perm_m<6>(P, chunk, pack, start, stride); return;
    case 7: run_perm_m<7>(P, chunk, pack, start, stride); return;
    case 8: run_perm_m<8>(P, chunk, pack, start, stride); return;
    default: return;
    }
}

constexpr int kBatchLds = 3 * 49152; // largest GEMM ring (M = 4, BN = 256 / M = 8, BN = 128)
static_assert(dma_lds_bytes<FusedV<4, 256>, kGemmBK, kGemmStages>() <= kBatchLds, "LDS");
static_assert(dma_lds_bytes<FusedV<8, 128>, kGemmBK, kGemmStages>() <= kBatchLds, "LDS");
static_assert(cv_lds_bytes(kCvMaxSlots) <= kBatchLds, "LDS");
static_assert(sizeof(DevHeader) <= kHeaderBytes, "header");

// Workgroup w (on XCD w mod 8: workgroups are placed on the XCDs in turn)
// runs its own list, which the plan filled from that XCD's items: the tiles
// that share an XCD's L2 are neighbours in their problem, and no item is
// fetched through a global counter.
__global__ __launch_bounds__(kBatchThreads, 1) void k_batch(const uint8_t *table, int phase)
{
    __shared__ __attribute__((aligned(1024))) int8_t lds[kBatchLds];
    const auto *h = (const DevHeader *)table;
    const auto *problems = (const DevProblem *)(table + h->problems_off);
    const auto *items = (const DevItem *)(table + h->items_off);
    const auto *wg = (const int32_t *)(table + h->wg_off) + phase * (uni(h->grid) + 1);
    const int lo = uni(wg[blockIdx.x]), hi = uni(wg[blockIdx.x + 1]);
    for (int i = lo; i < hi; ++i) {
        const DevItem im0 = items[i];
        const DevItem im = {uni(im0.problem), uni(im0.a), uni(im0.b), uni(im0.kind)};
        const DevProblem P = uniform(problems[im.problem]);
        if (P.op == NE_OP_GEMM)
            run_gemm(P, im.a, im.b, lds);
        else if (P.op == NE_OP_CONV)
            run_conv(P, im.a, lds);
        else
            run_perm(P, im.a, im.kind == 1);
        __syncthreads(); // the next item reuses the LDS
    }
}

// Phases 0 and 2 hold only permutation row copies and gathers, which need
// many memory accesses in flight rather than LDS: kGatherSplit workgroups
// without LDS share each list, part q taking the blocks of 256 positions
// q, q + kGatherSplit, ... of every item (chunks are multiples of 64, so a
// wavefront's 64 positions stay one aligned run for its flag words).
constexpr int kGatherSplit = 8;
__global__ __launch_bounds__(kBatchThreads) void k_batch_gather(const uint8_t *table, int phase)
{
    const auto *h = (const DevHeader *)table;
    const auto *problems = (const DevProblem *)(table + h->problems_off);
    const auto *items = (const DevItem *)(table + h->items_off);
    const auto *wg = (const int32_t *)(table + h->wg_off) + phase * (uni(h->grid) + 1);
    const int list = blockIdx.x / kGatherSplit, part = blockIdx.x % kGatherSplit;
    const int lo = uni(wg[list]), hi = uni(wg[list + 1]);
    for (int i = lo; i < hi; ++i) {
        const DevItem im0 = items[i];
        const DevItem im = {uni(im0.problem), uni(im0.a), uni(im0.b), uni(im0.kind)};
        const DevProblem P = uniform(problems[im.problem]);
        run_perm(P, im.a, im.kind == 1, (int64_t)part * kBatchThreads,
                 (int64_t)kGatherSplit * kBatchThreads);
    }
}

// ------------------------------------------------------------------- host

int size_class(int64_t s)
{
    return s <= 256 ? 0 : (s <= 1024 ? 1 : 2);
}

int64_t problem_size(const ne_problem_t &p)
{
    if (p.op == NE_OP_GEMM)
        return std::max(p.n, std::max(p.K, p.N));
    return p.N;
}

} // namespace

struct BatchPlan {
    void *table;
    int64_t bytes;
    int n_items[3];
    int grid; // a multiple of 8: every XCD gets the same number of workgroups
};

} // namespace ne

using namespace ne;

namespace {

int params_for(int M, int r, ne_params_t *p)
{
    int rc = ne_params_default(M, 64, p);
    if (rc)
        return rc;
    p->r_check = r;
    return NE_OK;
}

int validate(const ne_problem_t &q, const ne_params_t &p)
{
    if (q.M < 3 || q.M > kMaxStreamsFused || q.r_check < 0 || q.r_check >= q.M)
        return NE_EINVAL;
    if (q.out_dtype != NE_I32 && q.out_dtype != NE_I64)
        return NE_EINVAL;
    if (!q.c || !q.d_hat)
        return NE_EINVAL;
    int64_t D = 0;
    ne_range_bound(&p, &D);
    if (q.op == NE_OP_GEMM) {
        if (q.n <= 0 || q.N <= 0 || q.K <= 0 || q.K > kMaxK || !q.g)
            return NE_EINVAL;
        if (q.K % 16 || ((uintptr_t)q.c & 15) || ((uintptr_t)q.g & 15))
            return NE_EALIGN;
        if (q.K * 128 * 128 > D)
            return NE_ERANGE;
    } else if (q.op == NE_OP_CONV) {
        if (q.N <= 0 || q.N > kMaxK || !q.g)
            return NE_EINVAL;
        if (q.N * 128 * 128 > D)
            return NE_ERANGE;
    } else if (q.op == NE_OP_PERM) {
        if (q.N <= 0 || q.N > 0x7fffffff || !q.perm)
            return NE_EINVAL;
    } else {
        return NE_EINVAL;
    }
    if ((uintptr_t)q.d_hat % q.out_dtype || (uintptr_t)q.flags % 4 || (uintptr_t)q.n_bad % 8)
        return NE_EALIGN;
    return NE_OK;
}

// Cost estimate (seconds on one CU, from the standalone kernels' measured
// rates) used to balance the workgroups' lists.
double item_cost(const ne_problem_t &q, int bn, int64_t chunk)
{
    if (q.op == NE_OP_GEMM) // matrix-core work at ~7.8 TOP/s per CU, plus the epilogue
        return 2.0 * 2.0 * q.M * 32.0 * bn * q.K / 7.8e12 + 1.0e-6;
    if (q.op == NE_OP_CONV) { // ~2.6 us per staged 256-tap step; M > 4 takes two passes
        const double steps = (double)((q.N + kCvStep - 1) / kCvStep);
        return (q.M > 4 ? 2.0 : 1.0) * (steps * 2.6e-6 + 4.0e-6);
    }
    return (double)chunk * q.M * (1.0 + q.out_dtype) / 2.0e10;
}

struct Built {
    std::vector<DevProblem> probs;
    std::vector<DevItem> items; // by phase, then by workgroup
    std::vector<int32_t> wg;    // [3][grid + 1] list boundaries
    int grid = 0;
    int n_phase[3] = {};
    std::vector<int64_t> rows_off; // per problem, offset of its row copy (or -1)
    int64_t rows_bytes = 0;
};

int build(const ne_problem_t *problems, int count, const ne_batch_tuning_t *tuning, int grid,
          Built &out)
{
    struct Tmp {
        DevItem it;
        double cost;
        int xcd;
    };
    std::vector<Tmp> tmp[3]; // row copies, GEMM tiles and conv blocks, gathers
    int rr = 0;              // XCD of the next item without locality
    out.probs.resize(count);
    out.rows_off.assign(count, -1);
    out.rows_bytes = 0;
    for (int i = 0; i < count; ++i) {
        const ne_problem_t &q = problems[i];
        ne_params_t p;
        if (params_for(q.M, q.r_check, &p))
            return NE_EINVAL;
        int rc = validate(q, p);
        if (rc)
            return rc;
        const int cls = size_class(problem_size(q));
        DevProblem &d = out.probs[i];
        memset(&d, 0, sizeof d);
        d.op = q.op;
        d.M = q.M;
        d.l = p.l;
        d.r = q.r_check;
        d.out64 = q.out_dtype == NE_I64;
        d.n = q.n;
        d.K = q.K;
        d.N = q.N;
        d.c = q.c;
        d.g = q.g;
        d.perm = q.perm;
        d.scale = q.scale;
        d.add = q.add;
        d.dhat = q.d_hat;
        d.flags = q.flags;
        d.n_bad = q.n_bad;
        if (q.op == NE_OP_GEMM) {
            int bn = tuning ? tuning->gemm_bn[q.M - 3][cls] : (q.M <= 4 && cls == 2 ? 256 : 128);
            if (bn != 256 || q.M > 4)
                bn = 128;
            d.bn = bn;
            d.tiles_m = (int)((q.n + 31) / 32);
            d.tiles_n = (int)((q.N + bn - 1) / bn);
            const double c1 = item_cost(q, bn, 0);
            // groups of 8 row tiles by every column tile (row tile fastest),
            // cut into one contiguous run per XCD: each L2 holds a compact
            // block of the problem's rows and columns
            const int64_t ntiles = (int64_t)d.tiles_m * d.tiles_n;
            int64_t j = 0;
            for (int g0 = 0; g0 < d.tiles_m; g0 += 8) {
                const int gm = std::min(8, d.tiles_m - g0);
                for (int tn = 0; tn < d.tiles_n; ++tn)
                    for (int tm = g0; tm < g0 + gm; ++tm, ++j)
                        tmp[1].push_back({{i, tm, tn, 0}, c1, (int)(j * kXcds / ntiles)});
            }
        } else if (q.op == NE_OP_CONV) {
            const int blocks = (int)((q.N + kCvBlock - 1) / kCvBlock);
            const double c1 = item_cost(q, 0, 0);
            for (int b = 0; b < blocks; ++b)
                tmp[1].push_back({{i, b, 0, 0}, c1, rr++ % kXcds});
        } else {
            int64_t chunk = tuning ? tuning->perm_chunk[q.M - 3][cls] : 16384;
            if (chunk < 64)
                chunk = 64;
            chunk = (chunk + 63) / 64 * 64;
            d.chunk = chunk;
            const int chunks = (int)((q.N + chunk - 1) / chunk);
            const double c1 = item_cost(q, 0, chunk);
            out.rows_off[i] = out.rows_bytes;
            out.rows_bytes += (permute_rows_bytes(q.N, q.M, NE_I8) + 255) / 256 * 256;
            for (int b = 0; b < chunks; ++b) {
                tmp[0].push_back({{i, b, 0, 1}, c1 / 4, rr % kXcds}); // row copy: streaming
                tmp[2].push_back({{i, b, 0, 0}, c1, rr++ % kXcds});
            }
        }
    }
    // Each XCD's items, longest first (stable: a problem's run keeps its
    // order), go one by one to the least loaded of that XCD's workgroups
    // (w = x, x + 8, ...); each workgroup runs its items longest first.
    auto by_xcd_cost = [](const Tmp &a, const Tmp &b) {
        return a.xcd != b.xcd ? a.xcd < b.xcd : a.cost > b.cost;
    };
    const int per = grid / kXcds;
    out.grid = grid;
    out.items.clear();
    out.wg.assign(3 * (grid + 1), 0);
    for (int ph = 0; ph < 3; ++ph) {
        std::stable_sort(tmp[ph].begin(), tmp[ph].end(), by_xcd_cost);
        out.n_phase[ph] = (int)tmp[ph].size();
        std::vector<std::vector<DevItem>> lists(grid);
        size_t i = 0;
        for (int x = 0; x < kXcds; ++x) {
            std::vector<double> load(per, 0.0);
            for (; i < tmp[ph].size() && tmp[ph][i].xcd == x; ++i) {
                const int k = (int)(std::min_element(load.begin(), load.end()) - load.begin());
                load[k] += tmp[ph][i].cost;
                lists[x + kXcds * k].push_back(tmp[ph][i].it);
            }
        }
        int32_t *wg = out.wg.data() + ph * (grid + 1);
        for (int w = 0; w < grid; ++w) {
            wg[w] = (int32_t)out.items.size();
            out.items.insert(out.items.end(), lists[w].begin(), lists[w].end());
        }
        wg[grid] = (int32_t)out.items.size();
    }
    return NE_OK;
}

// Table layout: header | problems | items | (256-aligned) row copies.
int64_t table_head_bytes(const Built &b)
{
    const int64_t h = kHeaderBytes + (int64_t)b.probs.size() * sizeof(DevProblem) +
                      (int64_t)b.items.size() * sizeof(DevItem) +
                      (int64_t)b.wg.size() * sizeof(int32_t);
    return (h + 255) / 256 * 256;
}

int64_t table_bytes(const Built &b)
{
    return table_head_bytes(b) + b.rows_bytes;
}

int upload(Built &b, void *table_dev)
{
    const int64_t head = table_head_bytes(b);
    std::vector<uint8_t> host(head, 0);
    DevHeader h{};
    h.grid = b.grid;
    h.n_problems = (int32_t)b.probs.size();
    h.problems_off = kHeaderBytes;
    h.items_off = kHeaderBytes + (int64_t)b.probs.size() * sizeof(DevProblem);
    h.wg_off = h.items_off + (int64_t)b.items.size() * sizeof(DevItem);
    for (size_t i = 0; i < b.probs.size(); ++i)
        b.probs[i].rows = b.rows_off[i] < 0 ? nullptr
                                            : (uint64_t *)((uint8_t *)table_dev + head +
                                                           b.rows_off[i]);
    memcpy(host.data(), &h, sizeof h);
    if (!b.probs.empty())
        memcpy(host.data() + h.problems_off, b.probs.data(), b.probs.size() * sizeof(DevProblem));
    if (!b.items.empty())
        memcpy(host.data() + h.items_off, b.items.data(), b.items.size() * sizeof(DevItem));
    memcpy(host.data() + h.wg_off, b.wg.data(), b.wg.size() * sizeof(int32_t));
    return hipMemcpy(table_dev, host.data(), host.size(), hipMemcpyHostToDevice) == hipSuccess
               ? NE_OK
               : NE_ELAUNCH;
}

int cu_count()
{
    int dev = 0, cus = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
        cus <= 0)
        return 256;
    return cus;
}

int launch_plan(const BatchPlan &bp, hipStream_t s)
{
    for (int ph = 0; ph < 3; ++ph) {
        if (bp.n_items[ph] == 0)
            continue;
        if (ph == 1)
            k_batch<<<bp.grid, kBatchThreads, 0, s>>>((const uint8_t *)bp.table, ph);
        else
            k_batch_gather<<<bp.grid * kGatherSplit, kBatchThreads, 0, s>>>(
                (const uint8_t *)bp.table, ph);
        if (launch_status())
            return NE_ELAUNCH;
    }
    return NE_OK;
}

} // namespace

extern "C" {

int ne_batch_plan(const ne_problem_t *problems, int32_t count, const ne_batch_tuning_t *tuning,
                  void *table_dev, int64_t table_bytes_avail, int64_t *table_needed,
                  ne_batch_t **plan)
{
    if (count < 0 || (count > 0 && !problems) || !table_needed)
        return NE_EINVAL;
    Built b;
    const int grid = std::max(kXcds, cu_count() / kXcds * kXcds);
    int rc = build(problems, count, tuning, grid, b);
    if (rc)
        return rc;
    *table_needed = table_bytes(b);
    if (!table_dev)
        return NE_OK; // size query
    if (!plan || table_bytes_avail < *table_needed || ((uintptr_t)table_dev & 255))
        return table_bytes_avail < *table_needed ? NE_EINVAL : NE_EALIGN;
    rc = upload(b, table_dev);
    if (rc)
        return rc;
    auto *bp = (BatchPlan *)malloc(sizeof(BatchPlan));
    if (!bp)
        return NE_EINVAL;
    bp->table = table_dev;
    bp->bytes = *table_needed;
    bp->n_items[0] = b.n_phase[0];
    bp->n_items[1] = b.n_phase[1];
    bp->n_items[2] = b.n_phase[2];
    bp->grid = grid;
    *plan = (ne_batch_t *)bp;
    return NE_OK;
}

int ne_batch_run(const ne_batch_t *plan, ne_stream_t stream)
{
    if (!plan)
        return NE_EINVAL;
    return launch_plan(*(const BatchPlan *)plan, (hipStream_t)stream);
}

int ne_batch_items(const ne_batch_t *plan)
{
    if (!plan)
        return -1;
    const auto *bp = (const BatchPlan *)plan;
    return bp->n_items[0] + bp->n_items[1] + bp->n_items[2];
}

void ne_batch_free(ne_batch_t *plan) { free(plan); }

int ne_batch_autotune(const ne_problem_t *problems, int32_t count, void *table_dev,
                      int64_t table_bytes_avail, int32_t reps, ne_batch_tuning_t *out,
                      ne_stream_t stream)
{
    if (!out || count < 0 || (count > 0 && !problems) || !table_dev || reps < 1)
        return NE_EINVAL;
    hipStream_t s = (hipStream_t)stream;
    // defaults
    for (int m = 0; m < 6; ++m)
        for (int c = 0; c < 3; ++c) {
            out->gemm_bn[m][c] = (m <= 1 && c == 2) ? 256 : 128;
            out->perm_chunk[m][c] = 16384;
        }
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess)
        return NE_ELAUNCH;
    int rc = NE_OK;
    for (int op = NE_OP_GEMM; op <= NE_OP_PERM && rc == NE_OK; ++op) {
        if (op == NE_OP_CONV)
            continue; // one block shape only
        for (int m = 3; m <= kMaxStreamsFused && rc == NE_OK; ++m)
            for (int cls = 0; cls < 3 && rc == NE_OK; ++cls) {
                std::vector<ne_problem_t> sub;
                for (int i = 0; i < count; ++i)
                    if (problems[i].op == op && problems[i].M == m &&
                        size_class(problem_size(problems[i])) == cls)
                        sub.push_back(problems[i]);
                if (sub.empty())
                    continue;
                std::vector<int64_t> cands;
                if (op == NE_OP_GEMM) {
                    cands.push_back(128);
                    if (m <= 4)
                        cands.push_back(256);
                } else {
                    cands = {4096, 16384, 65536};
                }
                double best = 1e30;
                for (int64_t cand : cands) {
                    ne_batch_tuning_t t = *out;
                    if (op == NE_OP_GEMM)
                        t.gemm_bn[m - 3][cls] = (int32_t)cand;
                    else
                        t.perm_chunk[m - 3][cls] = cand;
                    int64_t need = 0;
                    ne_batch_t *bp = nullptr;
                    rc = ne_batch_plan(sub.data(), (int)sub.size(), &t, table_dev,
                                       table_bytes_avail, &need, &bp);
                    if (rc)
                        break;
                    rc = ne_batch_run(bp, s); // warm-up
                    (void)hipEventRecord(e0, s);
                    for (int r = 0; r < reps && rc == NE_OK; ++r)
                        rc = ne_batch_run(bp, s);
                    (void)hipEventRecord(e1, s);
                    (void)hipEventSynchronize(e1);
                    float ms = 0.f;
                    (void)hipEventElapsedTime(&ms, e0, e1);
                    ne_batch_free(bp);
                    if (rc == NE_OK && ms < best) {
                        best = ms;
                        if (op == NE_OP_GEMM)
                            out->gemm_bn[m - 3][cls] = (int32_t)cand;
                        else
                            out->perm_chunk[m - 3][cls] = cand;
                    }
                }
            }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    return rc;
}

} // extern "C"
