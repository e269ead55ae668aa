// ne_api.hip -- the C ABI declared in include/ne.h: argument validation,
// parameter rules, and dispatch to the kernels.  No allocation, no global
// state; every launch goes to the caller's stream.
#include <stdint.h>

#include <initializer_list>
#include <utility>

#include "ne_arith.h"
#include "ne_internal.h"
#include "ne_rc.h"

using namespace ne;

namespace {

constexpr int kVersion = 100; // 0.1.0

bool overlap(const void *a, int64_t abytes, const void *b, int64_t bbytes)
{
    if (!a || !b || abytes <= 0 || bbytes <= 0)
        return false;
    const uintptr_t a0 = (uintptr_t)a, b0 = (uintptr_t)b;
    return a0 < b0 + (uintptr_t)bbytes && b0 < a0 + (uintptr_t)abytes;
}

// Parameters admissible for the method (section III-C) and built for the GPU:
// w = 64, or w = 32 where the entry point has 32-bit word kernels (w32).
int check_params(const ne_params_t *p, int max_m, bool w32 = false)
{
    if (!p)
        return NE_EINVAL;
    if (p->M < 3 || p->w < 4 || p->w > 64 || p->l < 2 || p->k < 0 || p->k > p->l ||
        (int64_t)(p->M - 1) * p->l + p->k > p->w || p->r_check < 0 || p->r_check >= p->M)
        return NE_EINVAL;
    if (!(p->w == 64 || (w32 && p->w == 32)) || p->M > max_m)
        return NE_EUNSUP;
    return NE_OK;
}

hipStream_t hs(ne_stream_t s) { return (hipStream_t)s; }

// Linear convolution sizes: N >= 1 samples, 1 <= L <= kMaxK taps (exact
// int32 digit sums), N + L - 1 <= 2^30 outputs per stream.
bool linconv_sizes_ok(int64_t N, int64_t L)
{
    return N >= 1 && L >= 1 && L <= kMaxK && N <= ((int64_t)1 << 30) - L + 1;
}

// Row/column checksum ABFT sizes: 1 <= M <= 4096 subblocks of n x K by
// K x N, K <= kMaxK, n and N up to 2^20 (exact 64-bit sums, grid limits).
constexpr int64_t kRcMaxM = 4096, kRcMaxRows = (int64_t)1 << 20;

bool rc_sizes_ok(int64_t M, int64_t n, int64_t K, int64_t N)
{
    return M >= 1 && M <= kRcMaxM && n >= 1 && n <= kRcMaxRows && K >= 1 && K <= kMaxK &&
           N >= 1 && N <= kRcMaxRows;
}

int rc_entry(const int8_t *c, const int8_t *Gt, int32_t *d, uint32_t *row_flags,
             uint32_t *col_flags, unsigned long long *n_bad, int32_t M, int64_t n, int64_t K,
             int64_t N, void *ws, int64_t ws_bytes, bool gemm, hipStream_t s)
{
    if (!rc_sizes_ok(M, n, K, N) || !c || !Gt || !d || !ws)
        return NE_EINVAL;
    const int64_t need = ne::rc_workspace_bytes(M, K, N);
    if (ws_bytes < need)
        return NE_EINVAL;
    const int64_t cb = M * n * K, gb = N * K, db = M * n * N * 4;
    const int64_t rfb = M * ((n + 31) / 32) * 4, cfb = M * ((N + 31) / 32) * 4;
    const std::pair<const void *, int64_t> bufs[] = {{c, cb},         {Gt, gb},        {d, db},
                                                     {row_flags, rfb}, {col_flags, cfb}, {n_bad, 8},
                                                     {ws, need}};
    // every written buffer (d only when the GEMM runs) apart from the rest
    for (int i = gemm ? 2 : 3; i < 7; ++i)
        for (int j = 0; j < 7; ++j)
            if (i != j && overlap(bufs[i].first, bufs[i].second, bufs[j].first, bufs[j].second))
                return NE_EALIAS;
    if ((uintptr_t)d % 4 || (uintptr_t)row_flags % 4 || (uintptr_t)col_flags % 4 ||
        (uintptr_t)n_bad % 8 || (uintptr_t)ws % 16)
        return NE_EALIGN;
    return ne::launch_abft_rc(c, Gt, d, row_flags, col_flags, n_bad, M, n, K, N, ws, gemm, s);
}

// A linear-convolution workspace: NULL, or at least need bytes, 16-byte
// aligned and overlapping none of the buffers.
int linconv_ws_ok(const void *ws, int64_t bytes, int64_t need,
                  std::initializer_list<std::pair<const void *, int64_t>> bufs)
{
    if (!ws)
        return NE_OK;
    if (need <= 0 || bytes < need)
        return NE_EINVAL;
    for (const auto &b : bufs)
        if (overlap(ws, need, b.first, b.second))
            return NE_EALIAS;
    if ((uintptr_t)ws % 16)
        return NE_EALIGN;
    return NE_OK;
}

} // namespace

extern "C" {

const char *ne_strerror(int code)
{
    switch (code) {
    case NE_OK: return "success";
    case NE_EINVAL: return "invalid argument";
    case NE_ERANGE: return "output range exceeds the entangled dynamic range";
    case NE_EALIAS: return "buffers overlap";
    case NE_EALIGN: return "misaligned pointer or pitch";
    case NE_EUNSUP: return "not supported on this GPU build";
    case NE_ELAUNCH: return "kernel launch failed";
    default: return "unknown error";
    }
}

int ne_version(void) { return kVersion; }

int ne_params_default(int32_t M, int32_t w, ne_params_t *out)
{
    if (!out || M < 3 || w < 4 || w > 64)
        return NE_EINVAL;
    // Scan l; for each l the best overlap is k = min(l, w - (M-1) l).
    int best_l = -1, best_k = -1, best_width = -1;
    bool best_fills = false;
    for (int l = 1; (M - 1) * l <= w; ++l) {
        const int room = w - (M - 1) * l;
        const int k = room < l ? room : l;
        const int width = (M - 2) * l + k;
        const bool fills = (k == room);
        if (width > best_width || (width == best_width && fills && !best_fills) ||
            (width == best_width && fills == best_fills && l > best_l)) {
            best_width = width;
            best_l = l;
            best_k = k;
            best_fills = fills;
        }
    }
    if (best_l < 0)
        return NE_EINVAL;
    out->M = M;
    out->w = w;
    out->l = best_l;
    out->k = best_k;
    out->r_check = 0;
    return NE_OK;
}

int ne_range_bound(const ne_params_t *p, int64_t *D)
{
    if (!p || !D || p->M < 3 || p->l < 2 || p->k < 0 || p->k > p->l ||
        (int64_t)(p->M - 1) * p->l + p->k > p->w || p->w > 64)
        return NE_EINVAL;
    const int e = (p->M - 3) * p->l + p->k; // <= w - 2l <= 60
    *D = ((int64_t)1 << e) * (((int64_t)1 << (p->l - 1)) - 1);
    return NE_OK;
}

int ne_entangle(const void *c, int32_t c_dtype, void *eps, int64_t N, const ne_params_t *p,
                ne_stream_t stream)
{
    int rc = check_params(p, kMaxStreamsElementwise, true);
    if (rc)
        return rc;
    if (N < 0 || (c_dtype != NE_I8 && c_dtype != NE_I32 && c_dtype != NE_I64))
        return NE_EINVAL;
    if (N == 0)
        return NE_OK;
    if (!c || !eps)
        return NE_EINVAL;
    const int wb = p->w / 8; // bytes per word
    const int64_t cb = N * p->M * c_dtype, eb = N * p->M * wb;
    const bool same = (const void *)eps == c;
    if (same && c_dtype != wb)
        return NE_EALIAS;
    if (!same && overlap(c, cb, eps, eb))
        return NE_EALIAS;
    if (((uintptr_t)c % c_dtype) || ((uintptr_t)eps % wb))
        return NE_EALIGN;
    return launch_entangle(c, c_dtype, eps, N, p->M, p->l, p->w, hs(stream));
}

int ne_lsb_gemm(const int64_t *eps, int32_t eps_bits, const int8_t *Gt, int64_t *delta,
                int64_t n, int64_t K, int64_t N, const ne_params_t *p, ne_stream_t stream)
{
    int rc = check_params(p, kMaxStreamsElementwise);
    if (rc)
        return rc;
    if (n < 0 || K < 0 || N < 0 || K > kMaxK || eps_bits < 1 || eps_bits > 64)
        return NE_EINVAL;
    if (n == 0 || N == 0)
        return NE_OK;
    if (!delta || ((!eps || !Gt) && K > 0))
        return NE_EINVAL;
    const int64_t R = n * p->M;
    if (overlap(eps, R * K * 8, delta, R * N * 8) || overlap(Gt, N * K, delta, R * N * 8))
        return NE_EALIAS;
    if ((uintptr_t)eps % 8 || (uintptr_t)delta % 8)
        return NE_EALIGN;
    return launch_gemm_eps(eps, ne::digits_for_bits(eps_bits), Gt, delta, R, K, N,
                           hs(stream));
}

// Validates an optional convolution workspace (NULL: none).
static int check_conv_ws(const void *ws, int64_t ws_bytes, int64_t need, const void *out,
                         int64_t out_bytes)
{
    if (!ws)
        return NE_OK;
    if (ws_bytes < need)
        return NE_EINVAL;
    if (overlap(ws, need, out, out_bytes))
        return NE_EALIAS;
    if ((uintptr_t)ws % 8)
        return NE_EALIGN;
    return NE_OK;
}

int64_t ne_circconv_workspace(int64_t N, int32_t M, int32_t fused)
{
    if (N <= 0 || N > kMaxK || M < 3 || M > kMaxStreamsElementwise)
        return 0;
    return conv_split(N, M, fused != 0).bytes;
}

int ne_lsb_circconv(const int64_t *eps, int32_t eps_bits, const int8_t *g, int64_t *delta,
                    int64_t N, const ne_params_t *p, void *workspace, int64_t workspace_bytes,
                    ne_stream_t stream)
{
    int rc = check_params(p, kMaxStreamsElementwise);
    if (rc)
        return rc;
    if (N < 0 || N > kMaxK || eps_bits < 1 || eps_bits > 64)
        return NE_EINVAL;
    if (N == 0)
        return NE_OK;
    if (!eps || !g || !delta)
        return NE_EINVAL;
    const int64_t bytes = N * p->M * 8;
    if (overlap(eps, bytes, delta, bytes) || overlap(g, N, delta, bytes))
        return NE_EALIAS;
    if ((uintptr_t)eps % 8 || (uintptr_t)delta % 8)
        return NE_EALIGN;
    const int64_t need = conv_split(N, p->M, false).bytes;
    if ((rc = check_conv_ws(workspace, workspace_bytes, need, delta, bytes)) != NE_OK)
        return rc;
    if (workspace && (overlap(workspace, need, eps, bytes) || overlap(workspace, need, g, N)))
        return NE_EALIAS;
    return launch_circconv_eps(eps, ne::digits_for_bits(eps_bits), g, delta, N, p->M,
                               need ? workspace : nullptr, hs(stream));
}

int ne_lsb_permute_scale(const void *eps, const int32_t *perm, const void *scale, const void *add,
                         void *delta, int64_t N, const ne_params_t *p, ne_stream_t stream)
{
    int rc = check_params(p, kMaxStreamsElementwise, true);
    if (rc)
        return rc;
    if (N < 0 || N > 0x7fffffff)
        return NE_EINVAL;
    if (N == 0)
        return NE_OK;
    if (!eps || !perm || !delta)
        return NE_EINVAL;
    const int wb = p->w / 8;
    const int64_t bytes = N * p->M * wb;
    if (overlap(eps, bytes, delta, bytes) || overlap(perm, N * 4, delta, bytes) ||
        overlap(scale, N * wb, delta, bytes) || overlap(add, N * wb, delta, bytes))
        return NE_EALIAS;
    if ((uintptr_t)eps % wb || (uintptr_t)delta % wb || (uintptr_t)perm % 4 ||
        (uintptr_t)scale % wb || (uintptr_t)add % wb)
        return NE_EALIGN;
    return launch_permute_scale(eps, perm, scale, add, delta, N, p->M, p->l, p->w, hs(stream));
}

int ne_disentangle_check(const void *delta, void *d_hat, uint32_t *flags,
                         unsigned long long *n_bad, int64_t N, const ne_params_t *p,
                         ne_stream_t stream)
{
    int rc = check_params(p, kMaxStreamsElementwise, true);
    if (rc)
        return rc;
    if (N < 0)
        return NE_EINVAL;
    if (N == 0)
        return NE_OK;
    if (!delta || !d_hat)
        return NE_EINVAL;
    const int wb = p->w / 8;
    const int64_t bytes = N * p->M * wb;
    if (d_hat != delta && overlap(delta, bytes, d_hat, bytes))
        return NE_EALIAS;
    if (overlap(flags, ((N + 31) / 32) * 4, d_hat, bytes) ||
        overlap(flags, ((N + 31) / 32) * 4, delta, bytes))
        return NE_EALIAS;
    if ((uintptr_t)delta % wb || (uintptr_t)d_hat % wb || (uintptr_t)flags % 4 ||
        (uintptr_t)n_bad % 8)
        return NE_EALIGN;
    return launch_disentangle_check(delta, d_hat, flags, n_bad, N, p->M, p->l, p->r_check, p->w,
                                    hs(stream));
}

int ne_recover(const void *const *delta, int32_t lost, void *d_hat, void *delta_rebuilt, int64_t N,
               const ne_params_t *p, ne_stream_t stream)
{
    int rc = check_params(p, kMaxStreamsElementwise, true);
    if (rc)
        return rc;
    if (!delta || lost < 0 || lost >= p->M || N < 0)
        return NE_EINVAL;
    if (N == 0)
        return NE_OK;
    if (!d_hat)
        return NE_EINVAL;
    StreamPtrs sp{};
    const int wb = p->w / 8;
    const int64_t out_bytes = N * p->M * wb;
    for (int m = 0; m < p->M; ++m) {
        if (m == lost)
            continue;
        if (!delta[m])
            return NE_EINVAL;
        if (overlap(delta[m], N * wb, d_hat, out_bytes) ||
            overlap(delta[m], N * wb, delta_rebuilt, N * wb))
            return NE_EALIAS;
        if ((uintptr_t)delta[m] % wb)
            return NE_EALIGN;
        sp.p[m] = (const int64_t *)delta[m];
    }
    if (overlap(delta_rebuilt, N * wb, d_hat, out_bytes))
        return NE_EALIAS;
    if ((uintptr_t)d_hat % wb || (uintptr_t)delta_rebuilt % wb)
        return NE_EALIGN;
    return launch_recover(sp, lost, d_hat, delta_rebuilt, N, p->M, p->l, p->w, hs(stream));
}

int ne_gemm_fused(const int8_t *c, const int8_t *Gt, void *d_hat, int32_t out_dtype,
                  uint32_t *flags, unsigned long long *n_bad, int64_t n, int64_t K, int64_t N,
                  const ne_params_t *p, const ne_inject_t *inject, ne_stream_t stream)
{
    int rc = check_params(p, kMaxStreamsFused);
    if (rc)
        return rc;
    if (n < 0 || K < 0 || N < 0 || K > kMaxK || (out_dtype != NE_I32 && out_dtype != NE_I64))
        return NE_EINVAL;
    int64_t D = 0;
    ne_range_bound(p, &D);
    if (K * 128 * 128 > D)
        return NE_ERANGE;
    if (inject && inject->count > 0 &&
        (!inject->position || !inject->stream || !inject->xor_mask))
        return NE_EINVAL;
    if (n == 0 || N == 0)
        return NE_OK;
    if (!d_hat || ((!c || !Gt) && K > 0))
        return NE_EINVAL;
    const int64_t ob = p->M * n * N * out_dtype;
    const int64_t fb = n * ((N + 31) / 32) * 4;
    if (overlap(c, p->M * n * K, d_hat, ob) || overlap(Gt, N * K, d_hat, ob) ||
        overlap(flags, fb, d_hat, ob))
        return NE_EALIAS;
    if ((uintptr_t)d_hat % out_dtype || (uintptr_t)flags % 4 || (uintptr_t)n_bad % 8)
        return NE_EALIGN;
    return launch_gemm_fused(c, Gt, d_hat, out_dtype == NE_I64, flags, n_bad, n, K, N, p->M, p->l,
                             p->r_check, inject, hs(stream));
}

int ne_plain_gemm_i8(const int8_t *A, const int8_t *Bt, int32_t *C, int64_t R, int64_t K,
                     int64_t N, ne_stream_t stream)
{
    if (R < 0 || K < 0 || N < 0 || K > kMaxK)
        return NE_EINVAL;
    if (R == 0 || N == 0)
        return NE_OK;
    if (!C || ((!A || !Bt) && K > 0))
        return NE_EINVAL;
    if (overlap(A, R * K, C, R * N * 4) || overlap(Bt, N * K, C, R * N * 4))
        return NE_EALIAS;
    if ((uintptr_t)C % 4)
        return NE_EALIGN;
    return launch_gemm_plain(A, Bt, C, R, K, N, hs(stream));
}

int64_t ne_abft_rc_workspace(int32_t M, int64_t K, int64_t N)
{
    if (!rc_sizes_ok(M, 1, K, N))
        return 0;
    return ne::rc_workspace_bytes(M, K, N);
}

int ne_abft_rc_gemm_i8(const int8_t *c, const int8_t *Gt, int32_t *d, uint32_t *row_flags,
                       uint32_t *col_flags, unsigned long long *n_bad, int32_t M, int64_t n,
                       int64_t K, int64_t N, void *workspace, int64_t workspace_bytes,
                       ne_stream_t stream)
{
    return rc_entry(c, Gt, d, row_flags, col_flags, n_bad, M, n, K, N, workspace, workspace_bytes,
                    true, hs(stream));
}

int ne_abft_rc_check_i8(const int8_t *c, const int8_t *Gt, const int32_t *d, uint32_t *row_flags,
                        uint32_t *col_flags, unsigned long long *n_bad, int32_t M, int64_t n,
                        int64_t K, int64_t N, void *workspace, int64_t workspace_bytes,
                        ne_stream_t stream)
{
    return rc_entry(c, Gt, const_cast<int32_t *>(d), row_flags, col_flags, n_bad, M, n, K, N,
                    workspace, workspace_bytes, false, hs(stream));
}

int64_t ne_abft_workspace(int64_t n, int64_t K)
{
    if (n < 0 || K < 0 || (K > 0 && n > INT64_MAX / 2 / K))
        return 0;
    return 2 * n * K;
}

int ne_abft_gemm_i8(const int8_t *c, const int8_t *Gt, int32_t *d, uint32_t *flags,
                    unsigned long long *n_bad, int32_t M, int64_t n, int64_t K, int64_t N,
                    void *workspace, int64_t workspace_bytes, ne_stream_t stream)
{
    if (M < 1 || M > kMaxStreamsFused || n < 0 || K < 0 || N < 0 || K > kMaxK)
        return NE_EINVAL;
    if (n == 0 || N == 0)
        return NE_OK;
    if (!d || ((!c || !Gt) && K > 0))
        return NE_EINVAL;
    const int64_t ob = (int64_t)M * n * N * 4;
    if (overlap(c, (int64_t)M * n * K, d, ob) || overlap(Gt, N * K, d, ob) ||
        overlap(flags, n * ((N + 31) / 32) * 4, d, ob))
        return NE_EALIAS;
    if ((uintptr_t)d % 4 || (uintptr_t)flags % 4 || (uintptr_t)n_bad % 8)
        return NE_EALIGN;
    if (workspace) {
        const int64_t need = ne_abft_workspace(n, K);
        if (workspace_bytes < need)
            return NE_EINVAL;
        if (overlap(workspace, need, c, (int64_t)M * n * K) || overlap(workspace, need, Gt, N * K) ||
            overlap(workspace, need, d, ob) ||
            overlap(workspace, need, flags, n * ((N + 31) / 32) * 4))
            return NE_EALIAS;
        if ((uintptr_t)workspace % 16)
            return NE_EALIGN;
    }
    return launch_gemm_abft(c, Gt, d, flags, n_bad, n, K, N, M, workspace, hs(stream));
}

int ne_circconv_fused(const void *c, int32_t c_dtype, int32_t c_bits, const int8_t *g,
                      void *d_hat, int32_t out_dtype, uint32_t *flags,
                      unsigned long long *n_bad, int64_t N, const ne_params_t *p,
                      void *workspace, int64_t workspace_bytes, ne_stream_t stream)
{
    int rc = check_params(p, kMaxStreamsFused);
    if (rc)
        return rc;
    if (N < 0 || N > kMaxK || (c_dtype != NE_I8 && c_dtype != NE_I32 && c_dtype != NE_I64) ||
        (out_dtype != NE_I32 && out_dtype != NE_I64) || c_bits < 1 || c_bits > 8 * c_dtype)
        return NE_EINVAL;
    int64_t D = 0;
    ne_range_bound(p, &D);
    if (N == 0)
        return NE_OK;
    // a-priori bound N * 2^(c_bits-1) * 128 <= D, compared without overflow
    if (c_bits - 1 + 7 >= 63 || N > (D >> (c_bits - 1 + 7)))
        return NE_ERANGE;
    if (!c || !g || !d_hat)
        return NE_EINVAL;
    const int64_t ob = N * p->M * out_dtype;
    if (overlap(c, N * p->M * c_dtype, d_hat, ob) || overlap(g, N, d_hat, ob) ||
        overlap(flags, ((N + 31) / 32) * 4, d_hat, ob))
        return NE_EALIAS;
    if ((uintptr_t)c % c_dtype || (uintptr_t)d_hat % out_dtype || (uintptr_t)flags % 4 ||
        (uintptr_t)n_bad % 8)
        return NE_EALIGN;
    const int64_t need = conv_split(N, p->M, true).bytes;
    if ((rc = check_conv_ws(workspace, workspace_bytes, need, d_hat, ob)) != NE_OK)
        return rc;
    if (workspace && (overlap(workspace, need, c, N * p->M * c_dtype) ||
                      overlap(workspace, need, g, N) ||
                      overlap(workspace, need, flags, ((N + 31) / 32) * 4)))
        return NE_EALIAS;
    return launch_circconv_fused(c, c_dtype, c_bits, g, d_hat, out_dtype == NE_I64, flags, n_bad,
                                 N, p->M, p->l, p->r_check, need ? workspace : nullptr,
                                 hs(stream));
}

int64_t ne_permute_workspace(int64_t N, int32_t M, int32_t c_dtype)
{
    if (N <= 0 || N > 0x7fffffff || M < 3 || M > kMaxStreamsElementwise ||
        (c_dtype != NE_I8 && c_dtype != NE_I32 && c_dtype != NE_I64))
        return 0;
    return permute_rows_bytes(N, M, c_dtype);
}

int ne_permute_scale_fused(const void *c, int32_t c_dtype, const int32_t *perm, const void *scale,
                           const void *add, void *d_hat, int32_t out_dtype, uint32_t *flags,
                           unsigned long long *n_bad, int64_t N, const ne_params_t *p,
                           void *workspace, int64_t workspace_bytes, ne_stream_t stream)
{
    int rc = check_params(p, kMaxStreamsElementwise, true);
    if (rc)
        return rc;
    if (N < 0 || N > 0x7fffffff || (c_dtype != NE_I8 && c_dtype != NE_I32 && c_dtype != NE_I64) ||
        (out_dtype != NE_I32 && out_dtype != NE_I64) || (p->w == 32 && out_dtype != NE_I32))
        return NE_EINVAL;
    if (N == 0)
        return NE_OK;
    if (!c || !perm || !d_hat)
        return NE_EINVAL;
    const int wb = p->w / 8;
    const int64_t ob = N * p->M * out_dtype;
    if (overlap(c, N * p->M * c_dtype, d_hat, ob) || overlap(perm, N * 4, d_hat, ob) ||
        overlap(scale, N * wb, d_hat, ob) || overlap(add, N * wb, d_hat, ob) ||
        overlap(flags, ((N + 31) / 32) * 4, d_hat, ob))
        return NE_EALIAS;
    if ((uintptr_t)c % c_dtype || (uintptr_t)d_hat % out_dtype || (uintptr_t)perm % 4 ||
        (uintptr_t)scale % wb || (uintptr_t)add % wb || (uintptr_t)flags % 4 ||
        (uintptr_t)n_bad % 8)
        return NE_EALIGN;
    if (workspace) {
        const int64_t need = permute_rows_bytes(N, p->M, c_dtype);
        if (workspace_bytes < need)
            return NE_EINVAL;
        if (overlap(workspace, need, c, N * p->M * c_dtype) || overlap(workspace, need, d_hat, ob) ||
            overlap(workspace, need, perm, N * 4) || overlap(workspace, need, scale, N * wb) ||
            overlap(workspace, need, add, N * wb) ||
            overlap(workspace, need, flags, ((N + 31) / 32) * 4))
            return NE_EALIAS;
        if ((uintptr_t)workspace % 8)
            return NE_EALIGN;
    }
    return launch_permute_scale_fused(c, c_dtype, perm, scale, add, d_hat, out_dtype == NE_I64,
                                      flags, n_bad, N, p->M, p->l, p->r_check, p->w, workspace,
                                      hs(stream));
}

int64_t ne_linconv_workspace(int64_t N, int64_t L, int32_t M, int32_t bits, int32_t fused)
{
    if (!linconv_sizes_ok(N, L) || M < 3 || M > (fused ? kMaxStreamsFused : kMaxStreamsElementwise) ||
        bits < 1 || bits > 64)
        return 0;
    return ne::linconv_workspace_bytes(N, L, M,
                                       fused && bits <= 8 ? 1 : ne::digits_for_bits(bits));
}

int ne_lsb_linconv(const int64_t *eps, int32_t eps_bits, const int8_t *g, int64_t L,
                   int64_t *delta, int64_t N, const ne_params_t *p, void *workspace,
                   int64_t workspace_bytes, ne_stream_t stream)
{
    int rc = check_params(p, kMaxStreamsElementwise);
    if (rc)
        return rc;
    if (!linconv_sizes_ok(N, L) || eps_bits < 1 || eps_bits > 64)
        return NE_EINVAL;
    if (!eps || !g || !delta)
        return NE_EINVAL;
    const int64_t ib = N * p->M * 8, ob = (N + L - 1) * p->M * 8;
    if (overlap(eps, ib, delta, ob) || overlap(g, L, delta, ob))
        return NE_EALIAS;
    if ((uintptr_t)eps % 8 || (uintptr_t)delta % 8)
        return NE_EALIGN;
    rc = linconv_ws_ok(workspace, workspace_bytes, ne_linconv_workspace(N, L, p->M, eps_bits, 0),
                       {{eps, ib}, {g, L}, {delta, ob}});
    if (rc)
        return rc;
    return launch_linconv_eps(eps, ne::digits_for_bits(eps_bits), g, L, delta, N, p->M, workspace,
                              hs(stream));
}

int ne_linconv_fused(const void *c, int32_t c_dtype, int32_t c_bits, const int8_t *g, int64_t L,
                     void *d_hat, int32_t out_dtype, uint32_t *flags, unsigned long long *n_bad,
                     int64_t N, const ne_params_t *p, void *workspace, int64_t workspace_bytes,
                     ne_stream_t stream)
{
    int rc = check_params(p, kMaxStreamsFused);
    if (rc)
        return rc;
    if (!linconv_sizes_ok(N, L) ||
        (c_dtype != NE_I8 && c_dtype != NE_I32 && c_dtype != NE_I64) ||
        (out_dtype != NE_I32 && out_dtype != NE_I64) || c_bits < 1 || c_bits > 8 * c_dtype)
        return NE_EINVAL;
    int64_t D = 0;
    ne_range_bound(p, &D);
    // a-priori bound L * 2^(c_bits-1) * 128 <= D, compared without overflow
    if (c_bits - 1 + 7 >= 63 || L > (D >> (c_bits - 1 + 7)))
        return NE_ERANGE;
    if (!c || !g || !d_hat)
        return NE_EINVAL;
    const int64_t No = N + L - 1;
    const int64_t ob = No * p->M * out_dtype;
    if (overlap(c, N * p->M * c_dtype, d_hat, ob) || overlap(g, L, d_hat, ob) ||
        overlap(flags, ((No + 31) / 32) * 4, d_hat, ob))
        return NE_EALIAS;
    if ((uintptr_t)c % c_dtype || (uintptr_t)d_hat % out_dtype || (uintptr_t)flags % 4 ||
        (uintptr_t)n_bad % 8)
        return NE_EALIGN;
    rc = linconv_ws_ok(workspace, workspace_bytes, ne_linconv_workspace(N, L, p->M, c_bits, 1),
                       {{c, N * p->M * c_dtype}, {g, L}, {d_hat, ob},
                        {flags, ((No + 31) / 32) * 4}, {n_bad, 8}});
    if (rc)
        return rc;
    return launch_linconv_fused(c, c_dtype, c_bits, g, L, d_hat, out_dtype == NE_I64, flags, n_bad,
                                N, p->M, p->l, p->r_check, workspace, hs(stream));
}

int ne_series_range(const ne_params_t *p, int64_t c_max, int32_t n_ops, const ne_series_op_t *ops,
                    int32_t *eps_bits, int64_t *out_max)
{
    int64_t D = 0;
    if (ne_range_bound(p, &D) != NE_OK || c_max < 0 || n_ops < 0 || (n_ops > 0 && !ops))
        return NE_EINVAL;
    for (int32_t i = 0; i < n_ops; ++i)
        if (ops[i].kind < NE_SERIES_GEMM || ops[i].kind > NE_SERIES_PERMUTE || ops[i].length < 0 ||
            ops[i].operand_max < 0)
            return NE_EINVAL;
    // Bounds are exact integers, saturated at 2^126 (far above any D).
    typedef unsigned __int128 u128;
    const u128 cap = (u128)1 << 126;
    auto mul = [](u128 a, u128 b) -> u128 {
        if (a == 0 || b == 0)
            return 0;
        return a > cap / b ? cap : a * b;
    };
    u128 B = (u128)c_max;
    for (int32_t i = 0; i < n_ops; ++i) {
        if (eps_bits) {
            // entangled words entering step i: |eps| <= (2^l + 1) B < 2^(bits-1)
            const u128 e = mul(B, ((u128)1 << p->l) + 1);
            int bits = 1;
            while (bits < 64 && ((u128)1 << (bits - 1)) <= e)
                ++bits;
            eps_bits[i] = bits;
        }
        const ne_series_op_t &o = ops[i];
        switch (o.kind) {
        case NE_SERIES_GEMM:
        case NE_SERIES_CONV: B = mul(mul(B, (u128)o.length), (u128)o.operand_max); break;
        case NE_SERIES_SCALE_ADD: {
            const u128 t = mul(B, (u128)o.length) + (u128)o.operand_max;
            B = t > cap ? cap : t;
            break;
        }
        default: break; // a permutation keeps the bound
        }
    }
    if (out_max)
        *out_max = B > (u128)INT64_MAX ? INT64_MAX : (int64_t)B;
    return B > (u128)D ? NE_ERANGE : NE_OK;
}

int64_t ne_series_workspace(int64_t n, int64_t N, int32_t M)
{
    if (n < 0 || N < 0 || M < 3 || M > kMaxStreamsFused || (N > 0 && n > INT64_MAX / 8 / M / N))
        return 0;
    return n * N * M * 8;
}

int ne_series_gemm_scale_permute(const int8_t *c, const int8_t *Gt, const int64_t *scale,
                                 const int64_t *add, const int32_t *perm, int64_t scale_max,
                                 int64_t add_max, void *d_hat, int32_t out_dtype, uint32_t *flags,
                                 unsigned long long *n_bad, int64_t n, int64_t K, int64_t N,
                                 const ne_params_t *p, void *workspace, int64_t workspace_bytes,
                                 ne_stream_t stream)
{
    int rc = check_params(p, kMaxStreamsFused);
    if (rc)
        return rc;
    if (n < 0 || K < 0 || N < 0 || K > kMaxK || (out_dtype != NE_I32 && out_dtype != NE_I64) ||
        (scale && scale_max < 0) || (add && add_max < 0))
        return NE_EINVAL;
    if (N > 0 && n > 0x7fffffff / N)
        return NE_EINVAL; // positions are int32 permutation indices
    const int64_t s_max = scale ? scale_max : 1, a_max = add ? add_max : 0;
    int64_t D = 0;
    ne_range_bound(p, &D);
    // a-priori bound K * 128 * 128 * s_max + a_max <= D, without overflow
    if (a_max > D || (K > 0 && s_max > (D - a_max) / (K * 128 * 128)))
        return NE_ERANGE;
    const int64_t Q = n * N;
    if (Q == 0)
        return NE_OK;
    if (((!c || !Gt) && K > 0) || !perm || !d_hat || !workspace)
        return NE_EINVAL;
    const int64_t need = ne_series_workspace(n, N, p->M);
    if (workspace_bytes < need)
        return NE_EINVAL;
    const int64_t ob = p->M * Q * out_dtype, fb = ((Q + 31) / 32) * 4;
    const int64_t cb = p->M * n * K, gb = N * K;
    if (overlap(c, cb, d_hat, ob) || overlap(Gt, gb, d_hat, ob) || overlap(perm, Q * 4, d_hat, ob) ||
        overlap(scale, Q * 8, d_hat, ob) || overlap(add, Q * 8, d_hat, ob) ||
        overlap(flags, fb, d_hat, ob) || overlap(workspace, need, c, cb) ||
        overlap(workspace, need, Gt, gb) || overlap(workspace, need, perm, Q * 4) ||
        overlap(workspace, need, scale, Q * 8) || overlap(workspace, need, add, Q * 8) ||
        overlap(workspace, need, d_hat, ob) || overlap(workspace, need, flags, fb))
        return NE_EALIAS;
    if ((uintptr_t)workspace % 16 || (uintptr_t)d_hat % out_dtype || (uintptr_t)perm % 4 ||
        (uintptr_t)scale % 8 || (uintptr_t)add % 8 || (uintptr_t)flags % 4 || (uintptr_t)n_bad % 8)
        return NE_EALIGN;
    rc = launch_series_gemm(c, Gt, scale, add, (int64_t *)workspace, n, K, N, p->M, p->l,
                            p->r_check, hs(stream));
    if (rc)
        return rc;
    return launch_permute_rows_check((const int64_t *)workspace, perm, d_hat, out_dtype == NE_I64,
                                     flags, n_bad, Q, p->M, p->l, p->r_check, hs(stream));
}

} // extern "C"
