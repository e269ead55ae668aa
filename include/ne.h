/*
 * ne.h -- numerical entanglement on MI355X (gfx950): the C ABI.
 *
 * Implements the method of M. A. Anam and Y. Andreopoulos, "Reliable Linear,
 * Sesquilinear and Bijective Operations on Integer Data Streams via
 * Numerical Entanglement" (IEEE Trans. Signal Processing; arXiv 1604.04740):
 * M >= 3 integer streams are entangled in place, an LSB operation runs on the
 * entangled streams unchanged, and the results are disentangled with
 * additions and shifts, checked for any single-stream fault, or recovered
 * from M-1 streams after a fail-stop loss.
 *
 * General conventions (every entry point):
 *   - Pointers named as device pointers must point to device memory of the
 *     current HIP device (any allocator; 16-byte aligned where stated).
 *     The caller owns every buffer; the library allocates no device memory
 *     and keeps no global state (the batch planner's small host-side plan
 *     object is the one allocation, released by ne_batch_free).
 *   - Streams are stored stream-major: element n of stream m is at
 *     [m * N + n] (N = elements per stream); matrices are row-major.
 *   - Words are w = 64-bit two's complement (int64).  Every word operation
 *     wraps modulo 2^64; the paper's 2w-bit interim of the disentanglement
 *     is evaluated exactly.
 *   - `stream` is a hipStream_t (NULL = the default stream).  Every call is
 *     asynchronous on that stream.  Argument errors are returned before any
 *     launch; a failed launch returns NE_ELAUNCH.  Nothing throws.
 *   - Fault flags are bitmasks: bit (n % 32) of word (n / 32) is set when
 *     position n fails the reliability check.  Every word of the mask is
 *     written (no pre-clearing needed).  `n_bad` (a device
 *     unsigned long long) is INCREMENTED by the number of flagged positions:
 *     clear it before the first call whose count you want.
 *   - GPU limits: 3 <= M <= 16 for element-wise entry points, 3 <= M <= 8
 *     for the fused GEMM; l >= 2.
 *   - Word width: w = 64 everywhere.  The element-wise entry points
 *     (ne_entangle, ne_lsb_permute_scale, ne_disentangle_check, ne_recover,
 *     ne_permute_scale_fused) also take w = 32, the word width of the
 *     paper's Table II: their word buffers (eps, delta, d_hat, scale, add,
 *     delta_rebuilt) are then int32, every word operation wraps modulo
 *     2^32, and the disentanglement's 2w-bit interim is 64-bit.  Other
 *     entry points return NE_EUNSUP for w != 64.
 */
#ifndef NE_H
#define NE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ------------------------------------------------------------ return codes */
#define NE_OK 0
#define NE_EINVAL (-1)  /* bad M/w/l/k/r, negative size, NULL pointer, bad dtype  */
#define NE_ERANGE (-2)  /* a-priori output bound exceeds the entangled range D     */
#define NE_EALIAS (-3)  /* two buffers overlap where they must not                */
#define NE_EALIGN (-4)  /* a pointer or row pitch is not aligned as required      */
#define NE_EUNSUP (-5)  /* valid for the method but not built for the GPU         */
#define NE_ELAUNCH (-6) /* the HIP launch failed                                  */

/* ------------------------------------------------------------- element types */
#define NE_I8 1
#define NE_I32 4
#define NE_I64 8

typedef void *ne_stream_t; /* hipStream_t */

/*
 * Entanglement parameters (section III-C): M streams, word width w, shift l
 * and overlap k with (M-1) l + k <= w and k <= l.  r_check selects the
 * stream that the reliability check rebuilds (any 0 <= r_check < M works;
 * the detection proofs in the appendix use stream 0).
 */
typedef struct ne_params {
    int32_t M, w, l, k, r_check;
} ne_params_t;

/* Human-readable message for a return code (static storage). */
const char *ne_strerror(int code);

/* Library version: major * 10000 + minor * 100 + patch. */
int ne_version(void);

/*
 * (l, k) by the rule of section III-C: maximise the supported output width
 * (M-2) l + k subject to (M-1) l + k <= w and k <= l.  The paper leaves ties
 * open (at w = 64 they occur for M = 3 and M = 7); this picks the pair with
 * (M-1) l + k == w, which guarantees M l >= w (then every single-stream
 * corruption is detectable, not only bit flips), then the larger l.
 * Fills *out with r_check = 0.  NE_EINVAL if M < 3, w not in [4, 64], or no
 * admissible pair exists.
 */
int ne_params_default(int32_t M, int32_t w, ne_params_t *out);

/*
 * The output dynamic range of section III-C: every output d of the LSB
 * operation must satisfy |d| <= D = 2^((M-3) l + k) (2^(l-1) - 1) for
 * extraction to be exact.  NE_EINVAL on invalid parameters.
 */
int ne_range_bound(const ne_params_t *p, int64_t *D);

/*
 * Entanglement, section III-C (the circulant operator E; section III-A for
 * M = 3): for every position n and stream m,
 *     eps[m][n] = c[m][n] + 2^l * c[(m - 1) mod M][n]    (mod 2^w).
 *   c       device, [M][N] elements of type c_dtype (NE_I8, NE_I32, NE_I64;
 *           taken modulo 2^w).
 *   eps     device, [M][N] words (int64; int32 for w = 32).  May equal c
 *           when c_dtype is the word type (in place, as the paper stores
 *           entangled streams in place of the inputs); must not otherwise
 *           overlap c.
 *   N       elements per stream, >= 0.
 */
int ne_entangle(const void *c, int32_t c_dtype, void *eps, int64_t N,
                const ne_params_t *p, ne_stream_t stream);

/*
 * The GEMM of section III-A applied, unchanged, to the entangled streams:
 *     delta[m] = eps[m] * G     (int64 words, mod 2^64),
 * for every stream m, with G the shared operand.  The routine is unaware of
 * entanglement: it treats eps as generic 64-bit words, split into signed
 * int8 digits on int8 matrix cores with exact int32 accumulation.
 *   eps       device, [M][n][K] int64.
 *   eps_bits  bound on the words: every eps value lies in
 *             [-2^(eps_bits-1), 2^(eps_bits-1)); 1..64.  Sets the digit count
 *             min(8, eps_bits/8 + 1); 64 is always safe.
 *   Gt        device, the shared operand TRANSPOSED: Gt[j][k] = G[k][j],
 *             [N][K] int8 (K contiguous, the layout int8 matrix cores read).
 *   delta     device, [M][n][N] int64; must not overlap eps or Gt.
 *   K         <= 131071 (keeps every int32 digit accumulator exact).
 */
int ne_lsb_gemm(const int64_t *eps, int32_t eps_bits, const int8_t *Gt, int64_t *delta,
                int64_t n, int64_t K, int64_t N, const ne_params_t *p, ne_stream_t stream);

/*
 * Circular convolution of each entangled stream with the shared kernel g
 * (section II, the star operator):
 *     delta[m][t] = sum_{j=0}^{N-1} eps[m][(t - j) mod N] * g[j]   (mod 2^64).
 *   eps       device, [M][N] int64;  eps_bits as for ne_lsb_gemm.
 *   g         device, [N] int8.
 *   delta     device, [M][N] int64; must not overlap eps.
 *   N         1 .. 131071.  Evaluated on int8 matrix cores: each block of
 *             1024 outputs is a Toeplitz x Hankel matrix product over the
 *             taps, the words split into min(8, eps_bits/8 + 1) signed int8
 *             digits with exact int32 accumulation, recombined mod 2^64.
 *   workspace device scratch of ne_circconv_workspace(N, M, 0) bytes, or
 *             NULL.  With it the taps of every block are split over
 *             workgroups (64-bit partial sums in the workspace, then a
 *             reduction launch), which fills the chip when N is small; with
 *             NULL one workgroup computes each block.  Caller-owned, 8-byte
 *             aligned, must not overlap the other arguments; its contents on
 *             entry do not matter.  A workspace smaller than required is
 *             NE_EINVAL.
 */
int ne_lsb_circconv(const int64_t *eps, int32_t eps_bits, const int8_t *g, int64_t *delta,
                    int64_t N, const ne_params_t *p, void *workspace, int64_t workspace_bytes,
                    ne_stream_t stream);

/*
 * Linear convolution of each entangled stream (N samples) with a short
 * kernel of L taps (section IV: long streams filtered by short kernels,
 * which the paper processes in overlap-save blocks):
 *     delta[m][t] = sum_{j=0}^{L-1} eps[m][t - j] * g[j]   (mod 2^64),
 *     0 <= t < N + L - 1, eps taken as zero outside [0, N).
 * Every block of 1024 outputs is one Toeplitz x Hankel matrix product over
 * the L + 32 taps that reach it, on int8 matrix cores (digits as for
 * ne_lsb_gemm), so the work is proportional to L, not to N.
 *   eps       device, [M][N] int64; eps_bits as for ne_lsb_gemm.
 *   g         device, [L] int8.
 *   delta     device, [M][N + L - 1] int64; must not overlap eps or g.
 *   workspace device scratch of ne_linconv_workspace(N, L, M, eps_bits, 0)
 *             bytes (16-byte aligned, overlapping no other buffer), or
 *             NULL.  With a workspace a pre-pass writes the int8 digits of
 *             every stream, zero-padded, as byte planes, and the blocks
 *             stage their operands from them with aligned 4-byte loads and
 *             no bounds tests; with NULL the blocks form the digits from
 *             eps themselves.  Results are identical.  Contents on entry do
 *             not matter; a smaller workspace is NE_EINVAL.
 *   N >= 1, 1 <= L <= 131071, N + L - 1 <= 2^30 (else NE_EINVAL).
 */
int ne_lsb_linconv(const int64_t *eps, int32_t eps_bits, const int8_t *g, int64_t L,
                   int64_t *delta, int64_t N, const ne_params_t *p, void *workspace,
                   int64_t workspace_bytes, ne_stream_t stream);

/*
 * Workspace bytes of ne_lsb_linconv (fused = 0, bits = eps_bits) and
 * ne_linconv_fused (fused = 1, bits = c_bits) for M streams of N samples
 * and L taps: M * digits * planes of about N + 2 L + 4096 bytes each, plus
 * L + 1024 bytes for the padded taps; 0 for invalid sizes.
 */
int64_t ne_linconv_workspace(int64_t N, int64_t L, int32_t M, int32_t bits, int32_t fused);

/*
 * Workspace bytes that ne_lsb_circconv (fused = 0) or ne_circconv_fused
 * (fused = 1) uses for N taps and M streams; 0 when the taps are not split
 * (then the workspace argument is ignored), and 0 for invalid sizes.
 */
int64_t ne_circconv_workspace(int64_t N, int32_t M, int32_t fused);

/*
 * Fixed permutation, scaling and addition on the entangled streams (section
 * II, op in {permutation, x, +}; the constant is self-entangled as the
 * footnote of section III-A requires for + and -):
 *     delta[m][n] = scale[n] * eps[m][perm[n]] + (2^l + 1) * add[n]  (mod 2^w)
 *   eps       device, [M][N] words (int64; int32 for w = 32).
 *   perm      device, [N] int32, a bijection of 0..N-1 (values out of range
 *             are clamped, never read out of bounds).
 *   scale     device, [N] words, or NULL for 1.
 *   add       device, [N] words, un-entangled constant, or NULL for 0.
 *   delta     device, [M][N] words; must not overlap eps.
 */
int ne_lsb_permute_scale(const void *eps, const int32_t *perm, const void *scale,
                         const void *add, void *delta, int64_t N, const ne_params_t *p,
                         ne_stream_t stream);

/*
 * Disentanglement and the post-computation reliability check (section
 * III-C; the check of the generalised detection proof in the appendix),
 * with r = p->r_check:
 *     d_temp = (-1)^M sum_{m=0}^{M-2} (-1)^m 2^((M-2-m) l) delta[(r+1+m) mod M]
 *     d_hat[(r+M-1) mod M] = sign-extended low (M-1) l bits of d_temp
 *     d_hat[r] = (-1)^M (d_temp - d_hat[(r+M-1) mod M]) >> (M-1) l
 *     d_hat[(r+m) mod M] = delta[(r+m) mod M] - 2^l d_hat[(r+m-1) mod M], 1 <= m <= M-2
 *     flag[n] = delta[r][n] != d_hat[r][n] + 2^l d_hat[(r+M-1) mod M][n]  (exact)
 * (the leading (-1)^M and the chain bound m <= M-2 are the readings of the
 * printed formulas that make them exact for every M; for M = 3 they reduce
 * to the special form of section III-A).  d_hat keeps the low w bits; the
 * check compares the stored d_hat exactly in 2w bits.
 *   delta     device, [M][N] words (int64; int32 for w = 32).
 *   d_hat     device, [M][N] words; may equal delta (in place).
 *   flags     device, [ceil(N/32)] uint32 bitmask, or NULL.
 *   n_bad     device counter (incremented), or NULL.
 */
int ne_disentangle_check(const void *delta, void *d_hat, uint32_t *flags,
                         unsigned long long *n_bad, int64_t N, const ne_params_t *p,
                         ne_stream_t stream);

/*
 * Fail-stop recovery (Propositions 1 and 3): every output from the M-1
 * surviving entangled streams, i.e. the disentanglement above with r = lost.
 *   delta          HOST array of M device pointers to the [N] word output
 *                  of each stream (int64; int32 for w = 32); delta[lost] is
 *                  never read (may be NULL).
 *   lost           0 <= lost < M.
 *   d_hat          device, [M][N] words; must not overlap any delta[m].
 *   delta_rebuilt  device, [N] words or NULL: the lost stream re-created as
 *                  d_hat[lost] + 2^l d_hat[(lost+M-1) mod M] (mod 2^w).
 */
int ne_recover(const void *const *delta, int32_t lost, void *d_hat, void *delta_rebuilt,
               int64_t N, const ne_params_t *p, ne_stream_t stream);

/*
 * Optional fault injection into the fused GEMM (for measuring detection):
 * before extraction, entangled output word delta[stream[i]] at flat position
 * position[i] (= row * N + col) is XOR-ed with xor_mask[i].  Positions must
 * be sorted ascending.  All arrays are device arrays of length count.
 */
typedef struct ne_inject {
    int64_t count;
    const int64_t *position;
    const int32_t *stream;
    const uint64_t *xor_mask;
} ne_inject_t;

/*
 * The fused hot path for the GEMM of section III-A on int8 inputs, one
 * launch: entangle in the prologue, int8-matrix-core GEMM on the entangled
 * words, then disentangle and check in the epilogue; delta never reaches
 * memory.  For stream m the entangled word is c[m] + 2^l c[m-1 mod M], whose
 * signed int8 digits at bit offsets 0 and l are c[m] and c[m-1]; each is
 * multiplied by G on its own (so a fault in one stream's product stays in
 * that stream), and delta[m] = P_lo + 2^l P_hi is formed in int64.
 *   c         device, [M][n][K] int8 (16-byte aligned; K % 16 == 0 is the
 *             fast path, any K works).
 *   Gt        device, [N][K] int8, the shared operand transposed.
 *   d_hat     device, [M][n][N] of out_dtype (NE_I32 or NE_I64; I32 keeps
 *             the low 32 bits, exact whenever |d| < 2^31, which holds for
 *             K <= 131071 on int8 inputs).
 *   flags     device bitmask, ROW-PADDED: [n][ceil(N/32)] uint32 (bit
 *             (col % 32) of word [row][col / 32]), or NULL.
 *   n_bad     device counter (incremented), or NULL.
 *   inject    HOST pointer to an injection table (device arrays), or NULL.
 * NE_ERANGE if K * 128 * 128 > D (the a-priori bound for int8 data).
 */
int ne_gemm_fused(const int8_t *c, const int8_t *Gt, void *d_hat, int32_t out_dtype,
                  uint32_t *flags, unsigned long long *n_bad, int64_t n, int64_t K, int64_t N,
                  const ne_params_t *p, const ne_inject_t *inject, ne_stream_t stream);

/*
 * Baseline: the plain (fault-intolerant) int8 GEMM of the stacked streams,
 * C[R][N] = A[R][K] * B (int32), with B given transposed as Bt[N][K].
 * Same matrix-core pipeline as the fused path.  K <= 131071.
 */
int ne_plain_gemm_i8(const int8_t *A, const int8_t *Bt, int32_t *C, int64_t R, int64_t K,
                     int64_t N, ne_stream_t stream);

/*
 * Baseline: checksum-stream ABFT of section II-A for the same GEMM.  The
 * checksum stream r = sum_m c[m] (two signed int8 digits, since
 * |r| <= 128 M) is multiplied by G alongside the M streams, and the epilogue
 * flags positions where sum_m d[m] != e (section II-A).
 *   c  device [M][n][K] int8;  Gt device [N][K] int8;
 *   d  device [M][n][N] int32;  flags row-padded as for ne_gemm_fused.
 *   workspace  device, ne_abft_workspace(n, K) bytes (16-byte aligned, no
 *              overlap with the other arguments), or NULL.  With it a first
 *              launch writes the checksum stream as two int8 digit planes
 *              and the GEMM runs every source through the DMA pipeline of
 *              the fused path (K % 16 == 0 and 16-byte aligned c and Gt;
 *              otherwise the workspace is not used); with NULL one launch
 *              builds the checksum while staging its operands.
 */
int ne_abft_gemm_i8(const int8_t *c, const int8_t *Gt, int32_t *d, uint32_t *flags,
                    unsigned long long *n_bad, int32_t M, int64_t n, int64_t K, int64_t N,
                    void *workspace, int64_t workspace_bytes, ne_stream_t stream);

/* Workspace bytes of ne_abft_gemm_i8: 2 n K (0 for invalid sizes). */
int64_t ne_abft_workspace(int64_t n, int64_t K);

/*
 * Baseline: row/column checksum ABFT (Huang and Abraham; the "RC-check" of
 * the GEMM comparison in section V) for M independent subblock products
 * d[m] = c[m] G.  The checksums of the inputs, e^T c[m] and G e (e all
 * ones), give every row sum and column sum the product must have:
 *     sum_p d[m][i][p] = c[m][i] . (G e),   sum_i d[m][i][p] = (e^T c[m]) . G[:, p]
 * A row or column whose sum differs (exact 64-bit integers) is flagged; a
 * wrong position is at the crossing of a flagged row and a flagged column,
 * and up to three wrong positions per subblock are always detected.  The
 * product itself is the plain int8 GEMM (ne_plain_gemm_i8); the checks are
 * separate passes over c, G and d.
 *   c          device [M][n][K] int8;  Gt device [N][K] int8 (G transposed).
 *   d          device [M][n][N] int32 (written).
 *   row_flags  device [M][ceil(n/32)] uint32, bit i % 32 of word
 *              [m][i / 32] set for a flagged row, or NULL.
 *   col_flags  device [M][ceil(N/32)] uint32, likewise for columns, or NULL.
 *   n_bad      device counter, incremented by the number of flagged rows
 *              and columns, or NULL.
 *   workspace  device, ne_abft_rc_workspace(M, K, N) bytes, 16-byte aligned
 *              (required; contents on entry do not matter).
 *   1 <= M <= 4096, 1 <= n, N <= 2^20, 1 <= K <= 131071, else NE_EINVAL.
 *   Written buffers must not overlap any other argument (NE_EALIAS).
 */
int ne_abft_rc_gemm_i8(const int8_t *c, const int8_t *Gt, int32_t *d, uint32_t *row_flags,
                       uint32_t *col_flags, unsigned long long *n_bad, int32_t M, int64_t n,
                       int64_t K, int64_t N, void *workspace, int64_t workspace_bytes,
                       ne_stream_t stream);

/*
 * The check of ne_abft_rc_gemm_i8 alone, on a given product d (read
 * only): for callers that compute the product themselves, and for fault
 * injection into d.  Arguments as above.
 */
int ne_abft_rc_check_i8(const int8_t *c, const int8_t *Gt, const int32_t *d, uint32_t *row_flags,
                        uint32_t *col_flags, unsigned long long *n_bad, int32_t M, int64_t n,
                        int64_t K, int64_t N, void *workspace, int64_t workspace_bytes,
                        ne_stream_t stream);

/* Workspace bytes of the row/column checksum ABFT: 4 (M + 1) K rounded up
 * to 16, plus 8 M N; 0 for invalid sizes. */
int64_t ne_abft_rc_workspace(int32_t M, int64_t K, int64_t N);

/*
 * Fused circular convolution, one launch: the star operator of section II on
 * the entangled words, then disentangle and check (section III-C).  delta
 * never reaches memory.  Each block of 1024 outputs is a Toeplitz x Hankel
 * product on int8 matrix cores; the entangled word of stream m is formed in
 * the accumulation, conv(c_m, g) + 2^l conv(c_{m-1}, g), with the two
 * products of every stream computed separately (a fault in one stream's
 * computation reaches only that stream).  Inputs wider than a byte are
 * split into signed int8 digits (1 digit if c_bits <= 8, else
 * min(8, c_bits/8 + 1)), one pass over the taps per digit.
 *   c         device, [M][N] of c_dtype (NE_I8, NE_I32 or NE_I64).
 *   c_bits    bound on the inputs: |c| < 2^(c_bits-1); with |g| <= 128 it
 *             gives the a-priori bound N * 2^(c_bits-1) * 128, which must not
 *             exceed D (section III-C), else NE_ERANGE.
 *   g         device, [N] int8.
 *   d_hat     device, [M][N] of out_dtype (NE_I32 keeps the low 32 bits).
 *   flags     device, [ceil(N/32)] uint32 bitmask, or NULL.
 *   n_bad     device counter (incremented), or NULL.
 *   N         1 .. 131071.
 *   workspace as for ne_lsb_circconv, ne_circconv_workspace(N, M, 1) bytes.
 */
int ne_circconv_fused(const void *c, int32_t c_dtype, int32_t c_bits, const int8_t *g,
                      void *d_hat, int32_t out_dtype, uint32_t *flags,
                      unsigned long long *n_bad, int64_t N, const ne_params_t *p,
                      void *workspace, int64_t workspace_bytes, ne_stream_t stream);

/*
 * Fused permutation + scaling + addition (section II, op in
 * {permutation, x, +}, with the constant self-entangled per the footnote of
 * section III-A): for every position n the M inputs at perm[n] are
 * entangled, delta = scale[n] eps + (2^l + 1) add[n], then disentangled and
 * checked.  The caller guarantees |scale[n] c + add[n]| <= D (the range of
 * section III-C); it is not checked a priori.
 *   c          device, [M][N] of c_dtype;  perm device [N] int32 (clamped);
 *   scale/add  device [N] words (int64; int32 for w = 32) or NULL;
 *   d_hat      device [M][N] out_dtype (NE_I32 only for w = 32);
 *   flags      device [ceil(N/32)] or NULL; n_bad device counter or NULL.
 *   workspace  device scratch of ne_permute_workspace(N, M, c_dtype) bytes,
 *              or NULL.  With it a first launch copies the inputs into rows
 *              (the M inputs of a position side by side, 64-bit padded) so
 *              that each position's random gather touches one cache line
 *              instead of M; with NULL one launch gathers from c directly.
 *              Caller-owned, 8-byte aligned, no overlap with the other
 *              arguments, contents on entry irrelevant; too small is
 *              NE_EINVAL.
 */
int ne_permute_scale_fused(const void *c, int32_t c_dtype, const int32_t *perm,
                           const void *scale, const void *add, void *d_hat, int32_t out_dtype,
                           uint32_t *flags, unsigned long long *n_bad, int64_t N,
                           const ne_params_t *p, void *workspace, int64_t workspace_bytes,
                           ne_stream_t stream);

/*
 * The linear convolution above fused with entanglement, disentanglement
 * and the check (the pattern of ne_circconv_fused): c in plain form, the
 * entangled words formed on load, d_hat = the linear convolution of every
 * input stream with g, exactly.
 *   c         device, [M][N] of c_dtype (NE_I8, NE_I32, NE_I64), |c| <
 *             2^(c_bits-1).
 *   g         device, [L] int8.
 *   d_hat     device, [M][N + L - 1] of out_dtype (NE_I32 or NE_I64).
 *   flags     device, [ceil((N + L - 1) / 32)] uint32, or NULL; n_bad as
 *             usual.
 *   workspace as for ne_lsb_linconv, ne_linconv_workspace(N, L, M, c_bits,
 *             1) bytes, or NULL (the planes hold the digits of c).
 *   Sizes as for ne_lsb_linconv; NE_ERANGE unless L 2^(c_bits-1) 128 <= D.
 *   One workgroup per block of 1024 outputs; M <= 8.
 */
int ne_linconv_fused(const void *c, int32_t c_dtype, int32_t c_bits, const int8_t *g, int64_t L,
                     void *d_hat, int32_t out_dtype, uint32_t *flags, unsigned long long *n_bad,
                     int64_t N, const ne_params_t *p, void *workspace, int64_t workspace_bytes,
                     ne_stream_t stream);

/*
 * Workspace bytes of ne_permute_scale_fused: N * ceil(M * c_dtype / 8) * 8;
 * 0 for invalid sizes.
 */
int64_t ne_permute_workspace(int64_t N, int32_t M, int32_t c_dtype);

/* ------------------------------------------------------- operation series */

#define NE_SERIES_GEMM 0
#define NE_SERIES_CONV 1
#define NE_SERIES_SCALE_ADD 2
#define NE_SERIES_PERMUTE 3

/*
 * One operation of a series applied consecutively to the entangled streams
 * before a single disentanglement (section II), described by its a-priori
 * bounds:
 *   NE_SERIES_GEMM       length = K (contraction length), operand_max >= |G|
 *   NE_SERIES_CONV       length = taps N,                 operand_max >= |g|
 *   NE_SERIES_SCALE_ADD  length >= |scale|,               operand_max >= |add|
 *   NE_SERIES_PERMUTE    both ignored
 */
typedef struct ne_series_op {
    int32_t kind, reserved;
    int64_t length, operand_max;
} ne_series_op_t;

/*
 * Range composition of a series.  The output condition of section III-C,
 * |d| <= D, applies to the series' final output only: every operation is
 * linear modulo 2^64 (the + constant entering self-entangled), so the words
 * after the last operation are E(d) mod 2^64 even where intermediate values
 * leave the range.  With B_0 = c_max (|inputs| <= c_max):
 *     GEMM, conv:  B_{i+1} = B_i * length * operand_max
 *     scale/add:   B_{i+1} = B_i * length + operand_max
 *     permute:     B_{i+1} = B_i
 *   eps_bits  host, [n_ops] int32, or NULL: for operation i, the eps_bits
 *             argument of ne_lsb_gemm / ne_lsb_circconv for the entangled
 *             words entering it: the smallest b with (2^l + 1) B_i <
 *             2^(b-1), at most 64 (words that may have wrapped need all 64).
 *   out_max   host, or NULL: B_{n_ops}, saturated at INT64_MAX.
 * Returns NE_ERANGE when B_{n_ops} > D (outputs are still written), and
 * NE_EINVAL for invalid parameters, c_max < 0, n_ops < 0, ops == NULL with
 * n_ops > 0, an unknown kind or a negative bound.  Host arithmetic only (no
 * device work; callable without a GPU).
 */
int ne_series_range(const ne_params_t *p, int64_t c_max, int32_t n_ops,
                    const ne_series_op_t *ops, int32_t *eps_bits, int64_t *out_max);

/*
 * The series GEMM -> scale / add -> permutation on the entangled streams
 * with one disentanglement at the end (section II's series; the + constant
 * self-entangled as in the footnote of section III-A):
 *     delta1[m] = eps[m] * G,   eps[m] = c[m] + 2^l c[(m-1) mod M]
 *     delta2[m][q] = scale[q] * delta1[m][q] + (2^l + 1) * add[q]
 *     delta3[m][q] = delta2[m][perm[q]]
 *     d_hat, flags = disentanglement and check of delta3 (as
 *                    ne_disentangle_check, r = p->r_check)
 * (all mod 2^64), q = row * N + col indexing the n * N outputs of a stream.
 * Two launches: the GEMM on int8 matrix cores as in ne_gemm_fused, with
 * scale and add applied to the entangled words in its epilogue, writes
 * delta2 into the workspace position-major (the M words of a position side
 * by side, [n * N][M]); the second reads one such row per output position
 * at perm[q], disentangles and checks.  The words stay entangled from the
 * prologue of the first launch to the check of the second.
 *   c, Gt, n, K, N  as for ne_gemm_fused; n * N <= 2^31 - 1.
 *   scale, add      device, [n * N] int64, or NULL (1 and 0).
 *   perm            device, [n * N] int32, a bijection of 0..n*N-1 (values
 *                   out of range are clamped, never read out of bounds).
 *   scale_max, add_max  bounds on |scale| and |add| (ignored for NULL);
 *                   NE_ERANGE unless K * 128 * 128 * scale_max + add_max
 *                   <= D.  The library cannot read device data before the
 *                   launch, so it trusts them.
 *   d_hat           device, [M][n * N] of out_dtype (NE_I32 or NE_I64).
 *   flags           device, [ceil(n * N / 32)] uint32, or NULL.
 *   n_bad           device counter (incremented), or NULL.
 *   workspace       device, ne_series_workspace(n, N, M) bytes, 16-byte
 *                   aligned, caller-owned, no overlap with any other
 *                   argument; contents on entry irrelevant.  Too small is
 *                   NE_EINVAL.
 */
int ne_series_gemm_scale_permute(const int8_t *c, const int8_t *Gt, const int64_t *scale,
                                 const int64_t *add, const int32_t *perm, int64_t scale_max,
                                 int64_t add_max, void *d_hat, int32_t out_dtype,
                                 uint32_t *flags, unsigned long long *n_bad, int64_t n,
                                 int64_t K, int64_t N, const ne_params_t *p, void *workspace,
                                 int64_t workspace_bytes, ne_stream_t stream);

/* Workspace bytes of ne_series_gemm_scale_permute: n * N * M * 8; 0 for
 * invalid sizes or M outside 3..8. */
int64_t ne_series_workspace(int64_t n, int64_t N, int32_t M);

/* ------------------------------------------------------------------ batch */

#define NE_OP_GEMM 0
#define NE_OP_CONV 1
#define NE_OP_PERM 2

/*
 * One independent problem of a batch.  Parameters (l, k) follow the rule of
 * ne_params_default for its M (3..8, w = 64); r_check picks the check stream.
 *   NE_OP_GEMM: c [M][n][K] int8 (16-byte aligned, K % 16 == 0), g = Gt
 *               [N][K] int8; d_hat [M][n][N]; flags row-padded
 *               [n][ceil(N/32)] as in ne_gemm_fused.
 *   NE_OP_CONV: c [M][N] int8, g [N] int8 (circular convolution); d_hat
 *               [M][N]; flags [ceil(N/32)].
 *   NE_OP_PERM: c [M][N] int8, perm [N] int32, scale / add [N] int64 or
 *               NULL; d_hat [M][N]; flags [ceil(N/32)].
 * All pointers are device pointers; flags and n_bad may be NULL.
 */
typedef struct ne_problem {
    int32_t op, M, r_check, out_dtype;
    int64_t n, K, N;
    const void *c;
    const void *g;
    const int32_t *perm;
    const int64_t *scale;
    const int64_t *add;
    void *d_hat;
    uint32_t *flags;
    unsigned long long *n_bad;
} ne_problem_t;

/*
 * Per-bucket choices, indexed [M - 3][size class]; size class 0: largest
 * dimension <= 256, 1: <= 1024, 2: larger.  gemm_bn is the output-tile width
 * of a GEMM work item (128, or 256 for M <= 4); perm_chunk the number of
 * positions of a permute/scale work item (a multiple of 64).
 */
typedef struct ne_batch_tuning {
    int32_t gemm_bn[6][3];
    int64_t perm_chunk[6][3];
} ne_batch_tuning_t;

typedef struct ne_batch ne_batch_t; /* opaque host-side plan */

/*
 * Plan a batch: validates every problem, splits it into work items (GEMM
 * output tiles, 1024-position convolution blocks, permute/scale chunks: a
 * copy of the inputs into rows, then the gather), deals them to the XCDs (a
 * GEMM's tiles in eight runs of neighbouring tiles, so that the tiles
 * sharing an L2 share operands; the other items in turn), balances each
 * XCD's items over its workgroups by a cost estimate (longest first, each
 * to the least loaded workgroup), and writes the problem table, the
 * per-workgroup lists and room for the row copies into the caller's device
 * buffer table_dev (256-byte
 * aligned, table_bytes long; it must not be in use by a pending run).  With
 * table_dev == NULL only *table_needed is set.  tuning may be NULL
 * (defaults).  On success *plan is a small host object (the only thing the
 * library allocates; free it with ne_batch_free).  Setup call: blocking,
 * not for graph capture.
 */
int ne_batch_plan(const ne_problem_t *problems, int32_t count, const ne_batch_tuning_t *tuning,
                  void *table_dev, int64_t table_bytes, int64_t *table_needed,
                  ne_batch_t **plan);

/*
 * Run a planned batch: up to three launches, in order: the permutations'
 * row copies, the GEMM tiles and convolution blocks (one persistent
 * workgroup per compute unit, each running the list the plan gave it),
 * and the permutation gathers (the two permutation phases split each list
 * over several workgroups without LDS).  Plain kernels only, so the call
 * can be captured into a HIP graph and replayed.  Runs that share a table
 * must not overlap (the row copies live in the table).
 */
int ne_batch_run(const ne_batch_t *plan, ne_stream_t stream);

/* Number of work items of a plan (-1 for NULL). */
int ne_batch_items(const ne_batch_t *plan);

void ne_batch_free(ne_batch_t *plan);

/*
 * Autotuner: for every (operation, M, size class) bucket present in the
 * problem list, plans and times (reps runs, HIP events) each candidate of
 * that bucket on the device and keeps the fastest in *out (other buckets get
 * defaults).  Runs the problems (overwriting their outputs) and uses
 * table_dev as scratch for the plans.  Blocking.
 */
int ne_batch_autotune(const ne_problem_t *problems, int32_t count, void *table_dev,
                      int64_t table_bytes, int32_t reps, ne_batch_tuning_t *out,
                      ne_stream_t stream);

#ifdef __cplusplus
}
#endif

#endif /* NE_H */
