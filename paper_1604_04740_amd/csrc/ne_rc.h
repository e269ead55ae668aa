// ne_rc.h -- launchers of the row/column checksum ABFT baseline
// (ne_abft_rc.hip), called by the C-ABI layer.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace ne {

// Workspace bytes: column sums of every subblock [M][K] and of G [K]
// (int32), then the column sums of the product [M][N] (int64).
int64_t rc_workspace_bytes(int64_t M, int64_t K, int64_t N);

// gemm: also compute d = c G (the plain int8 GEMM) before the check.
int launch_abft_rc(const int8_t *c, const int8_t *Gt, int32_t *d, uint32_t *row_flags,
                   uint32_t *col_flags, unsigned long long *n_bad, int64_t M, int64_t n, int64_t K,
                   int64_t N, void *ws, bool gemm, hipStream_t s);

} // namespace ne
