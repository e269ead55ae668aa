"""CPU tests of the C ABI's host logic: the library loads, exports every
symbol include/ne.h declares, applies the paper's parameter rule, and
rejects bad arguments before any launch (no GPU needed)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def ne():
    import paper_1604_04740_amd as ne
    ne.lib()
    return ne


def _declared():
    src = open(os.path.join(ROOT, "include", "ne.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(ne_[a-z0-9_]+)\s*\(", src)))


def test_exports_every_declared_symbol(ne):
    names = _declared()
    assert "ne_gemm_fused" in names and "ne_recover" in names
    for n in names:
        assert hasattr(ne.lib(), n), n


def test_params_rule_matches_oracle(ne, orc):
    for w in (16, 24, 32, 48, 64):
        for M in range(3, 33):
            try:
                ref = orc.params(M, w)
            except ValueError:
                continue
            p = ne.ne_params_default(M, w)
            assert (p.l, p.k) == ref, (M, w)
            if ref[0] >= 2 and w == 64:
                assert ne.ne_range_bound(p) == orc.range_bound(M, *ref)


def test_argument_errors_before_launch(ne):
    L = ne.lib()
    P = ne.Params
    bad = [P(2, 64, 22, 20, 0), P(3, 64, 22, 23, 0), P(3, 64, 30, 20, 0), P(3, 64, 22, 20, 3),
           P(3, 64, 1, 1, 0)]
    for p in bad:
        rc = L.ne_disentangle_check(ctypes.c_void_p(16), ctypes.c_void_p(64), None, None, 10,
                                    ctypes.byref(p), None)
        assert rc == -1, p
    # valid for the method, not built for the GPU: w = 48, and w = 32 for
    # the matrix-core entry points; w = 32 is accepted element-wise
    p = ne.ne_params_default(3, 48)
    rc = L.ne_disentangle_check(ctypes.c_void_p(16), ctypes.c_void_p(64), None, None, 10,
                                ctypes.byref(p), None)
    assert rc == -5
    p = ne.ne_params_default(3, 32)
    rc = L.ne_disentangle_check(ctypes.c_void_p(16), ctypes.c_void_p(4096), ctypes.c_void_p(16),
                                None, 10, ctypes.byref(p), None)
    assert rc == -3  # accepted, then rejected for the flags overlap, before any launch
    rc = L.ne_lsb_gemm(ctypes.c_void_p(16), 8, ctypes.c_void_p(4096), ctypes.c_void_p(8192), 4,
                       16, 4, ctypes.byref(p), None)
    assert rc == -5
    p = ne.ne_params_default(3)
    # overlapping delta / d_hat (not identical)
    rc = L.ne_disentangle_check(ctypes.c_void_p(4096), ctypes.c_void_p(4096 + 8), None, None, 10,
                                ctypes.byref(p), None)
    assert rc == -3
    # misaligned
    rc = L.ne_disentangle_check(ctypes.c_void_p(4097), ctypes.c_void_p(1 << 20), None, None, 10,
                                ctypes.byref(p), None)
    assert rc == -4
    # K too large for exact int32 digit accumulation
    rc = L.ne_lsb_gemm(ctypes.c_void_p(16), 64, ctypes.c_void_p(1 << 30), ctypes.c_void_p(1 << 31),
                       4, 131072, 4, ctypes.byref(p), None)
    assert rc == -1
    # fused: M beyond the fused build
    p9 = ne.ne_params_default(9)
    rc = L.ne_gemm_fused(ctypes.c_void_p(16), ctypes.c_void_p(1 << 20), ctypes.c_void_p(1 << 30),
                         4, None, None, 4, 16, 4, ctypes.byref(p9), None, None)
    assert rc == -5
    # empty inputs are a no-op success, even with NULL buffers
    rc = L.ne_entangle(None, 8, None, 0, ctypes.byref(p), None)
    assert rc == 0
    assert ne.ne_strerror(-2).startswith("output range")


def test_range_rejection_fused(ne):
    """The a-priori bound K * 128 * 128 must not exceed D (section III-C)."""
    L = ne.lib()
    p = ne.Params(3, 64, 22, 20, 0)
    D = ne.ne_range_bound(p)
    K_ok = D // (128 * 128)
    assert K_ok > 131071  # every admissible K fits at w = 64, M = 3
    # a narrower l makes the bound bite
    p_small = ne.Params(3, 64, 10, 10, 0)
    D2 = ne.ne_range_bound(p_small)
    K_bad = D2 // (128 * 128) + 1
    rc = L.ne_gemm_fused(ctypes.c_void_p(16), ctypes.c_void_p(1 << 20), ctypes.c_void_p(1 << 30),
                         4, None, None, 4, K_bad, 4, ctypes.byref(p_small), None, None)
    assert rc == -2


def test_conv_workspace_size_and_rejection(ne):
    """The split of the taps the workspace query reports, and a workspace
    smaller than that is rejected before any launch."""
    L = ne.lib()
    # 16 blocks of 1024 outputs, 64 steps of 256 taps: 16 splits of 4 steps
    assert L.ne_circconv_workspace(16384, 3, 1) == 16 * 3 * 16384 * 8
    # one block, 4 steps: 4 splits of one step
    assert L.ne_circconv_workspace(1000, 3, 1) == 4 * 3 * 1024 * 8
    # staged with 11 streams: two groups of workgroups per block
    assert L.ne_circconv_workspace(1000, 11, 0) == 4 * 11 * 1024 * 8
    # a single step (N <= 256) is never split; invalid sizes report 0
    assert L.ne_circconv_workspace(200, 3, 1) == 0
    assert L.ne_circconv_workspace(0, 3, 1) == 0 and L.ne_circconv_workspace(10, 2, 1) == 0
    p = ne.ne_params_default(3)
    need = L.ne_circconv_workspace(1000, 3, 1)
    c, g, d, ws = (ctypes.c_void_p(a) for a in (1 << 20, 2 << 20, 3 << 20, 4 << 20))
    rc = L.ne_circconv_fused(c, 8, 11, g, d, 8, None, None, 1000, ctypes.byref(p), ws, need - 8,
                             None)
    assert rc == -1
    rc = L.ne_circconv_fused(c, 8, 11, g, d, 8, None, None, 1000, ctypes.byref(p), d, need, None)
    assert rc == -3  # overlaps d_hat
    rc = L.ne_lsb_circconv(c, 40, g, d, 1000, ctypes.byref(p), ws, need - 8, None)
    assert rc == -1


def test_permute_workspace_size_and_rejection(ne):
    L = ne.lib()
    assert L.ne_permute_workspace(1000, 3, 1) == 1000 * 8       # 3 int8 inputs -> one word
    assert L.ne_permute_workspace(1000, 9, 1) == 1000 * 16
    assert L.ne_permute_workspace(1000, 5, 4) == 1000 * 24      # 20 bytes -> three words
    assert L.ne_permute_workspace(1000, 3, 8) == 1000 * 24
    assert L.ne_permute_workspace(0, 3, 1) == 0 and L.ne_permute_workspace(10, 3, 2) == 0
    p = ne.ne_params_default(3)
    c, perm, d, ws = (ctypes.c_void_p(a) for a in (1 << 20, 2 << 20, 3 << 20, 4 << 20))
    rc = L.ne_permute_scale_fused(c, 1, perm, None, None, d, 8, None, None, 1000, ctypes.byref(p),
                                  ws, 1000 * 8 - 8, None)
    assert rc == -1
    rc = L.ne_permute_scale_fused(c, 1, perm, None, None, d, 8, None, None, 1000, ctypes.byref(p),
                                  c, 1000 * 8, None)
    assert rc == -3  # overlaps the inputs


def test_series_range_matches_oracle(ne, orc):
    """ne_series_range composes the a-priori bound exactly as the oracle's
    series bound, reports NE_ERANGE exactly when it exceeds D, and gives
    eps_bits that hold the entangled words entering every operation."""
    G_, C_, S_, P_ = ne.NE_SERIES_GEMM, ne.NE_SERIES_CONV, ne.NE_SERIES_SCALE_ADD, ne.NE_SERIES_PERMUTE
    cases = [
        (127, [(G_, 4096, 127), (S_, 3, 1000), (P_, 0, 0)]),
        (127, [(G_, 64, 128), (P_, 0, 0), (C_, 16, 64), (S_, 1, 5)]),
        (1024, [(C_, 16384, 64)]),
        (5, [(S_, 1, 0), (P_, 0, 0)]),
        (127, [(G_, 4096, 127), (G_, 4096, 127)]),   # far beyond D: words wrap
        (0, [(G_, 10, 10)]),
        (127, []),
    ]
    kind = {G_: "gemm", C_: "conv", S_: "scale_add"}
    for M in (3, 4, 8):
        p = ne.ne_params_default(M)
        D = ne.ne_range_bound(p)
        for c_max, ops in cases:
            oops = [(kind[k], a, b) if k != P_ else ("permute",) for k, a, b in ops]
            bits, out_max, ok = ne.ne_series_range(p, c_max, ops)
            B = orc.series_bound(c_max, oops)
            assert out_max == min(B, 2**63 - 1)
            assert ok == (B <= D)
            for i in range(len(ops)):
                e = (2**p.l + 1) * orc.series_bound(c_max, oops[:i])
                want = min(64, e.bit_length() + 1)
                assert bits[i] == want, (M, c_max, ops, i)
                assert bits[i] == 64 or e < 2 ** (bits[i] - 1)


def test_series_argument_errors(ne):
    L = ne.lib()
    p = ne.ne_params_default(4)
    ops = (ne._SeriesOp * 1)()
    ops[0].kind, ops[0].length, ops[0].operand_max = 7, 1, 1
    assert L.ne_series_range(ctypes.byref(p), 1, 1, ops, None, None) == ne.NE_EINVAL
    ops[0].kind, ops[0].length = ne.NE_SERIES_GEMM, -1
    assert L.ne_series_range(ctypes.byref(p), 1, 1, ops, None, None) == ne.NE_EINVAL
    assert L.ne_series_range(ctypes.byref(p), -1, 0, None, None, None) == ne.NE_EINVAL
    assert L.ne_series_range(ctypes.byref(p), 1, 1, None, None, None) == ne.NE_EINVAL
    assert L.ne_series_range(ctypes.byref(p), 1, 0, None, None, None) == ne.NE_OK
    assert ne.ne_series_workspace(4096, 4096, 4) == 4096 * 4096 * 4 * 8
    assert ne.ne_series_workspace(4, 4, 9) == 0 and ne.ne_series_workspace(-1, 4, 4) == 0
    # fused series: range, sizes and workspace rejected before any launch
    fake = ctypes.c_void_p(1 << 20)
    D = ne.ne_range_bound(p)  # 2^47 - 2^31 at M = 4
    K = 4096
    s_ok = D // (K * 128 * 128)
    args = lambda smax, amax, n, Kk, N, ws, wsb: L.ne_series_gemm_scale_permute(
        fake, fake, fake, fake, fake, smax, amax, fake, ne.NE_I32, None, None, n, Kk, N,
        ctypes.byref(p), ws, wsb, None)
    assert args(s_ok + 1, 0, 64, K, 64, fake, 1 << 30) == ne.NE_ERANGE
    assert args(1, D + 1, 64, K, 64, fake, 1 << 30) == ne.NE_ERANGE
    assert args(-1, 0, 64, K, 64, fake, 1 << 30) == ne.NE_EINVAL
    assert args(1, 0, 1 << 16, K, 1 << 16, fake, 1 << 62) == ne.NE_EINVAL  # n N > 2^31 - 1
    assert args(1, 0, 64, K, 64, None, 1 << 30) == ne.NE_EINVAL
    assert args(1, 0, 64, K, 64, fake, 64 * 64 * 4 * 8 - 1) == ne.NE_EINVAL
    assert args(1, 0, 64, K, 64, ctypes.c_void_p((1 << 20) + 8), 1 << 30) in (ne.NE_EALIAS,
                                                                              ne.NE_EALIGN)
    assert args(1, 0, 0, K, 64, None, 0) == ne.NE_OK


def test_linconv_argument_errors(ne):
    """Sizes and ranges of the linear convolution are rejected before any
    launch."""
    L_ = ne.lib()
    p = ne.ne_params_default(4)
    fake = ctypes.c_void_p(1 << 20)
    fused = lambda N, L, bits: L_.ne_linconv_fused(fake, ne.NE_I32, bits, fake, L, fake,
                                                   ne.NE_I64, None, None, N, ctypes.byref(p), None,
                                                   0, None)
    staged = lambda N, L: L_.ne_lsb_linconv(fake, 40, fake, L, fake, N, ctypes.byref(p), None, 0,
                                            None)
    for N, L in [(0, 5), (5, 0), (-1, 5), (10, 131072), ((1 << 30) - 100, 200)]:
        assert fused(N, L, 15) == ne.NE_EINVAL, (N, L)
        assert staged(N, L) == ne.NE_EINVAL, (N, L)
    assert fused(1000, 100, 33) == ne.NE_EINVAL        # more bits than int32 holds
    assert fused(1000, 4500, 30) == ne.NE_ERANGE       # 4500 * 2^29 * 128 > D at M = 4
    assert fused(1000, 100, 15) == ne.NE_EALIAS        # everything at one address
    assert staged(1000, 100) == ne.NE_EALIAS


def test_linconv_workspace(ne):
    """Workspace size of the plane-staged linear convolution, and its
    argument errors (all raised before any launch)."""
    L_ = ne.lib()
    pad = lambda L: (L + 2048 + 3) // 4 * 4 + 3
    plane = lambda N, L: (N + 2 * pad(L) + 8 + 3) // 4 * 4
    taps = lambda L: (L + 1024 + 15) // 16 * 16
    # fused, c_bits 15: two digits; staged, eps_bits 40: six digits
    assert L_.ne_linconv_workspace(1000, 100, 4, 15, 1) == 4 * 2 * plane(1000, 100) + taps(100)
    assert L_.ne_linconv_workspace(1000, 100, 4, 8, 1) == 4 * 1 * plane(1000, 100) + taps(100)
    assert L_.ne_linconv_workspace(1000, 100, 4, 8, 0) == 4 * 2 * plane(1000, 100) + taps(100)
    assert L_.ne_linconv_workspace(10**6, 4500, 16, 40, 0) == 16 * 6 * plane(10**6, 4500) + taps(4500)
    for args in [(0, 5, 4, 15, 1), (5, 0, 4, 15, 1), (10, 5, 2, 15, 1), (10, 5, 9, 15, 1),
                 (10, 5, 4, 0, 0), (10, 5, 4, 65, 0), (10, 131072, 4, 15, 1)]:
        assert L_.ne_linconv_workspace(*args) == 0, args
    p = ne.ne_params_default(4)
    c, g, d = (ctypes.c_void_p(a << 20) for a in (1, 2, 3))
    need = L_.ne_linconv_workspace(1000, 100, 4, 15, 1)
    fused = lambda ws, nb: L_.ne_linconv_fused(c, ne.NE_I32, 15, g, 100, d, ne.NE_I64, None, None,
                                               1000, ctypes.byref(p), ctypes.c_void_p(ws), nb, None)
    assert fused(64 << 20, need - 1) == ne.NE_EINVAL          # too small
    assert fused(3 << 20, need) == ne.NE_EALIAS               # on top of d_hat
    assert fused((64 << 20) + 8, need) == ne.NE_EALIGN        # not 16-byte aligned
    needs = L_.ne_linconv_workspace(1000, 100, 4, 40, 0)
    staged = lambda ws, nb: L_.ne_lsb_linconv(c, 40, g, 100, d, 1000, ctypes.byref(p),
                                              ctypes.c_void_p(ws), nb, None)
    assert staged(64 << 20, needs - 1) == ne.NE_EINVAL
    assert staged(1 << 20, needs) == ne.NE_EALIAS             # on top of eps
    assert staged((64 << 20) + 4, needs) == ne.NE_EALIGN


def test_abft_rc_arguments(ne):
    """Workspace size and argument errors of the row/column checksum ABFT
    (all raised before any launch)."""
    L_ = ne.lib()
    assert L_.ne_abft_rc_workspace(4, 2000, 1200) == (5 * 2000 * 4 + 15) // 16 * 16 + 4 * 1200 * 8
    assert L_.ne_abft_rc_workspace(1, 1, 1) == 16 + 8
    for args in [(0, 10, 10), (4097, 10, 10), (4, 0, 10), (4, 131072, 10), (4, 10, 0),
                 (4, 10, (1 << 20) + 1)]:
        assert L_.ne_abft_rc_workspace(*args) == 0, args
    c, g, d, ws = (ctypes.c_void_p(a << 24) for a in (1, 2, 3, 4))
    need = L_.ne_abft_rc_workspace(4, 100, 60)
    f = lambda c_, d_, ws_, nb=need, rf=None, M=4, n=50, K=100, N=60: L_.ne_abft_rc_gemm_i8(
        c_, g, d_, rf, None, None, M, n, K, N, ws_, nb, None)
    assert f(c, d, ws, nb=need - 1) == ne.NE_EINVAL          # workspace too small
    assert f(c, d, None) == ne.NE_EINVAL                     # workspace required
    assert f(c, d, ws, M=0) == ne.NE_EINVAL
    assert f(c, d, ws, n=(1 << 20) + 1) == ne.NE_EINVAL
    assert f(c, d, ws, K=131072) == ne.NE_EINVAL
    assert f(c, c, ws) == ne.NE_EALIAS                       # d on top of c
    assert f(c, d, d) == ne.NE_EALIAS                        # workspace on top of d
    assert f(c, d, ctypes.c_void_p((4 << 24) + 8)) == ne.NE_EALIGN
    assert f(c, d, ws, rf=ctypes.c_void_p((5 << 24) + 2)) == ne.NE_EALIGN
    assert L_.ne_abft_rc_check_i8(c, g, d, ctypes.c_void_p(3 << 24), None, None, 4, 50, 100, 60,
                                  ws, need, None) == ne.NE_EALIAS   # flags on top of d
