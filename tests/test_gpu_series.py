"""GPU parity of operation series on the entangled streams (several LSB
operations, one disentanglement at the end) against the CPU oracle, bit for
bit: the fused GEMM -> scale/add -> permutation entry point, and a longer
series chained from the staged entry points with the eps_bits that the range
composition gives."""
import numpy as np
import pytest
import torch

import ne_synth

pytestmark = pytest.mark.gpu

DEV = "cuda"


@pytest.fixture(scope="module")
def ne():
    import paper_1604_04740_amd as ne
    ne.lib()
    return ne


def _t(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to(DEV)


def _h(t):
    return t.cpu().numpy()


def _bits(words, count):
    w = np.asarray(words).astype(np.int64) & 0xFFFFFFFF
    bits = (w[..., None] >> np.arange(32)) & 1
    return bits.reshape(*w.shape[:-1], -1)[..., :count].astype(bool)


def _inputs(seed, M, n, K, N):
    c, G = ne_synth.gemm_streams(seed, M, n, K, N, -128, 128)
    q = n * N
    s = ne_synth.uniform_int(seed, 11, (q,), -100, 100)
    a = ne_synth.uniform_int(seed, 12, (q,), -1000, 1000)
    perm = ne_synth.permutation(seed, 13, q)
    return c, G, s, a, perm


@pytest.mark.parametrize("M,n,K,N", [(3, 33, 64, 70), (4, 64, 256, 256), (5, 100, 40, 300),
                                     (8, 31, 128, 129), (4, 1, 16, 1)])
def test_series_gemm_scale_permute(ne, orc, M, n, K, N):
    c, G, s, a, perm = _inputs(2400 + M + n, M, n, K, N)
    q = n * N
    p = ne.ne_params_default(M)
    Gt = _t(np.ascontiguousarray(G.T))
    for r in sorted({0, M - 1}):
        p.r_check = r
        ref = orc.series_pipeline(c, [("gemm", G), ("scale_add", s, a), ("permute", perm)], r=r)
        for odt in (torch.int32, torch.int64):
            dh, fl, nb = ne.ne_series_gemm_scale_permute(
                _t(c), Gt, _t(s), _t(a), _t(perm.astype(np.int32)), p, scale_max=100,
                add_max=1000, out_dtype=odt)
            want = ref["dhat"].reshape(M, q)
            if odt == torch.int32:
                want = want.astype(np.int32)
            assert np.array_equal(_h(dh), want), (r, odt)
            assert int(nb.item()) == 0 and not _bits(_h(fl), q).any()
    # no scale, no add: GEMM then permutation
    ref = orc.series_pipeline(c, [("gemm", G), ("permute", perm)], r=p.r_check)
    dh, fl, nb = ne.ne_series_gemm_scale_permute(_t(c), Gt, None, None,
                                                 _t(perm.astype(np.int32)), p,
                                                 out_dtype=torch.int64)
    assert np.array_equal(_h(dh), ref["dhat"].reshape(M, q)) and int(nb.item()) == 0


def test_series_fused_full_size_sampled(ne, orc):
    """The benchmark's shape (M = 4, 4096 x 4096 x 4096): sampled output
    positions against the oracle computed one row at a time."""
    M, n, K, N = 4, 4096, 4096, 4096
    c, G, s, a, perm = _inputs(2450, M, n, K, N)
    p = ne.ne_params_default(M)
    dh, fl, nb = ne.ne_series_gemm_scale_permute(
        _t(c), _t(np.ascontiguousarray(G.T)), _t(s), _t(a), _t(perm.astype(np.int32)), p,
        scale_max=100, add_max=1000)
    assert int(nb.item()) == 0
    rng = np.random.default_rng(5)
    qs = np.concatenate([[0, n * N - 1], rng.integers(0, n * N, 14)])
    src = perm[qs]                     # positions of the GEMM output that land at qs
    rows = np.unique(src // N)
    got = _h(dh)
    for row in rows:
        sel = qs[src // N == row]
        ref = orc.series_pipeline(c[:, row:row + 1, :], [("gemm", G)])["dhat"][:, 0, :]
        for qq in sel:
            col = perm[qq] % N
            want = s[perm[qq]] * ref[:, col] + a[perm[qq]]
            assert np.array_equal(got[:, qq].astype(np.int64), want), qq


def test_series_range_rejected(ne):
    p = ne.ne_params_default(8)  # D = 127 * 2^48 < 4096 * 128 * 128 * 2^30
    c = torch.zeros((8, 16, 4096), dtype=torch.int8, device=DEV)
    Gt = torch.zeros((32, 4096), dtype=torch.int8, device=DEV)
    sc = torch.zeros((16 * 32,), dtype=torch.int64, device=DEV)
    perm = torch.arange(16 * 32, dtype=torch.int32, device=DEV)
    with pytest.raises(ne.NEError) as e:
        ne.ne_series_gemm_scale_permute(c, Gt, sc, None, perm, p, scale_max=1 << 30)
    assert e.value.code == ne.NE_ERANGE


@pytest.mark.parametrize("M", [3, 4, 7])
def test_series_staged_chain(ne, orc, M):
    """GEMM -> permute/scale/add -> circular convolution -> disentangle, each
    step a staged entry point on entangled int64 words, the words' bit
    widths from ne_series_range; a bit flipped in one stream between two
    steps is flagged at the position the permutation moves it to."""
    n, K, N = 12, 48, 20
    q = n * N
    c, G, s, a, perm = _inputs(2500 + M, M, n, K, N)
    s = s % 7 - 3
    g = ne_synth.uniform_int(2500 + M, 14, (q,), -16, 16)
    p = ne.ne_params_default(M)
    ops = [(ne.NE_SERIES_GEMM, K, 128), (ne.NE_SERIES_PERMUTE, 0, 0),
           (ne.NE_SERIES_SCALE_ADD, 3, 1000), (ne.NE_SERIES_CONV, q, 16)]
    bits, bound, ok = ne.ne_series_range(p, 128, ops)
    assert ok and bound == ((128 * K * 128) * 3 + 1000) * q * 16
    ref = orc.series_pipeline(c, [("gemm", G), ("permute", perm), ("scale_add", s, a),
                                  ("conv", g)])
    eps = ne.ne_entangle(_t(c), p)
    d1 = ne.ne_lsb_gemm(eps, bits[0], _t(np.ascontiguousarray(G.T)), p).reshape(M, q)
    d2 = ne.ne_lsb_permute_scale(d1, _t(perm.astype(np.int32)), _t(s), _t(a), p)
    d3 = ne.ne_lsb_circconv(d2.contiguous(), bits[3], _t(g.astype(np.int8)), p)
    assert np.array_equal(_h(d3), ref["delta"].reshape(M, q))
    dh, fl, nb = ne.ne_disentangle_check(d3, p)
    assert np.array_equal(_h(dh), ref["dhat"].reshape(M, q)) and int(nb.item()) == 0
    # a fault in stream 1 after the GEMM at GEMM position x; the permutation
    # moves it to y with perm[y] = x; the element-wise check then flags y
    x = 37
    y = int(np.nonzero(perm == x)[0][0])
    d1f = d1.clone()
    d1f[1, x] ^= 1 << 20
    d2f = ne.ne_lsb_permute_scale(d1f, _t(perm.astype(np.int32)), None, None, p)
    dh, fl, nb = ne.ne_disentangle_check(d2f, p)
    flagged = np.nonzero(_bits(_h(fl), q))[0]
    assert list(flagged) == [y] and int(nb.item()) == 1
