"""GPU parity of the row/column checksum ABFT baseline (the RC-check of the
paper's GEMM comparison) against the CPU oracle: the product bit for bit,
and every row and column flag, on clean products and on products with
injected wrong positions."""
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


def _bits(words, count):
    w = np.asarray(words).astype(np.int64) & 0xFFFFFFFF
    bits = (w[..., None] >> np.arange(32)) & 1
    return bits.reshape(*w.shape[:-1], -1)[..., :count].astype(bool)


def _inputs(seed, M, n, K, N):
    c = ne_synth.uniform_int(seed, 1, (M, n, K), -128, 128).astype(np.int8)
    G = ne_synth.uniform_int(seed, 2, (K, N), -128, 128).astype(np.int8)
    return c, G


# (M, n, K, N): single elements; ragged sizes over several tiles and
# checksum chunks; the paper's 2000 x K by K x 1200 subblocks at K = 200;
# one subblock.
CASES = [(1, 1, 1, 1), (3, 70, 272, 300), (2, 257, 33, 65), (5, 64, 1000, 96), (4, 2000, 200, 1200),
         (1, 33, 17, 31)]


@pytest.mark.parametrize("M,n,K,N", CASES)
def test_abft_rc_clean(ne, orc, M, n, K, N):
    c, G = _inputs(4400 + M + n + K + N, M, n, K, N)
    ref = orc.abft_rc(c, G)
    d, rf, cf, nb = ne.ne_abft_rc_gemm_i8(_t(c), _t(np.ascontiguousarray(G.T)))
    assert np.array_equal(d.cpu().numpy(), ref["d"])
    assert not _bits(rf.cpu().numpy(), n).any() and not _bits(cf.cpu().numpy(), N).any()
    assert int(nb.item()) == 0


@pytest.mark.parametrize("M,n,K,N", [(3, 70, 272, 300), (4, 130, 64, 200), (2, 2000, 200, 1200)])
def test_abft_rc_injected(ne, orc, M, n, K, N):
    """One to three wrong positions in some subblocks and a +-e rectangle in
    another: the check-only entry flags exactly the oracle's rows and
    columns (a reused workspace and flag buffers with garbage contents)."""
    c, G = _inputs(4500 + M + n, M, n, K, N)
    c_d, gt_d = _t(c), _t(np.ascontiguousarray(G.T))
    d, rf, cf, nb = ne.ne_abft_rc_gemm_i8(c_d, gt_d)
    ws = torch.full((ne.ne_abft_rc_workspace(M, K, N) // 8 + 2,), -1, dtype=torch.int64,
                    device=DEV)
    host = d.cpu().numpy()
    rng = np.random.default_rng(M * 100 + n)
    for trial in range(4):
        bad = host.copy()
        for m in range(M):
            kind = (m + trial) % 4
            if kind == 3 and n >= 2 and N >= 2:
                i0, i1 = rng.choice(n, 2, replace=False)
                p0, p1 = rng.choice(N, 2, replace=False)
                e = int(rng.integers(1, 1000))
                bad[m, i0, p0] += e
                bad[m, i0, p1] -= e
                bad[m, i1, p0] -= e
                bad[m, i1, p1] += e
            elif kind > 0:
                for q in rng.choice(n * N, kind, replace=False):
                    bad[m, q // N, q % N] ^= 1 << int(rng.integers(31))
        ref = orc.abft_rc(c, G, bad)
        rf.fill_(-1)
        cf.fill_(-1)
        nb.zero_()
        rf2, cf2, nb2 = ne.ne_abft_rc_check_i8(c_d, gt_d, _t(bad), rf, cf, nb, workspace=ws)
        assert np.array_equal(_bits(rf2.cpu().numpy(), n), ref["row_bad"]), trial
        assert np.array_equal(_bits(cf2.cpu().numpy(), N), ref["col_bad"]), trial
        assert int(nb2.item()) == ref["n_bad"], trial


def test_abft_rc_full_size_sampled(ne, orc):
    """The paper's largest subblock product, 2000 x 2000 by 2000 x 1200, M = 4:
    no flags on the clean product, sampled outputs against the oracle's dot
    products one at a time, and one wrong position located."""
    M, n, K, N = 4, 2000, 2000, 1200
    c, G = _inputs(4600, M, n, K, N)
    c_d, gt_d = _t(c), _t(np.ascontiguousarray(G.T))
    d, rf, cf, nb = ne.ne_abft_rc_gemm_i8(c_d, gt_d)
    assert int(nb.item()) == 0
    rng = np.random.default_rng(9)
    c64, G64 = c.astype(np.int64), G.astype(np.int64)
    for _ in range(24):
        m, i, p = int(rng.integers(M)), int(rng.integers(n)), int(rng.integers(N))
        want = orc.gemm(c64[m, i][None, :], G64[:, p][:, None])[0, 0]
        assert int(d[m, i, p].item()) == want, (m, i, p)
    d[2, 1234, 777] += 1
    rf2, cf2, nb2 = ne.ne_abft_rc_check_i8(c_d, gt_d, d)
    assert np.nonzero(_bits(rf2.cpu().numpy(), n))[0].tolist() == [2]
    assert np.nonzero(_bits(rf2.cpu().numpy(), n)[2])[0].tolist() == [1234]
    assert np.nonzero(_bits(cf2.cpu().numpy(), N)[2])[0].tolist() == [777]
    assert int(nb2.item()) == 2
