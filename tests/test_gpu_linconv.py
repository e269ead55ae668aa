"""GPU parity of the linear convolution of long streams with short kernels
(fused with entanglement, disentanglement and the check; and staged, on
entangled words) against the CPU oracle, bit for bit.  Every case runs both
ways of staging the operands: from the inputs directly (ws False) and from
the digit planes of the pre-pass (ws True, a workspace whose contents on
entry are garbage)."""
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


def _ws(ne, ws, N, L, M, bits, fused):
    """False, or a workspace of the asked size filled with garbage."""
    if not ws:
        return False
    need = ne.ne_linconv_workspace(N, L, M, bits, fused)
    assert need > 0
    return torch.full(((need + 7) // 8,), 0x5A5A5A5A5A5A5A5A, dtype=torch.int64,
                      device=DEV)


WS = pytest.mark.parametrize("ws", [False, True], ids=["direct", "planes"])


def _inputs(seed, M, nx, L, bits=15):
    c = ne_synth.uniform_int(seed, 1, (M, nx), -(1 << (bits - 1)), 1 << (bits - 1))
    g = ne_synth.uniform_int(seed, 2, (L,), -128, 128).astype(np.int8)
    return c, g


# (M, samples, taps): one block; several blocks in one 256-tap step; L + 32
# exactly one step and one past it; several steps staged at once; sliding
# steps; a kernel longer than the stream; a single tap and a single sample.
CASES = [(3, 100, 7), (4, 3000, 300), (6, 1500, 224), (7, 1024, 225), (8, 5000, 1100),
         (3, 20000, 4500), (5, 700, 2500), (3, 1, 1), (4, 2049, 1)]


@WS
@pytest.mark.parametrize("M,nx,L", CASES)
def test_linconv_fused(ne, orc, M, nx, L, ws):
    c, g = _inputs(2700 + M + nx + L, M, nx, L)
    p = ne.ne_params_default(M)
    no = nx + L - 1
    for r in sorted({0, M - 1}):
        p.r_check = r
        ref = orc.linconv_pipeline(c, g.astype(np.int64), r=r)
        dh, fl, nb = ne.ne_linconv_fused(_t(c.astype(np.int32)), _t(g), p, c_bits=15,
                                         workspace=_ws(ne, ws, nx, L, M, 15, True))
        assert np.array_equal(_h(dh), ref["dhat"]), r
        assert int(nb.item()) == 0 and not _bits(_h(fl), no).any()
    dh32, _, _ = ne.ne_linconv_fused(_t(c), _t(g), p, c_bits=15, out_dtype=torch.int32,
                                     workspace=_ws(ne, ws, nx, L, M, 15, True))
    assert np.array_equal(_h(dh32), ref["dhat"].astype(np.int32))


@WS
@pytest.mark.parametrize("M,nx,L,cdt,bits", [(3, 900, 40, np.int8, 8), (8, 2100, 600, np.int64, 22),
                                             (5, 1300, 77, np.int32, 24)])
def test_linconv_fused_digit_counts(ne, orc, M, nx, L, cdt, bits, ws):
    """One, three and four int8 digits per input value."""
    c, g = _inputs(2750 + M, M, nx, L, bits)
    p = ne.ne_params_default(M)
    ref = orc.linconv_pipeline(c, g.astype(np.int64), r=0)
    dh, fl, nb = ne.ne_linconv_fused(_t(c.astype(cdt)), _t(g), p, c_bits=bits,
                                     workspace=_ws(ne, ws, nx, L, M, bits, True))
    assert np.array_equal(_h(dh), ref["dhat"])
    assert int(nb.item()) == 0 and not _bits(_h(fl), nx + L - 1).any()


@WS
def test_linconv_full_size_sampled(ne, orc, ws):
    """The paper's long-stream shape (10^6 samples, 4500 taps, M = 8):
    sampled outputs against the oracle's linear convolution of the samples
    that reach them, one output at a time."""
    M, nx, L = 8, 1_000_000, 4500
    c, g = _inputs(2790, M, nx, L)
    p = ne.ne_params_default(M)
    dh, fl, nb = ne.ne_linconv_fused(_t(c.astype(np.int32)), _t(g), p, c_bits=15,
                                     workspace=_ws(ne, ws, nx, L, M, 15, True))
    assert int(nb.item()) == 0
    got = _h(dh)
    no = nx + L - 1
    rng = np.random.default_rng(3)
    ts = np.concatenate([[0, 1, L - 1, L, nx - 1, nx, no - 1], rng.integers(0, no, 9)])
    g64 = g.astype(np.int64)
    for t in ts:
        lo = t - (L - 1)
        for m in range(M):
            seg = np.zeros(L, np.int64)
            a, b = max(lo, 0), min(t + 1, nx)
            seg[a - lo:b - lo] = c[m, a:b]
            want = orc.linconv(seg, g64)[L - 1]
            assert got[m, t] == want, (m, t)


@WS
@pytest.mark.parametrize("M", [3, 9, 16])
def test_linconv_staged(ne, orc, M, ws):
    """ne_lsb_linconv on entangled words (stream groups of eight above
    M = 8), then disentangle and check; a flipped bit in one stream's output
    is flagged at exactly its position."""
    nx, L = 2500, 300
    c, g = _inputs(2800 + M, M, nx, L)
    p = ne.ne_params_default(M)
    ref = orc.linconv_pipeline(c, g.astype(np.int64))
    eps = ne.ne_entangle(_t(c), p)
    bits, _, ok = ne.ne_series_range(p, 1 << 14, [(ne.NE_SERIES_CONV, L, 128)])
    assert ok
    delta = ne.ne_lsb_linconv(eps, bits[0], _t(g), p, workspace=_ws(ne, ws, nx, L, M, bits[0], False))
    assert np.array_equal(_h(delta), ref["delta"])
    dh, fl, nb = ne.ne_disentangle_check(delta, p)
    assert np.array_equal(_h(dh), ref["dhat"]) and int(nb.item()) == 0
    delta[M // 2, 1234] ^= 1 << 37
    dh, fl, nb = ne.ne_disentangle_check(delta, p)
    assert list(np.nonzero(_bits(_h(fl), nx + L - 1))[0]) == [1234] and int(nb.item()) == 1


def test_linconv_range_rejected(ne):
    p = ne.ne_params_default(3)  # D = 2^20 (2^21 - 1)
    c = torch.zeros((3, 64), dtype=torch.int32, device=DEV)
    g = torch.zeros((4500,), dtype=torch.int8, device=DEV)
    with pytest.raises(ne.NEError) as e:
        ne.ne_linconv_fused(c, g, p, c_bits=24)
    assert e.value.code == ne.NE_ERANGE


@WS
def test_linconv_fused_int32_extremes(ne, orc, ws):
    """Full-width int32 samples (c_bits = 32: five balanced digits), the
    extreme values included."""
    M, nx, L = 8, 3000, 7
    c = ne_synth.uniform_int(2850, 1, (M, nx), -(1 << 31), 1 << 31)
    c[:, :4] = [(1 << 31) - 1, -(1 << 31), -1, 0]
    g = ne_synth.uniform_int(2850, 2, (L,), -128, 128).astype(np.int8)
    g[:2] = [-128, 127]
    p = ne.ne_params_default(M)
    ref = orc.linconv_pipeline(c, g.astype(np.int64))
    dh, fl, nb = ne.ne_linconv_fused(_t(c.astype(np.int32)), _t(g), p, c_bits=32,
                                     workspace=_ws(ne, ws, nx, L, M, 32, True))
    assert np.array_equal(_h(dh), ref["dhat"])
    assert int(nb.item()) == 0 and not _bits(_h(fl), nx + L - 1).any()
