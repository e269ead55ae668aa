"""GPU parity: every entry point of the C ABI against the CPU oracle, bit for bit.

Inputs come from ne_synth (seeded); expected values only from oracle/.
Sizes span several tiles and ragged tails; edge cases cover empty inputs,
K not a multiple of 16 (the unaligned load path), every check stream r,
and arbitrary (corrupted) 64-bit words.
"""
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
    """Unpack int32 bitmask words (last axis) into `count` booleans."""
    w = np.asarray(words).astype(np.int64) & 0xFFFFFFFF
    bits = (w[..., None] >> np.arange(32)) & 1
    return bits.reshape(*w.shape[:-1], -1)[..., :count].astype(bool)


def _rand_words(seed, shape):
    raw = ne_synth.raw_u64(ne_synth.stream_key(seed, 99), int(np.prod(shape)))
    w = raw.view(np.int64).reshape(shape).copy()
    flat = w.reshape(-1)
    # some magnitudes small, some extreme values
    flat[::7] >>= 40
    flat[:5] = [np.iinfo(np.int64).min, np.iinfo(np.int64).max, 0, -1, 1]
    return w


# ----------------------------------------------------------- element-wise

@pytest.mark.parametrize("M", [3, 4, 5, 8, 16])
@pytest.mark.parametrize("dtype", [np.int8, np.int32, np.int64])
def test_entangle(ne, orc, M, dtype):
    p = ne.ne_params_default(M)
    for N in (0, 1, 1000, 65536 + 17):
        info = np.iinfo(dtype)
        lo, hi = (max(info.min, -(1 << 31)), min(info.max, (1 << 31) - 1))
        c = ne_synth.uniform_int(100 + M + N, 1, (M, N), lo, hi + 1, dtype=dtype)
        ref = orc.entangle(c.astype(np.int64), 64, p.l)
        got = ne.ne_entangle(_t(c), p)
        assert np.array_equal(_h(got), ref), (M, N, dtype)
        if dtype == np.int64 and N:
            buf = _t(c)
            ne.ne_entangle(buf, p, out=buf)  # in place
            assert np.array_equal(_h(buf), ref)


@pytest.mark.parametrize("M", [3, 4, 5, 7, 8, 11, 16])
def test_disentangle_check_arbitrary_words(ne, orc, M):
    """Any 64-bit words (corrupted or not), every r: d_hat, flags, n_bad."""
    p = ne.ne_params_default(M)
    N = 4099
    delta = _rand_words(200 + M, (M, N))
    for r in range(M):
        p.r_check = r
        dh_o, fl_o, bad_o = orc.extract_check(delta, 64, p.l, r)
        dh, fl, nb = ne.ne_disentangle_check(_t(delta), p)
        assert np.array_equal(_h(dh), dh_o), r
        assert np.array_equal(_bits(_h(fl), N), fl_o.astype(bool)), r
        assert int(nb.item()) == bad_o


@pytest.mark.parametrize("M", [3, 4, 6, 8])
def test_disentangle_check_codewords_in_place(ne, orc, M):
    """Entangled in-range data (storage-only use, op = x with g = 1): exact
    round trip, nothing flagged, computed in place."""
    p = ne.ne_params_default(M)
    D = orc.range_bound(M, p.l, p.k)
    N = 70001
    c = ne_synth.uniform_int(300 + M, 1, (M, N), -(1 << 31), 1 << 31)
    c[:, 0] = D
    c[:, 1] = -D
    delta = _t(orc.entangle(c, 64, p.l))
    dh, fl, nb = ne.ne_disentangle_check(delta, p, out=delta)
    assert np.array_equal(_h(dh), c) and int(nb.item()) == 0
    assert not _bits(_h(fl), N).any()


def test_disentangle_check_empty(ne):
    p = ne.ne_params_default(3)
    d = torch.empty((3, 0), dtype=torch.int64, device=DEV)
    dh, fl, nb = ne.ne_disentangle_check(d, p)
    assert dh.shape == (3, 0) and int(nb.item()) == 0


@pytest.mark.parametrize("M", [3, 4, 5, 8, 16])
def test_recover_every_lost_stream(ne, orc, M):
    p = ne.ne_params_default(M)
    N = 5000
    D = orc.range_bound(M, p.l, p.k)
    lim = min(D, (1 << 31) - 1)
    c = ne_synth.uniform_int(400 + M, 1, (M, N), -lim, lim + 1)
    delta = orc.entangle(c, 64, p.l)
    dd = [_t(delta[m]) for m in range(M)]
    for lost in range(M):
        streams = [None if m == lost else dd[m] for m in range(M)]
        dh, rb = ne.ne_recover(streams, lost, p, rebuild=True)
        assert np.array_equal(_h(dh), c), lost
        assert np.array_equal(_h(rb), delta[lost]), lost
        # arbitrary words: the recovery equals the oracle's extraction without `lost`
    w = _rand_words(401 + M, (M, N))
    for lost in range(M):
        streams = [None if m == lost else _t(w[m]) for m in range(M)]
        dh, _ = ne.ne_recover(streams, lost, p)
        assert np.array_equal(_h(dh), orc.recover(w, lost, 64, p.l)), lost


@pytest.mark.parametrize("M", [3, 5, 8])
def test_permute_scale(ne, orc, M):
    p = ne.ne_params_default(M)
    for N in (1, 777, 100003):
        c, perm, s, a = ne_synth.perm_scale_streams(500 + M + N, M, N, -128, 128)
        eps = orc.entangle(c, 64, p.l)
        a_ent = orc.self_entangle(a, 64, p.l)
        ref = np.stack([orc.permute_scale(eps[m], perm, s, a_ent) for m in range(M)])
        got = ne.ne_lsb_permute_scale(_t(eps), _t(perm.astype(np.int32)), _t(s), _t(a), p)
        assert np.array_equal(_h(got), ref)
        ref2 = np.stack([orc.permute_scale(eps[m], perm, None, None) for m in range(M)])
        got2 = ne.ne_lsb_permute_scale(_t(eps), _t(perm.astype(np.int32)), None, None, p)
        assert np.array_equal(_h(got2), ref2)
        # end to end: extraction gives the plain permuted/scaled/shifted streams
        dh, fl, nb = ne.ne_disentangle_check(got, p)
        assert np.array_equal(_h(dh), c[:, perm] * s[None] + a[None]) and int(nb.item()) == 0


# ----------------------------------------------------------- staged GEMM

# K: multiples of 16 (16-byte rows), of 8 (200) and of 4 only (100, 36),
# and odd (17, 1): every load path of the operand rows
GEMM_SHAPES = [(3, 64, 64, 64), (4, 100, 200, 300), (3, 33, 48, 45), (5, 7, 17, 129),
               (4, 1, 1, 1), (8, 70, 96, 200), (3, 50, 100, 70)]


@pytest.mark.parametrize("M,n,K,N", GEMM_SHAPES)
def test_lsb_gemm_on_entangled_words(ne, orc, M, n, K, N):
    p = ne.ne_params_default(M)
    c, G = ne_synth.gemm_streams(600 + n + K, M, n, K, N, -128, 128)
    eps = orc.entangle(c.astype(np.int64), 64, p.l)
    ref = orc.gemm(eps.reshape(M * n, K), G).reshape(M, n, N)
    bits = int(np.abs(eps).max()).bit_length() + 1
    Gt = _t(np.ascontiguousarray(G.T))
    for eb in (bits, 64):
        got = ne.ne_lsb_gemm(_t(eps), eb, Gt, p)
        assert np.array_equal(_h(got), ref), eb
    dh, fl, nb = ne.ne_disentangle_check(got, p)
    plain = np.einsum("mik,kj->mij", c.astype(np.int64), G.astype(np.int64))
    assert np.array_equal(_h(dh), plain) and int(nb.item()) == 0


@pytest.mark.parametrize("digits_bits", [8, 16, 24, 40, 56, 64])
def test_lsb_gemm_any_words_mod_2_64(ne, orc, digits_bits):
    """The unaware routine is exact modulo 2^64 for any words within eps_bits."""
    M, n, K, N = 3, 40, 80, 70
    p = ne.ne_params_default(M)
    w = _rand_words(700 + digits_bits, (M, n, K))
    if digits_bits < 64:
        w = w >> (64 - digits_bits)
    G = ne_synth.uniform_int(701, 2, (K, N), -128, 128, dtype=np.int8)
    ref = orc.gemm(w.reshape(M * n, K), G).reshape(M, n, N)
    got = ne.ne_lsb_gemm(_t(w), digits_bits, _t(np.ascontiguousarray(G.T)), p)
    assert np.array_equal(_h(got), ref)


@pytest.mark.parametrize("N", [1, 5, 300, 2049])
def test_circconv_on_entangled_words(ne, orc, N):
    M = 3
    p = ne.ne_params_default(M)
    c, g = ne_synth.conv_streams(800 + N, M, N, -1024, 1024, -64, 64)
    eps = orc.entangle(c, 64, p.l)
    ref = np.stack([orc.circconv(eps[m], g.astype(np.int64)) for m in range(M)])
    bits = int(np.abs(eps).max()).bit_length() + 1
    got = ne.ne_lsb_circconv(_t(eps), bits, _t(g), p)
    assert np.array_equal(_h(got), ref)
    dh, fl, nb = ne.ne_disentangle_check(got, p)
    plain = np.stack([orc.circconv(c[m], g.astype(np.int64)) for m in range(M)])
    assert np.array_equal(_h(dh), plain) and int(nb.item()) == 0


@pytest.mark.parametrize("M,N,bits", [(3, 1100, 64), (11, 700, 40), (4, 33, 9)])
def test_circconv_any_words(ne, orc, M, N, bits):
    """Staged convolution of arbitrary words (every digit count, more streams
    than one workgroup takes, ragged blocks) against the oracle, mod 2^64."""
    p = ne.ne_params_default(M)
    raw = ne_synth.raw_u64(ne_synth.stream_key(850 + M + N, 1), M * N).view(np.int64)
    x = (raw >> np.int64(64 - bits)).reshape(M, N)  # uniform in [-2^(bits-1), 2^(bits-1))
    g = ne_synth.uniform_int(850 + M + N, 3, (N,), -128, 128).astype(np.int8)
    ref = np.stack([orc.circconv(x[m], g.astype(np.int64)) for m in range(M)])
    for ws in (True, None):  # split taps over workgroups, and one workgroup per block
        got = ne.ne_lsb_circconv(_t(x), bits, _t(g), p, workspace=ws)
        assert np.array_equal(_h(got), ref), ws


# ------------------------------------------------------------- fused GEMM

FUSED = [(3, 64, 64, 64), (4, 100, 200, 300), (4, 33, 17, 45), (3, 65, 130, 257),
         (5, 40, 64, 100), (6, 31, 96, 64), (7, 20, 48, 40), (8, 50, 64, 130), (4, 1, 16, 1),
         (4, 70, 100, 90), (3, 40, 36, 33)]


@pytest.mark.parametrize("M,n,K,N", FUSED)
def test_fused_gemm_matches_oracle(ne, orc, M, n, K, N):
    c, G = ne_synth.gemm_streams(900 + M * n + K, M, n, K, N, -128, 128)
    Gt = _t(np.ascontiguousarray(G.T))
    cd = _t(c)
    p = ne.ne_params_default(M)
    for r in range(M):
        p.r_check = r
        ref = orc.gemm_pipeline(c, G, r=r)
        for dt in (torch.int32, torch.int64):
            dh, fl, nb = ne.ne_gemm_fused(cd, Gt, p, out_dtype=dt)
            exp = ref["dhat"] if dt == torch.int64 else ref["dhat"].astype(np.int32)
            assert np.array_equal(_h(dh), exp), (r, dt)
            assert int(nb.item()) == 0
            assert not _bits(_h(fl), N).any()


@pytest.mark.parametrize("M", [3, 4, 5, 8])
def test_fused_gemm_injected_faults(ne, orc, M):
    """Faults XOR-ed into one stream's entangled outputs: d_hat and flags equal
    the oracle's on the same corrupted words, and every fault is flagged."""
    n, K, N = 96, 64, 160
    c, G = ne_synth.gemm_streams(1000 + M, M, n, K, N, -128, 128)
    p = ne.ne_params_default(M)
    ref = orc.gemm_pipeline(c, G)
    F = 300
    pos = ne_synth.uniform_int(1001, 1, (F,), 0, n * N)
    pos = np.unique(pos)
    st = ne_synth.uniform_int(1001, 2, (pos.size,), 0, M)
    bit = ne_synth.uniform_int(1001, 3, (pos.size,), 0, 64)
    mask = (np.ones(pos.size, dtype=np.uint64) << bit.astype(np.uint64)).view(np.int64)
    delta = ref["delta"].reshape(M, -1).copy()
    for q, s, m in zip(pos, st, mask):
        delta[s, q] ^= m
    dh_o, fl_o, bad_o = orc.extract_check(delta, 64, p.l, 0)
    inj = ne.Inject(_t(pos), _t(st.astype(np.int32)), _t(mask))
    dh, fl, nb = ne.ne_gemm_fused(_t(c), _t(np.ascontiguousarray(G.T)), p, out_dtype=torch.int64,
                                  inject=inj)
    assert np.array_equal(_h(dh).reshape(M, -1), dh_o)
    got_flags = _bits(_h(fl), N).reshape(-1)
    assert np.array_equal(got_flags, fl_o.astype(bool))
    assert int(nb.item()) == bad_o == pos.size
    assert got_flags[pos].all()


def test_fused_gemm_range_and_errors(ne):
    p = ne.ne_params_default(4)
    c = torch.zeros((4, 2, 16), dtype=torch.int8, device=DEV)
    Gt = torch.zeros((3, 16), dtype=torch.int8, device=DEV)
    p.r_check = 4
    with pytest.raises(ne.NEError):
        ne.ne_gemm_fused(c, Gt, p)
    p.r_check = 0
    dh, fl, nb = ne.ne_gemm_fused(torch.zeros((4, 0, 16), dtype=torch.int8, device=DEV), Gt, p)
    assert dh.shape == (4, 0, 3)
    dh, fl, nb = ne.ne_gemm_fused(torch.zeros((4, 2, 0), dtype=torch.int8, device=DEV),
                                  torch.zeros((3, 0), dtype=torch.int8, device=DEV), p)
    assert int(dh.abs().sum().item()) == 0 and int(nb.item()) == 0


# --------------------------------------------------------------- baselines

@pytest.mark.parametrize("R,K,N", [(256, 128, 128), (300, 200, 130), (17, 33, 5), (1024, 512, 384),
                                   (90, 100, 70), (40, 36, 50)])
def test_plain_gemm(ne, R, K, N):
    A = ne_synth.uniform_int(1100 + R, 1, (R, K), -128, 128, dtype=np.int8)
    B = ne_synth.uniform_int(1100 + R, 2, (K, N), -128, 128, dtype=np.int8)
    ref = A.astype(np.int64) @ B.astype(np.int64)
    got = ne.ne_plain_gemm_i8(_t(A), _t(np.ascontiguousarray(B.T)))
    assert np.array_equal(_h(got).astype(np.int64), ref)


@pytest.mark.parametrize("M,n,K,N", [(4, 64, 128, 128), (3, 33, 17, 45), (8, 40, 64, 100),
                                     (4, 70, 272, 300), (1, 5, 16, 7), (3, 30, 100, 40),
                                     (2, 20, 200, 24)])
def test_abft_gemm(ne, orc, M, n, K, N):
    c, G = ne_synth.gemm_streams(1200 + M, M, n, K, N, -128, 128)
    c64 = c.astype(np.int64)
    plain = np.stack([c64[m] @ G.astype(np.int64) for m in range(M)])
    e = orc.gemm(orc.abft_checksum(c64), G)
    flags_o, bad_o = orc.abft_check(plain, e)
    assert bad_o == 0
    # checksum planes + DMA pipeline (used when K % 16 == 0), and one launch
    for ws in (True, None):
        d, fl, nb = ne.ne_abft_gemm_i8(_t(c), _t(np.ascontiguousarray(G.T)), workspace=ws)
        assert np.array_equal(_h(d).astype(np.int64), plain), ws
        assert int(nb.item()) == 0 and not _bits(_h(fl), N).any(), ws


# ---------------------------------------------- fault trials (small GEMM)

def test_bit_flip_trials_staged_path(ne, orc):
    """M = 3 streams of 64x64 times a shared 64x64 operand (values in
    [-2^7, 2^7)), entangled, multiplied, checked; then 1000 trials each
    flipping one random bit of one random entangled output word: every trial
    is flagged at exactly that position, and d_hat matches the oracle."""
    M, n, K, N = 3, 64, 64, 64
    seed = ne_synth.BASE_SEED + 0
    c, G = ne_synth.gemm_streams(seed, M, n, K, N, -128, 128)
    p = ne.ne_params_default(M)
    eps = ne.ne_entangle(_t(c), p)
    delta = ne.ne_lsb_gemm(eps.reshape(M, n, K), 32, _t(np.ascontiguousarray(G.T)), p)
    ref = orc.gemm_pipeline(c, G)
    assert np.array_equal(_h(delta), ref["delta"])
    dh, fl, nb = ne.ne_disentangle_check(delta, p)
    assert np.array_equal(_h(dh), ref["dhat"]) and int(nb.item()) == 0
    streams, positions, bits = ne_synth.bit_flip_trials(seed, 1000, M, n * N)
    flat = delta.reshape(M, -1)
    detected = 0
    for s, q, b in zip(streams, positions, bits):
        orig = flat[s, q].clone()
        flat[s, q] = orig ^ torch.tensor(np.int64(np.uint64(1) << np.uint64(b)).item(), device=DEV)
        _, fl, nb = ne.ne_disentangle_check(delta, p)
        f = _bits(_h(fl), n * N)
        detected += int(nb.item() == 1 and f[q] and f.sum() == 1)
        flat[s, q] = orig
    assert detected == 1000
