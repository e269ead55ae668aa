"""Pins of the CPU oracle against what the paper and the mathematics fix.

None of these re-implements the oracle's own formulas: each compares it with
a value printed in the paper (Table II), a hand-worked example from the
section III-A equations, a textbook/library computation of the plain
operation (numpy matmul, numpy roll, Python integers), the paper's
properties checked exhaustively at tiny word widths (Propositions 1-4), or
the section III-A special form for M = 3.
"""
import os

import numpy as np
import pytest

import ne_synth

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")

pytestmark = pytest.mark.filterwarnings("ignore::RuntimeWarning")


def _wrap(x, w):
    """Python-int reduction to a w-bit two's-complement value."""
    x &= (1 << w) - 1
    return x - (1 << w) if x >> (w - 1) else x


def _wrap_np(x, w):
    x = np.asarray(x, dtype=np.int64).astype(np.uint64)
    if w < 64:
        x &= np.uint64((1 << w) - 1)
    s = np.uint64(1 << (w - 1))
    return ((x ^ s) - s).astype(np.int64)


def _tuples(M, D):
    vals = np.arange(-D, D + 1, dtype=np.int64)
    return np.stack(np.meshgrid(*([vals] * M), indexing="ij"), 0).reshape(M, -1)


# ----------------------------------------------------------------- params

def _table2():
    rows = []
    with open(os.path.join(GOLDEN, "table2_w32.txt")) as f:
        for line in f:
            if line.strip() and not line.startswith("#"):
                rows.append(tuple(int(v) for v in line.split()))
    return rows


def test_table2_params(orc):
    """Table II (section III-C): (l, k) and the supported width (M-2)l + k at w = 32."""
    for M, l, k, width in _table2():
        assert orc.params(M, 32) == (l, k)
        assert (M - 2) * l + k == width


def test_table2_width_matches_range_formula(orc):
    """The section III-C range D, as a signed bit width, equals Table II's
    width column for every row with l >= 2.  (For l = 1 the range formula
    gives D = 0 while the table prints 31 bits: a discrepancy in the paper.)"""
    for M, l, k, width in _table2():
        D = orc.range_bound(M, l, k)
        if l >= 2:
            assert D.bit_length() + 1 == width
        else:
            assert D == 0


def test_params_w64_fill_word(orc):
    """At w = 64 the rule has ties for M = 3 and 7; the chosen pair fills the
    word exactly and attains the maximum of (M-2)l + k over admissible pairs."""
    for M in range(3, 9):
        l, k = orc.params(M, 64)
        best = max((M - 2) * ll + min(ll, 64 - (M - 1) * ll)
                   for ll in range(1, 64) if 64 - (M - 1) * ll >= 0)
        assert (M - 2) * l + k == best
        assert (M - 1) * l + k == 64 and k <= l
        assert M * l >= 64  # needed for the any-corruption guarantee below
    assert orc.params(3, 64) == (22, 20)
    assert orc.params(4, 64) == (16, 16)


# -------------------------------------------------------- worked example

def test_worked_example_m3_w32(orc):
    vals = {}
    with open(os.path.join(GOLDEN, "worked_m3_w32.txt")) as f:
        for line in f:
            if line.strip() and not line.startswith("#"):
                key, *rest = line.split()
                vals[key] = [int(v) for v in rest]
    w, l = vals["w"][0], vals["l"][0]
    c = np.array(vals["c"], dtype=np.int64).reshape(3, 1)
    eps = orc.entangle(c, w, l)
    assert eps.ravel().tolist() == vals["eps"]
    dhat, flags, bad = orc.extract_check(eps, w, l, 0)
    assert dhat.ravel().tolist() == vals["dhat"]
    assert bad == 0 and flags.tolist() == [0]
    d3, f3, b3 = orc.extract3(eps, w, l)
    assert d3.ravel().tolist() == vals["dhat"] and b3 == 0


# ----------------------------------------- exhaustive tiny-width properties

EXH = [(8, 3), (9, 3), (10, 3), (12, 3), (8, 4), (10, 4), (12, 4), (10, 5), (12, 5)]


@pytest.mark.parametrize("w,M", EXH)
def test_exhaustive_roundtrip_and_bitflips(orc, w, M):
    """Propositions 1-4 at tiny w, exhaustively over every in-range output
    tuple (sampled, corners included, where there are too many): extraction without any stream r returns d exactly (fail-stop
    recovery), no clean position is flagged, and every single-bit flip of
    any one entangled output is flagged, from every r."""
    pairs = [(l, k) for l in range(2, w + 1) for k in range(1, l + 1)
             if (M - 1) * l + k <= w]
    tested = 0
    rng = np.random.default_rng(w * 10 + M)
    for l, k in pairs:
        D = orc.range_bound(M, l, k)
        if (2 * D + 1) ** M <= 150_000:
            d = _tuples(M, D)
        else:  # too many tuples: the corners plus a uniform sample
            corners = _tuples(M, 1) * D
            d = np.concatenate([corners, rng.integers(-D, D + 1, size=(M, 20_000))], axis=1)
        delta = orc.entangle(d, w, l)  # storage-only use: op = x, g = 1
        for r in range(M):
            dhat, flags, bad = orc.extract_check(delta, w, l, r)
            assert (dhat == d).all() and bad == 0
        for j in range(M):
            for b in range(w):
                bad_delta = delta.copy()
                bad_delta[j] = _wrap_np(bad_delta[j] ^ (1 << b), w)
                for r in range(M):
                    _, flags, bad = orc.extract_check(bad_delta, w, l, r)
                    assert bad == d.shape[1], (l, k, j, b, r)
        tested += 1
    assert tested > 0


@pytest.mark.parametrize("w,M", [(8, 3), (9, 3), (10, 3), (8, 4), (10, 4)])
def test_exhaustive_arbitrary_corruption(orc, w, M):
    """Any replacement of one entangled output word by any other w-bit value
    is flagged when M*l >= w (true for the rule's pair here), and some such
    replacement escapes when M*l < w.  Checked over every w-bit value, for a
    stride-sample of in-range tuples."""
    pairs = [(l, k) for l in range(2, w + 1) for k in range(1, l + 1)
             if (M - 1) * l + k <= w]
    vals = np.arange(-(1 << (w - 1)), 1 << (w - 1), dtype=np.int64)
    seen_cover = seen_escape = False
    rng = np.random.default_rng(w * 100 + M)
    for l, k in pairs:
        D = orc.range_bound(M, l, k)
        if (2 * D + 1) ** M <= 400_000:
            d = _tuples(M, D)
            d = d[:, :: max(1, d.shape[1] // 150)]
        else:
            d = np.concatenate([_tuples(M, 1) * D,
                                rng.integers(-D, D + 1, size=(M, 100))], axis=1)
        delta = orc.entangle(d, w, l)
        T = delta.shape[1]
        missed = 0
        for j in range(M):
            dd = np.repeat(delta, len(vals), axis=1)
            newv = np.tile(vals, T)
            keep = newv != dd[j]
            dd[j] = newv
            dd = dd[:, keep]
            _, flags, bad = orc.extract_check(dd, w, l, 0)
            missed += dd.shape[1] - bad
        if M * l >= w:
            assert missed == 0, (l, k)
            seen_cover = True
        else:
            assert missed > 0, (l, k)
            seen_escape = True
    assert seen_cover
    assert orc.params(M, w)[0] * M >= w


# ------------------------------------------------ closed forms at w = 64

@pytest.mark.parametrize("M", [3, 4, 5, 6, 7, 8])
def test_gemm_extraction_equals_plain_matmul(orc, M):
    """Extraction of the entangled GEMM equals numpy's plain int64 matmul of
    the original streams, from every r (detection reference) and from every
    surviving set of M-1 streams (fail-stop recovery)."""
    n, K, N = 7, 33, 9
    c, G = ne_synth.gemm_streams(11 + M, M, n, K, N, -128, 128)
    plain = np.stack([c[m].astype(np.int64) @ G.astype(np.int64) for m in range(M)])
    out = orc.gemm_pipeline(c, G)
    assert out["n_bad"] == 0
    assert (out["dhat"] == plain).all()
    # the unaware routine equals numpy's matmul on the entangled words
    assert (out["delta"] == np.stack([out["eps"][m] @ G.astype(np.int64) for m in range(M)])).all()
    l = out["l"]
    for r in range(M):
        assert (orc.extract(out["delta"], 64, l, r) == plain).all()
        assert (orc.recover(out["delta"], r, 64, l) == plain).all()


def test_gemm_wraps_like_python_ints(orc):
    """GEMM on words wraps modulo 2^w exactly as Python big integers do."""
    rng = np.random.default_rng(5)
    for w in (64, 16, 9):
        A = rng.integers(-(1 << (w - 1)), (1 << (w - 1)) - 1, size=(3, 4), dtype=np.int64)
        B = rng.integers(-(1 << (w - 1)), (1 << (w - 1)) - 1, size=(4, 2), dtype=np.int64)
        C = orc.gemm(A, B, w)
        for i in range(3):
            for j in range(2):
                ref = sum(int(A[i, k]) * int(B[k, j]) for k in range(4))
                assert int(C[i, j]) == _wrap(ref, w)


@pytest.mark.parametrize("N", [1, 2, 31, 257])
def test_circconv_extraction_equals_definition(orc, N):
    """Circular convolution: extraction equals the textbook definition
    y[n] = sum_k x[n-k mod N] g[k] computed with numpy.roll."""
    M = 3
    c, g = ne_synth.conv_streams(21 + N, M, N, -1024, 1024, -64, 64)
    g64 = g.astype(np.int64)
    plain = np.stack([sum(np.roll(c[m], k) * g64[k] for k in range(N)) for m in range(M)])
    out = orc.conv_pipeline(c, g64)
    assert out["n_bad"] == 0 and (out["dhat"] == plain).all()


def test_permute_scale_extraction_equals_definition(orc):
    """Permutation + scaling + addition of a self-entangled constant:
    extraction equals numpy fancy indexing of the plain streams."""
    M, N = 5, 301
    c, perm, s, a = ne_synth.perm_scale_streams(31, M, N, -128, 128)
    plain = c[:, perm] * s[None, :] + a[None, :]
    out = orc.permute_scale_pipeline(c, perm, s, a)
    assert out["n_bad"] == 0 and (out["dhat"] == plain).all()
    # without self-entangling the constant the homomorphism breaks
    l = out["l"]
    eps = orc.entangle(c, 64, l)
    raw = np.stack([orc.permute_scale(eps[m], perm, s, a) for m in range(M)])
    dhat, _, bad = orc.extract_check(raw, 64, l, 0)
    assert bad > 0 or not (dhat == plain).all()


def test_range_limit_is_exact_at_the_bound(orc):
    """Every output at +D or -D survives the round trip (w = 64, M = 3..8)."""
    for M in range(3, 9):
        l, k = orc.params(M, 64)
        D = orc.range_bound(M, l, k)
        d = np.array([[D, -D, 0, 1, -1]] * M, dtype=np.int64)
        for m in range(M):
            d[m] = np.roll(d[m], m)
        delta = orc.entangle(d, 64, l)
        for r in range(M):
            dhat, _, bad = orc.extract_check(delta, 64, l, r)
            assert (dhat == d).all() and bad == 0


# ------------------------------------------ the M = 3 special form, readings

def test_general_form_equals_m3_special_form_on_any_words(orc):
    """At M = 3, r = 0 the general disentanglement (with the (-1)^M reading)
    and the check coincide with the section III-A special form on arbitrary
    words, corrupted or not (w = 64 and w = 32)."""
    rng = np.random.default_rng(7)
    for w in (64, 32, 12):
        l, _ = orc.params(3, w)
        lo, hi = -(1 << (w - 1)), (1 << (w - 1)) - 1
        delta = rng.integers(lo, hi, size=(3, 5000), dtype=np.int64)
        delta[:, :50] = np.array([lo, hi, 0, -1, 1] * 10)[None, :]
        d3, f3, b3 = orc.extract3(delta, w, l)
        dg, fg, bg = orc.extract_check(delta, w, l, 0)
        assert (d3 == dg).all() and (f3 == fg).all() and b3 == bg


def _printed_extract(delta_col, M, l, w, r):
    """The general disentanglement exactly as printed (no leading (-1)^M),
    in Python integers, for one position."""
    L = (M - 1) * l
    dtemp = sum((-1) ** m * (int(delta_col[(r + 1 + m) % M]) << ((M - 2 - m) * l))
                for m in range(M - 1))
    low = dtemp & ((1 << L) - 1)
    d_last = low - (1 << L) if low >> (L - 1) else low
    d_r = ((-1) ** M * (dtemp - d_last)) >> L
    return d_r, d_last


@pytest.mark.parametrize("M", [3, 4, 5, 6])
def test_printed_sign_reading(orc, M):
    """The printed d_temp returns -d for odd M and d for even M; the oracle
    (with the leading (-1)^M) returns d for every M."""
    l, _ = orc.params(M, 64)
    c, G = ne_synth.gemm_streams(40 + M, M, 2, 5, 3, -128, 128)
    out = orc.gemm_pipeline(c, G)
    plain = np.stack([c[m].astype(np.int64) @ G.astype(np.int64) for m in range(M)])
    delta = out["delta"].reshape(M, -1)
    d = plain.reshape(M, -1)
    sign = 1 if M % 2 == 0 else -1
    for p in range(delta.shape[1]):
        d_r, d_last = _printed_extract(delta[:, p], M, l, 64, 0)
        assert d_r == sign * d[0, p] and d_last == sign * d[M - 1, p]
    assert (out["dhat"] == plain).all()


def test_check_needs_exact_2w_compare(orc):
    """Single-bit flips at w = 64, M = 3: the exact check flags every one;
    a comparison reduced modulo 2^64 (not the paper's 2w-bit interim) would
    miss some.  Shows why the check is evaluated in 2w bits."""
    M, n, K, N = 3, 8, 16, 8
    c, G = ne_synth.gemm_streams(51, M, n, K, N, -128, 128)
    out = orc.gemm_pipeline(c, G)
    l = out["l"]
    delta = out["delta"].reshape(M, -1)
    s, p, b = ne_synth.bit_flip_trials(52, 2000, M, delta.shape[1])
    missed_mod = 0
    for j, pos, bit in zip(s, p, b):
        dd = delta.copy()
        dd[j, pos] = _wrap(int(dd[j, pos]) ^ (1 << int(bit)), 64)
        dhat, flags, bad = orc.extract_check(dd, 64, l, 0)
        assert bad == 1 and flags[pos] == 1
        rebuilt = (int(dhat[0, pos]) + (int(dhat[2, pos]) << l))
        if _wrap(rebuilt, 64) == int(dd[0, pos]):
            missed_mod += 1
    assert missed_mod > 0


# ------------------------------------------------------------------- ABFT

def test_abft_checksum_identities(orc):
    """Section II-A: the checksum stream's output equals the sum of the
    outputs; one corrupted stream is flagged; a lost stream is rebuilt."""
    M, n, K, N = 4, 5, 12, 6
    c, G = ne_synth.gemm_streams(61, M, n, K, N, -127, 128)
    c64 = c.astype(np.int64)
    d = np.stack([c64[m] @ G.astype(np.int64) for m in range(M)])
    rsum = orc.abft_checksum(c64)
    assert (rsum == c64.sum(axis=0)).all()
    e = orc.gemm(rsum, G)
    flags, bad = orc.abft_check(d, e)
    assert bad == 0
    bad_d = d.copy()
    bad_d[2, 1, 3] += 7
    flags, bad = orc.abft_check(bad_d, e)
    assert bad == 1 and flags[1, 3] == 1
    for lost in range(M):
        dd = d.copy()
        dd[lost] = 12345
        assert (orc.abft_recover(dd, e, lost) == d).all()


def test_opcount_limits(orc):
    """Section IV: the entanglement overhead ratio tends to 0 and the ABFT
    ratio to 1/M as N grows."""
    for M in (3, 8):
        big = 1e6
        assert orc.opcount("ne_gemm", M, big) / orc.opcount("gemm", M, big) < 1e-5
        assert abs(orc.opcount("abft_gemm", M, big) / orc.opcount("gemm", M, big) - 1 / M) < 1e-5
        assert orc.opcount("ne_conv", M, big) / orc.opcount("conv_time", M, big) < 1e-5


def test_empty_streams(orc):
    d = np.zeros((3, 0), dtype=np.int64)
    dhat, flags, bad = orc.extract_check(d, 64, 22, 0)
    assert dhat.shape == (3, 0) and bad == 0


@pytest.mark.parametrize("M", [3, 5, 8])
def test_lsb_homomorphism(orc, M):
    """Section III-A: an LSB operation on the entangled streams gives the
    entangled outputs, delta_i = d_i + 2^l d_{i-1} (mod 2^64), where d is the
    plain operation on the plain inputs.  d comes from numpy / Python
    integers; delta from the oracle's entangle followed by its operation on
    words.  GEMM, circular convolution and permute + scale + add."""
    l, k = orc.params(M, 64)
    rng = np.random.default_rng(1700 + M)

    def ent(d):
        out = np.empty_like(d)
        for i in range(M):
            for idx in np.ndindex(d.shape[1:]):
                out[(i,) + idx] = _wrap(int(d[(i,) + idx]) + (int(d[((i - 1) % M,) + idx]) << l), 64)
        return out

    # GEMM, 7 x 9 times 9 x 5
    c = rng.integers(-128, 128, (M, 7, 9))
    G = rng.integers(-128, 128, (9, 5))
    d = np.stack([c[i] @ G for i in range(M)])
    delta = np.stack([orc.gemm(e, G) for e in orc.entangle(c, 64, l)])
    assert np.array_equal(delta, ent(d))
    # circular convolution, N = 11
    x = rng.integers(-1000, 1000, (M, 11))
    g = rng.integers(-64, 64, 11)
    d = np.stack([[sum(int(x[i][(t - j) % 11]) * int(g[j]) for j in range(11)) for t in range(11)]
                  for i in range(M)])
    delta = np.stack([orc.circconv(e, g) for e in orc.entangle(x, 64, l)])
    assert np.array_equal(delta, ent(d))
    # permutation, scaling, addition (the constant enters self-entangled)
    n = 13
    x = rng.integers(-1000, 1000, (M, n))
    perm = rng.permutation(n)
    s = rng.integers(-50, 50, n)
    a = rng.integers(-50, 50, n)
    d = np.stack([s * x[i][perm] + a for i in range(M)])
    a_ent = orc.self_entangle(a, 64, l)
    delta = np.stack([orc.permute_scale(e, perm, s, a_ent) for e in orc.entangle(x, 64, l)])
    assert np.array_equal(delta, ent(d))


# ------------------------------------------------------------------ series

def _plain_series(c, ops, M):
    """The series applied to each plain stream with Python integers: numpy
    object arrays for the products, explicit sums for the convolution,
    fancy indexing for the permutation."""
    out = []
    for m in range(M):
        x = np.array(c[m], dtype=object)
        for op in ops:
            kind = op[0]
            if kind == "gemm":
                G = np.array(op[1], dtype=object)
                x = x.reshape(-1, G.shape[0]).dot(G)
            elif kind == "conv":
                x = x.reshape(-1)
                N = x.size
                g = [int(v) for v in op[1]]
                x = np.array([sum(x[(t - j) % N] * g[j] for j in range(N)) for t in range(N)],
                             dtype=object)
            elif kind == "scale_add":
                x = x.reshape(-1)
                s = np.array(op[1], dtype=object) if op[1] is not None else 1
                a = np.array(op[2], dtype=object) if op[2] is not None else 0
                x = s * x + a
            elif kind == "permute":
                x = x.reshape(-1)[np.asarray(op[1])]
        out.append(x.reshape(-1))
    return out


@pytest.mark.parametrize("M", [3, 4, 8])
def test_series_matches_plain_series(orc, M):
    """Section II: a series of LSB operations on the entangled streams,
    disentangled once at the end, returns the series applied to each plain
    stream, exactly, with no flags; the final entangled words are E(d)."""
    l, k = orc.params(M, 64)
    rng = np.random.default_rng(2200 + M)
    n, K, N = 6, 10, 7
    c = rng.integers(-128, 128, (M, n, K))
    G = rng.integers(-128, 128, (K, N))
    q = n * N
    s1 = rng.integers(-100, 100, q)
    a1 = rng.integers(-1000, 1000, q)
    p1 = rng.permutation(q)
    g2 = rng.integers(-64, 64, q)
    p2 = rng.permutation(q)
    G3 = rng.integers(-20, 20, (N, 3))
    series = [
        [("gemm", G), ("scale_add", s1, a1), ("permute", p1)],
        [("gemm", G), ("permute", p1), ("conv", g2), ("scale_add", None, a1)],
        [("gemm", G), ("scale_add", s1, None), ("permute", p2), ("gemm", G3)],
    ]
    for ops in series:
        res = orc.series_pipeline(c, ops)
        want = _plain_series(c, ops, M)
        assert res["n_bad"] == 0 and not res["flags"].any()
        for m in range(M):
            assert [int(v) for v in res["dhat"][m].reshape(-1)] == [int(v) for v in want[m]]
            ent = [_wrap(int(want[m][i]) + (int(want[(m - 1) % M][i]) << l), 64)
                   for i in range(want[m].size)]
            assert [int(v) for v in res["delta"][m].reshape(-1)] == ent


def test_series_bound_is_attained(orc):
    """The composed a-priori bound equals the output for the extremal input
    (every operand at its bound, same sign), and random inputs stay within
    it: the bound of a GEMM of length K is K c_max g_max, of a scale/add
    s_max B + a_max, a permutation leaves it unchanged."""
    M = 3
    rng = np.random.default_rng(2301)
    n, K, N = 4, 9, 5
    c_max, g_max, s_max, a_max = 120, 110, 7, 900
    q = n * N
    ops_b = [("gemm", K, g_max), ("scale_add", s_max, a_max), ("permute",), ("conv", q, 3)]
    B = orc.series_bound(c_max, ops_b)
    assert B == ((c_max * K * g_max) * s_max + a_max) * q * 3
    c = np.full((M, n, K), c_max)
    ops = [("gemm", np.full((K, N), g_max)), ("scale_add", np.full(q, s_max), np.full(q, a_max)),
           ("permute", rng.permutation(q)), ("conv", np.full(q, 3))]
    out = _plain_series(c, ops, M)
    assert all(int(v) == B for m in range(M) for v in out[m])
    for _ in range(3):
        c = rng.integers(-c_max, c_max + 1, (M, n, K))
        ops = [("gemm", rng.integers(-g_max, g_max + 1, (K, N))),
               ("scale_add", rng.integers(-s_max, s_max + 1, q), rng.integers(-a_max, a_max + 1, q)),
               ("permute", rng.permutation(q)), ("conv", rng.integers(-3, 4, q))]
        out = _plain_series(c, ops, M)
        assert max(abs(int(v)) for m in range(M) for v in out[m]) <= B


def test_series_intermediate_wrap_tiny_w(orc):
    """Only the series' final output must lie in [-D, D]: at w = 16 an
    intermediate far outside the range (the entangled words wrap mod 2^16)
    still disentangles exactly once a later operation brings it back, since
    every operation is linear mod 2^w.  A final output outside the range
    does not."""
    M, w = 3, 16
    l, k = orc.params(M, w)
    D = orc.range_bound(M, l, k)
    rng = np.random.default_rng(2302)
    n = 40
    c = rng.integers(-D, D + 1, (M, n))
    big = np.full(n, 50 * D)
    perm = rng.permutation(n)
    ops = [("scale_add", None, big), ("permute", perm), ("scale_add", None, -big)]
    res = orc.series_pipeline(c, ops, w=w)
    assert res["n_bad"] == 0
    assert np.array_equal(res["dhat"], c[:, perm])
    res = orc.series_pipeline(c, ops[:2], w=w)
    assert not np.array_equal(res["dhat"], c[:, perm] + 50 * D)


# ------------------------------------------------------ linear convolution

def test_linconv_textbook(orc):
    """The oracle's linear convolution equals numpy.convolve (full mode),
    including a kernel longer than the input and a single tap."""
    rng = np.random.default_rng(2600)
    for nx, L in [(50, 7), (5, 12), (33, 1), (1, 1), (300, 64)]:
        x = rng.integers(-1000, 1000, nx)
        g = rng.integers(-64, 64, L)
        assert np.array_equal(orc.linconv(x, g), np.convolve(x, g))


def test_linconv_overlap_save(orc):
    """Overlap-save (section IV's block realisation): blocks of B inputs
    overlapping by L - 1, each circularly convolved with the zero-padded
    kernel, keep their last B - L + 1 outputs; concatenated they are the
    linear convolution.  Pins the linear convolution against the (separately
    pinned) circular one."""
    rng = np.random.default_rng(2601)
    nx, L, B = 97, 9, 32
    x = rng.integers(-1000, 1000, nx)
    g = rng.integers(-64, 64, L)
    hop = B - L + 1
    ny = nx + L - 1
    xp = np.concatenate([np.zeros(L - 1, np.int64), x, np.zeros(B, np.int64)])
    gp = np.concatenate([g, np.zeros(B - L, np.int64)])
    out = []
    for s in range(0, ny, hop):
        yb = orc.circconv(xp[s:s + B], gp)
        out.append(yb[L - 1:])
    y = np.concatenate(out)[:ny]
    assert np.array_equal(y, orc.linconv(x, g))


@pytest.mark.parametrize("M", [3, 8])
def test_linconv_pipeline(orc, M):
    """Entangled linear convolution: exact outputs (numpy.convolve per
    stream), entangled words E(d), no flags on clean data, and a bit flipped
    in one stream's output flagged at exactly that position."""
    l, k = orc.params(M, 64)
    rng = np.random.default_rng(2602 + M)
    nx, L = 120, 17
    c = rng.integers(-(1 << 14), 1 << 14, (M, nx))
    g = rng.integers(-128, 128, L)
    res = orc.linconv_pipeline(c, g)
    want = np.stack([np.convolve(c[m], g) for m in range(M)])
    assert np.array_equal(res["dhat"], want)
    assert res["n_bad"] == 0
    for m in range(M):
        ent = [_wrap(int(want[m][t]) + (int(want[(m - 1) % M][t]) << l), 64)
               for t in range(want.shape[1])]
        assert [int(v) for v in res["delta"][m]] == ent
    delta = res["delta"].copy()
    delta[M - 1, 40] ^= 1 << 33
    _, flags, bad = orc.extract_check(delta, 64, l, 0)
    assert bad == 1 and flags[40] and flags.sum() == 1


# ---------------------------------------------------------------------------
# Row/column checksum ABFT (section V, the RC-check baseline)

def test_abft_rc_brute_force(orc):
    """d and both checksum comparisons against Python-integer loops over the
    definitions (product, row sums, column sums) on a tiny ragged case."""
    M, n, K, N = 2, 3, 5, 4
    c = ne_synth.uniform_int(4100, 1, (M, n, K), -128, 128)
    G = ne_synth.uniform_int(4100, 2, (K, N), -128, 128)
    d = [[[sum(int(c[m, i, k]) * int(G[k, p]) for k in range(K)) for p in range(N)]
          for i in range(n)] for m in range(M)]
    got = orc.abft_rc(c, G)
    assert got["d"].tolist() == d
    assert got["n_bad"] == 0 and not got["row_bad"].any() and not got["col_bad"].any()
    bad = [row[:] for row in d[1]]
    bad[2][1] += 7
    dd = np.array([d[0], bad])
    got = orc.abft_rc(c, G, dd)
    for i in range(n):
        want = sum(bad[i]) != sum(int(c[1, i, k]) * sum(int(G[k, p]) for p in range(N))
                                  for k in range(K))
        assert got["row_bad"][1, i] == want
    for p in range(N):
        want = sum(bad[i][p] for i in range(n)) != sum(
            sum(int(c[1, i, k]) for i in range(n)) * int(G[k, p]) for k in range(K))
        assert got["col_bad"][1, p] == want
    assert got["row_bad"][1].tolist() == [False, False, True]
    assert got["col_bad"][1].tolist() == [False, True, False, False]
    assert not got["row_bad"][0].any() and not got["col_bad"][0].any() and got["n_bad"] == 2


def test_abft_rc_detects_up_to_three(orc):
    """Every set of one to three wrong positions of a subblock is flagged
    (the guarantee the paper quotes for the RC-check), and a single wrong
    position is located at exactly its row and column."""
    M, n, K, N = 3, 9, 12, 7
    c = ne_synth.uniform_int(4200, 1, (M, n, K), -128, 128)
    G = ne_synth.uniform_int(4200, 2, (K, N), -128, 128)
    d = orc.abft_rc(c, G)["d"]
    rng = np.random.default_rng(42)
    for trial in range(300):
        m = int(rng.integers(M))
        cnt = 1 + trial % 3
        pos = rng.choice(n * N, size=cnt, replace=False)
        dd = d.copy()
        for q in pos:
            e = int(rng.integers(1, 1 << 20)) * (1 if rng.integers(2) else -1)
            dd[m, q // N, q % N] += e
        got = orc.abft_rc(c, G, dd)
        assert got["n_bad"] > 0, (trial, pos)
        others = [x for x in range(M) if x != m]
        assert not got["row_bad"][others].any() and not got["col_bad"][others].any()
        if cnt == 1:
            i, p = divmod(int(pos[0]), N)
            assert np.nonzero(got["row_bad"][m])[0].tolist() == [i]
            assert np.nonzero(got["col_bad"][m])[0].tolist() == [p]


def test_abft_rc_rectangle_undetected(orc):
    """Four errors +e, -e, -e, +e at the corners of a rectangle cancel in
    both sums: the RC-check's known blind spot (so four is not guaranteed)."""
    M, n, K, N = 1, 6, 8, 5
    c = ne_synth.uniform_int(4300, 1, (M, n, K), -128, 128)
    G = ne_synth.uniform_int(4300, 2, (K, N), -128, 128)
    d = orc.abft_rc(c, G)["d"]
    d[0, 1, 0] += 5
    d[0, 1, 3] -= 5
    d[0, 4, 0] -= 5
    d[0, 4, 3] += 5
    assert orc.abft_rc(c, G, d)["n_bad"] == 0
