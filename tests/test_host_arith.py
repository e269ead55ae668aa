"""The library's word arithmetic (ne_arith.h), compiled for the host into
libne_selftest.so, against the oracle on the CPU: the 64-bit exact
disentanglement and check must equal the oracle's 2w-bit evaluation on
arbitrary words (random, extreme, codewords) for every M and every r, and
the signed-digit split must reproduce every word."""
import ctypes
import os

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SELFTEST = os.path.join(ROOT, "paper_1604_04740_amd", "libne_selftest.so")

P64 = ctypes.POINTER(ctypes.c_int64)
PU8 = ctypes.POINTER(ctypes.c_uint8)


@pytest.fixture(scope="module")
def st():
    if not os.path.exists(SELFTEST):
        from paper_1604_04740_amd import _build
        _build.build()
    L = ctypes.CDLL(SELFTEST)
    L.ne_selftest_disentangle.argtypes = [P64, P64, PU8, ctypes.c_int, ctypes.c_int64,
                                          ctypes.c_int, ctypes.c_int]
    L.ne_selftest_disentangle.restype = ctypes.c_int64
    L.ne_selftest_digits.argtypes = [P64, ctypes.POINTER(ctypes.c_int8), ctypes.c_int64, ctypes.c_int]
    P32 = ctypes.POINTER(ctypes.c_int32)
    L.ne_selftest_disentangle32.argtypes = [P32, P32, PU8, ctypes.c_int, ctypes.c_int64,
                                            ctypes.c_int, ctypes.c_int]
    L.ne_selftest_disentangle32.restype = ctypes.c_int64
    return L


def _words(rng, M, N):
    info = np.iinfo(np.int64)
    d = rng.integers(info.min, info.max, size=(M, N), dtype=np.int64)
    d[:, : N // 4] >>= rng.integers(0, 63, size=(M, N // 4))
    edge = np.array([info.min, info.max, 0, 1, -1], dtype=np.int64)
    k = min(M, 5)
    E = np.stack(np.meshgrid(*([edge] * k), indexing="ij"), 0).reshape(k, -1)
    d[:k, : E.shape[1]] = E
    return d


@pytest.mark.parametrize("M", list(range(3, 17)))
def test_disentangle_equals_oracle(st, orc, M):
    rng = np.random.default_rng(M)
    l, k = orc.params(M, 64)
    N = 60000
    d = _words(rng, M, N)
    D = orc.range_bound(M, l, k)
    lim = min(D, (1 << 62))
    c = rng.integers(-lim, lim + 1, size=(M, 3000))
    d[:, N // 2: N // 2 + 3000] = orc.entangle(c, 64, l)
    for r in range(M):
        dh_o, fl_o, bad_o = orc.extract_check(d, 64, l, r)
        dh = np.zeros_like(d)
        fl = np.zeros(N, dtype=np.uint8)
        bad = st.ne_selftest_disentangle(d.ctypes.data_as(P64), dh.ctypes.data_as(P64),
                                         fl.ctypes.data_as(PU8), M, N, l, r)
        assert np.array_equal(dh, dh_o), r
        assert np.array_equal(fl, fl_o) and bad == bad_o, r


def test_digit_split_reproduces_words(st):
    rng = np.random.default_rng(3)
    info = np.iinfo(np.int64)
    v = rng.integers(info.min, info.max, size=20000, dtype=np.int64)
    for bits in (8, 9, 15, 16, 17, 24, 33, 56, 63, 64):
        x = v >> (64 - bits) if bits < 64 else v
        L = min(8, bits // 8 + 1)
        dig = np.zeros((x.size, L), dtype=np.int8)
        st.ne_selftest_digits(x.ctypes.data_as(P64), dig.ctypes.data_as(ctypes.POINTER(ctypes.c_int8)),
                              x.size, L)
        recon = np.zeros(x.size, dtype=np.uint64)
        with np.errstate(over="ignore"):
            for j in range(L):
                recon += dig[:, j].astype(np.int64).astype(np.uint64) << np.uint64(8 * j)
        assert np.array_equal(recon.view(np.int64), x), bits


@pytest.mark.parametrize("M", list(range(3, 17)))
def test_disentangle32_equals_oracle(st, orc, M):
    """w = 32: the 32-bit word arithmetic (64-bit interim) equals the
    oracle's 2w-bit evaluation on arbitrary 32-bit words and on codewords,
    for every r, wherever the paper's rule gives l >= 2."""
    try:
        l, k = orc.params(M, 32)
    except ValueError:
        pytest.skip("no admissible (l, k)")
    if l < 2:
        pytest.skip("l = 1")
    rng = np.random.default_rng(100 + M)
    N = 40000
    info = np.iinfo(np.int32)
    d = rng.integers(info.min, info.max, size=(M, N), dtype=np.int64)
    d[:, : N // 4] >>= rng.integers(0, 31, size=(M, N // 4))
    edge = np.array([info.min, info.max, 0, 1, -1], dtype=np.int64)
    kk = min(M, 5)
    E = np.stack(np.meshgrid(*([edge] * kk), indexing="ij"), 0).reshape(kk, -1)
    d[:kk, : E.shape[1]] = E
    D = orc.range_bound(M, l, k)
    c = rng.integers(-D, D + 1, size=(M, 3000))
    d[:, N // 2: N // 2 + 3000] = orc.entangle(c, 32, l)
    d32 = d.astype(np.int32)
    P32 = ctypes.POINTER(ctypes.c_int32)
    for r in range(M):
        dh_o, fl_o, bad_o = orc.extract_check(d, 32, l, r)
        dh = np.zeros_like(d32)
        fl = np.zeros(N, dtype=np.uint8)
        bad = st.ne_selftest_disentangle32(d32.ctypes.data_as(P32), dh.ctypes.data_as(P32),
                                           fl.ctypes.data_as(PU8), M, N, l, r)
        assert np.array_equal(dh.astype(np.int64), dh_o), r
        assert np.array_equal(fl, fl_o) and bad == bad_o, r
        assert np.array_equal(dh[:, N // 2: N // 2 + 3000].astype(np.int64), c), r
