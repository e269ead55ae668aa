"""CPU oracle for numerical entanglement (test infrastructure).

Thin numpy/ctypes front end over ``ne_oracle.c``.  Only the test-suite, the
smoke check and the CPU-baseline leg of the benchmark may import this
package; the product library never does, and the two share no code.

Every function follows one passage of Anam & Andreopoulos, "Reliable Linear,
Sesquilinear and Bijective Operations on Integer Data Streams via Numerical
Entanglement" (arXiv 1604.04740); the C source names the passage.  Word
width ``w`` is generic (4..64) so that tiny-width exhaustive tests can run.

Parity status of each function (what pins it is listed in tests/):
  params, range_bound           pinned (Table II; exhaustive tiny-w range)
  entangle, self_entangle       pinned (hand-worked example; operator E)
  gemm, circconv, permute_scale pinned (numpy / Python-int textbook results)
  linconv, linconv_pipeline     pinned (numpy convolve; overlap-save blocks
                                of the pinned circular convolution)
  extract, check, extract3      pinned (exhaustive tiny w, closed forms)
  abft_checksum, abft_check     pinned (sum identities, recovery)
  abft_rc                       pinned (Python-int brute force; every 1-3
                                wrong positions flagged, a +-e rectangle of
                                four not; a single one at its row x column)
  series_bound, series_pipeline pinned (plain series in Python integers,
                                homomorphism after every step, extremal
                                inputs at the bound, tiny-w range edge)
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "ne_oracle.c")
_LIB = os.path.join(_HERE, "libne_oracle.so")

_i64p = ctypes.POINTER(ctypes.c_int64)
_u8p = ctypes.POINTER(ctypes.c_uint8)


def build(force: bool = True) -> str:
    """Compile ne_oracle.c with gcc into oracle/libne_oracle.so."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp%d" % os.getpid()
        cmd = ["gcc", "-O2", "-std=c11", "-fopenmp", "-fPIC", "-shared",
               "-Wall", "-Wextra", "-o", tmp, _SRC, "-lm"]
        subprocess.check_call(cmd)
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=False)
        L = ctypes.CDLL(_LIB)
        i, I = ctypes.c_int, ctypes.c_int64
        L.ne_oracle_params.argtypes = [i, i, ctypes.POINTER(i), ctypes.POINTER(i)]
        L.ne_oracle_params.restype = i
        L.ne_oracle_range.argtypes = [i, i, i]
        L.ne_oracle_range.restype = I
        L.ne_oracle_entangle.argtypes = [_i64p, _i64p, i, I, i, i]
        L.ne_oracle_entangle.restype = None
        L.ne_oracle_self_entangle.argtypes = [_i64p, _i64p, I, i, i]
        L.ne_oracle_self_entangle.restype = None
        L.ne_oracle_gemm.argtypes = [_i64p, _i64p, _i64p, I, I, I, i]
        L.ne_oracle_gemm.restype = None
        L.ne_oracle_circconv.argtypes = [_i64p, _i64p, _i64p, I, i]
        L.ne_oracle_circconv.restype = None
        L.ne_oracle_linconv.argtypes = [_i64p, I, _i64p, I, _i64p, i]
        L.ne_oracle_linconv.restype = None
        L.ne_oracle_permute_scale.argtypes = [_i64p, _i64p, _i64p, _i64p, _i64p, I, i]
        L.ne_oracle_permute_scale.restype = None
        L.ne_oracle_extract.argtypes = [_i64p, _i64p, i, I, i, i, i]
        L.ne_oracle_extract.restype = None
        L.ne_oracle_check.argtypes = [_i64p, _i64p, _u8p, i, I, i, i, i]
        L.ne_oracle_check.restype = I
        L.ne_oracle_extract3.argtypes = [_i64p, _i64p, _u8p, I, i, i]
        L.ne_oracle_extract3.restype = I
        L.ne_oracle_abft_checksum.argtypes = [_i64p, _i64p, i, I, i]
        L.ne_oracle_abft_checksum.restype = None
        L.ne_oracle_abft_check.argtypes = [_i64p, _i64p, _u8p, i, I, i, i]
        L.ne_oracle_abft_check.restype = I
        L.ne_oracle_opcount.argtypes = [i, ctypes.c_double, ctypes.c_double]
        L.ne_oracle_opcount.restype = ctypes.c_double
        _lib = L
    return _lib


def set_threads(n: int) -> None:
    """Number of OpenMP threads the oracle's loops use from now on."""
    lib()
    ctypes.CDLL("libgomp.so.1").omp_set_num_threads(int(n))


def _a64(x) -> np.ndarray:
    return np.ascontiguousarray(x, dtype=np.int64)


def _p(x: np.ndarray):
    return x.ctypes.data_as(_i64p)


# ------------------------------------------------------------- parameters

def params(M: int, w: int = 64):
    """(l, k) by the paper's rule (section III-C), tight tie-break."""
    l, k = ctypes.c_int(), ctypes.c_int()
    if lib().ne_oracle_params(M, w, ctypes.byref(l), ctypes.byref(k)) != 0:
        raise ValueError("no admissible (l, k) for M=%d, w=%d" % (M, w))
    return l.value, k.value


def range_bound(M: int, l: int, k: int) -> int:
    """Output dynamic range D of section III-C: |d| <= D."""
    return int(lib().ne_oracle_range(M, l, k))


# ------------------------------------------------------------ entanglement

def entangle(c, w: int, l: int) -> np.ndarray:
    """eps[m] = c[m] + S_l{c[m-1 mod M]} (section III-C, operator E). c is [M][...]."""
    c = _a64(c)
    M = c.shape[0]
    if M > 256:
        raise ValueError("oracle supports M <= 256")
    N = c.size // M
    eps = np.empty_like(c)
    lib().ne_oracle_entangle(_p(c), _p(eps), M, N, w, l)
    return eps


def self_entangle(g, w: int, l: int) -> np.ndarray:
    """g <- S_l{g} + g (footnote in section III-A, for op in {+, -})."""
    g = _a64(g)
    out = np.empty_like(g)
    lib().ne_oracle_self_entangle(_p(g), _p(out), g.size, w, l)
    return out


# ------------------------------------------------------------- operations

def gemm(A, B, w: int = 64) -> np.ndarray:
    """C = A @ B on w-bit words (mod 2^w). A [R][K], B [K][N]."""
    A, B = _a64(A), _a64(B)
    R, K = A.shape
    K2, N = B.shape
    assert K == K2
    C = np.empty((R, N), dtype=np.int64)
    lib().ne_oracle_gemm(_p(A), _p(B), _p(C), R, K, N, w)
    return C


def circconv(x, g, w: int = 64) -> np.ndarray:
    """y[n] = sum_k x[(n-k) mod N] g[k] (mod 2^w)."""
    x, g = _a64(x), _a64(g)
    assert x.shape == g.shape and x.ndim == 1
    y = np.empty_like(x)
    lib().ne_oracle_circconv(_p(x), _p(g), _p(y), x.size, w)
    return y


def linconv(x, g, w: int = 64) -> np.ndarray:
    """y[t] = sum_j x[t-j] g[j], 0 <= t < len(x) + len(g) - 1, x zero outside
    its range (mod 2^w)."""
    x, g = _a64(x), _a64(g)
    assert x.ndim == 1 and g.ndim == 1 and x.size > 0 and g.size > 0
    y = np.empty(x.size + g.size - 1, dtype=np.int64)
    lib().ne_oracle_linconv(_p(x), x.size, _p(g), g.size, _p(y), w)
    return y


def permute_scale(x, perm, scale=None, add=None, w: int = 64) -> np.ndarray:
    """y[n] = scale[n] * x[perm[n]] + add[n] (mod 2^w)."""
    x, perm = _a64(x), _a64(perm)
    N = x.size
    s = _a64(scale) if scale is not None else None
    a = _a64(add) if add is not None else None
    y = np.empty_like(x)
    lib().ne_oracle_permute_scale(_p(x), _p(perm), _p(s) if s is not None else None,
                                  _p(a) if a is not None else None, _p(y), N, w)
    return y


# -------------------------------------------------------- disentanglement

def extract(delta, w: int, l: int, r: int = 0) -> np.ndarray:
    """dhat from all entangled outputs except stream r (section III-C)."""
    delta = _a64(delta)
    M = delta.shape[0]
    N = delta.size // M
    dhat = np.zeros_like(delta)
    lib().ne_oracle_extract(_p(delta), _p(dhat), M, N, w, l, r)
    return dhat


def check(delta, dhat, w: int, l: int, r: int = 0):
    """(flags, n_bad): delta_r against dhat_r + S_l{dhat_(r-1)} (appendix)."""
    delta, dhat = _a64(delta), _a64(dhat)
    M = delta.shape[0]
    N = delta.size // M
    flags = np.zeros(N, dtype=np.uint8)
    bad = lib().ne_oracle_check(_p(delta), _p(dhat), flags.ctypes.data_as(_u8p), M, N, w, l, r)
    return flags.reshape(delta.shape[1:]), int(bad)


def extract_check(delta, w: int, l: int, r: int = 0):
    dhat = extract(delta, w, l, r)
    flags, bad = check(delta, dhat, w, l, r)
    return dhat, flags, bad


def recover(delta, lost: int, w: int, l: int) -> np.ndarray:
    """All outputs from the M-1 surviving streams (fail-stop of stream `lost`)."""
    delta = _a64(delta).copy()
    delta[lost] = 0  # the lost stream's content is never read
    return extract(delta, w, l, lost)


def extract3(delta, w: int, l: int):
    """Section III-A special form (M = 3, r = 0): (dhat, flags, n_bad)."""
    delta = _a64(delta)
    assert delta.shape[0] == 3
    N = delta.size // 3
    dhat = np.zeros_like(delta)
    flags = np.zeros(N, dtype=np.uint8)
    bad = lib().ne_oracle_extract3(_p(delta), _p(dhat), flags.ctypes.data_as(_u8p), N, w, l)
    return dhat, flags.reshape(delta.shape[1:]), int(bad)


# -------------------------------------------------------------------- ABFT

def abft_checksum(c, w: int = 64) -> np.ndarray:
    """r_n = sum_m c_{m,n} (section II-A)."""
    c = _a64(c)
    M = c.shape[0]
    out = np.empty(c.shape[1:], dtype=np.int64)
    lib().ne_oracle_abft_checksum(_p(c), _p(out), M, c.size // M, w)
    return out


def abft_check(d, e, w: int = 64):
    """(flags, n_bad): sum_m d_m != e (section II-A)."""
    d, e = _a64(d), _a64(e)
    M = d.shape[0]
    N = d.size // M
    flags = np.zeros(N, dtype=np.uint8)
    bad = lib().ne_oracle_abft_check(_p(d), _p(e), flags.ctypes.data_as(_u8p), M, N, w, -1)
    return flags.reshape(d.shape[1:]), int(bad)


def abft_recover(d, e, lost: int, w: int = 64) -> np.ndarray:
    """Rebuild the lost output stream as e - sum of the others (section II-A)."""
    d, e = _a64(d).copy(), _a64(e)
    M = d.shape[0]
    lib().ne_oracle_abft_check(_p(d), _p(e), None, M, d.size // M, w, lost)
    return d


def abft_rc(c, G, d=None):
    """Row/column checksum ABFT (Huang and Abraham), the "RC-check" baseline
    of the GEMM comparison in section V, over M subblock products
    d[m] = c[m] G (c [M][n][K], G [K][N]; d computed here when None).
    The input checksums e^T c[m] and G e give the row sums c[m] (G e) and
    the column sums (e^T c[m]) G that d[m] must have; a row or column whose
    sum differs is flagged.  Returns d, row_bad [M][n], col_bad [M][N] and
    n_bad (flagged rows plus columns).  Sums are 64-bit exact for the sizes
    used here."""
    c = _a64(c)
    G = _a64(G)
    M = c.shape[0]
    if d is None:
        d = np.stack([gemm(c[m], G) for m in range(M)])
    d = _a64(d)
    ge = G.sum(axis=1)                       # G e
    row_bad = np.zeros(d.shape[:2], dtype=bool)
    col_bad = np.zeros((M, d.shape[2]), dtype=bool)
    for m in range(M):
        row_ref = gemm(c[m], ge[:, None])[:, 0]
        col_ref = gemm(c[m].sum(axis=0)[None, :], G)[0]
        row_bad[m] = d[m].sum(axis=1) != row_ref
        col_bad[m] = d[m].sum(axis=0) != col_ref
    return {"d": d, "row_bad": row_bad, "col_bad": col_bad,
            "n_bad": int(row_bad.sum() + col_bad.sum())}


def opcount(which: str, M: float, N: float) -> float:
    """Operation counts of section IV."""
    idx = {"gemm": 0, "conv_time": 1, "conv_freq": 2, "ne_conv": 3, "ne_gemm": 4,
           "abft_gemm": 5, "abft_conv_time": 6}[which]
    return float(lib().ne_oracle_opcount(idx, float(M), float(N)))


# ------------------------------------------------------ composed pipelines

def gemm_pipeline(c, G, w: int = 64, r: int = 0, l: int | None = None):
    """Entangle the M streams c[M][n][K], multiply each by the shared G[K][N]
    (section III-A: delta_m = eps_m op g), extract without stream r and check.
    Returns dict with eps, delta, dhat, flags, n_bad, (l, k)."""
    c = _a64(c)
    M, n, K = c.shape
    lk = params(M, w)
    l = lk[0] if l is None else l
    eps = entangle(c, w, l)
    delta = gemm(eps.reshape(M * n, K), G, w).reshape(M, n, -1)
    dhat, flags, bad = extract_check(delta, w, l, r)
    return dict(eps=eps, delta=delta, dhat=dhat, flags=flags, n_bad=bad, l=l, k=lk[1])


def conv_pipeline(c, g, w: int = 64, r: int = 0):
    c = _a64(c)
    M, N = c.shape
    l, k = params(M, w)
    eps = entangle(c, w, l)
    delta = np.stack([circconv(eps[m], g, w) for m in range(M)])
    dhat, flags, bad = extract_check(delta, w, l, r)
    return dict(eps=eps, delta=delta, dhat=dhat, flags=flags, n_bad=bad, l=l, k=k)


def linconv_pipeline(c, g, w: int = 64, r: int = 0):
    """Entangle c[M][Nx], convolve every entangled stream with the L-tap
    kernel g (linear convolution, section IV), extract without stream r and
    check."""
    c = _a64(c)
    M = c.shape[0]
    l, k = params(M, w)
    eps = entangle(c, w, l)
    delta = np.stack([linconv(eps[m], g, w) for m in range(M)])
    dhat, flags, bad = extract_check(delta, w, l, r)
    return dict(eps=eps, delta=delta, dhat=dhat, flags=flags, n_bad=bad, l=l, k=k)


def permute_scale_pipeline(c, perm, scale, add, w: int = 64, r: int = 0):
    c = _a64(c)
    M, N = c.shape
    l, k = params(M, w)
    eps = entangle(c, w, l)
    add_ent = self_entangle(add, w, l) if add is not None else None
    delta = np.stack([permute_scale(eps[m], perm, scale, add_ent, w) for m in range(M)])
    dhat, flags, bad = extract_check(delta, w, l, r)
    return dict(eps=eps, delta=delta, dhat=dhat, flags=flags, n_bad=bad, l=l, k=k)


# ------------------------------------------------------- operation series

def series_bound(c_max: int, ops) -> int:
    """A-priori bound on |output| after a series of LSB operations applied
    in turn to inputs with |c| <= c_max (section II: operators applied
    consecutively; the output range condition of section III-C then holds
    for the series' final output).  Exact Python integers.  ops are tuples
      ('gemm', K, g_max)     contraction of length K with |G| <= g_max
      ('conv', N, g_max)     circular convolution over N taps, |g| <= g_max
      ('scale_add', s_max, a_max)   s * x + a with |s| <= s_max, |a| <= a_max
      ('permute',)           bijective index map
    """
    B = int(c_max)
    for op in ops:
        kind = op[0]
        if kind in ("gemm", "conv"):
            B = B * int(op[1]) * int(op[2])
        elif kind == "scale_add":
            B = B * int(op[1]) + int(op[2])
        elif kind == "permute":
            pass
        else:
            raise ValueError(kind)
    return B


def _series_step(x, op, w: int, l: int):
    """One LSB operation applied to every stream of x [M][...] (words mod 2^w).
    The + constant is entangled with itself first (footnote of section III-A)."""
    M = x.shape[0]
    kind = op[0]
    if kind == "gemm":
        G = _a64(op[1])
        K = G.shape[0]
        y = gemm(x.reshape(-1, K), G, w)
        return y.reshape(M, -1, G.shape[1])
    flat = x.reshape(M, -1)
    if kind == "conv":
        return np.stack([circconv(flat[m], op[1], w) for m in range(M)])
    if kind == "scale_add":
        scale, add = op[1], op[2]
        n = flat.shape[1]
        ident = np.arange(n, dtype=np.int64)
        a = self_entangle(add, w, l) if add is not None else None
        return np.stack([permute_scale(flat[m], ident, scale, a, w) for m in range(M)])
    if kind == "permute":
        return np.stack([permute_scale(flat[m], op[1], None, None, w) for m in range(M)])
    raise ValueError(kind)


def series_pipeline(c, ops, w: int = 64, r: int = 0, l: int | None = None):
    """Entangle the M input streams once, apply a series of LSB operations to
    the entangled streams (section II), then disentangle and check once
    (section III-C).  c is [M][...]; ops are
      ('gemm', G)            each stream viewed as rows of G.shape[0] entries
      ('conv', g)            circular convolution of the flattened stream
      ('scale_add', s, a)    y[q] = s[q] x[q] + a[q] (either may be None)
      ('permute', perm)      y[q] = x[perm[q]]
    Returns dict with eps, delta (after the last operation), dhat, flags,
    n_bad, (l, k)."""
    c = _a64(c)
    M = c.shape[0]
    lk = params(M, w)
    l = lk[0] if l is None else l
    eps = entangle(c, w, l)
    x = eps
    for op in ops:
        x = _series_step(x, op, w, l)
    delta = x
    dhat, flags, bad = extract_check(delta, w, l, r)
    return dict(eps=eps, delta=delta, dhat=dhat, flags=flags, n_bad=bad, l=l, k=lk[1])
