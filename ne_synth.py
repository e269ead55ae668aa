"""Seeded synthetic inputs shared by the oracle side and the HIP side.

This module only draws numbers; it holds none of the method's arithmetic
(no entanglement, no operation, no extraction).  Every input of every test,
smoke run and benchmark is drawn here, so both implementations see the same
values.

Generator: SplitMix64 (Steele, Lea and Flood, "Fast splittable pseudorandom
number generators", OOPSLA 2014), used in counter form: output i of a
stream with key s is mix(s + (i + 1) * 0x9E3779B97F4A7C15), where mix is the
published SplitMix64 finaliser.  A uniform integer in [lo, hi) is
lo + ((z >> 32) * (hi - lo)) >> 32 (multiply-shift; span <= 2^32).

Each array in a workload gets its own key: key = seed * 1_000_003 + tag.
"""
from __future__ import annotations

import numpy as np

GAMMA = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)

BASE_SEED = 1604047400  # per-workload seed = BASE_SEED + workload index


def _mix(z: np.ndarray) -> np.ndarray:
    z = (z ^ (z >> np.uint64(30))) * _M1
    z = (z ^ (z >> np.uint64(27))) * _M2
    return z ^ (z >> np.uint64(31))


def raw_u64(key: int, count: int, start: int = 0) -> np.ndarray:
    """Outputs start .. start+count-1 of the SplitMix64 stream `key`."""
    with np.errstate(over="ignore"):
        i = np.arange(start + 1, start + count + 1, dtype=np.uint64)
        z = np.uint64(key & 0xFFFFFFFFFFFFFFFF) + i * GAMMA
        return _mix(z)


def stream_key(seed: int, tag: int) -> int:
    return (seed * 1_000_003 + tag) & 0xFFFFFFFFFFFFFFFF


def uniform_int(seed: int, tag: int, shape, lo: int, hi: int,
                dtype=np.int64, chunk: int = 1 << 24) -> np.ndarray:
    """Integers uniform in [lo, hi), drawn from stream (seed, tag)."""
    span = hi - lo
    if span <= 0 or span > (1 << 32):
        raise ValueError("span must be in (0, 2^32]")
    if isinstance(shape, int):
        shape = (shape,)
    count = int(np.prod(shape))
    out = np.empty(count, dtype=dtype)
    key = stream_key(seed, tag)
    with np.errstate(over="ignore"):
        for s in range(0, count, chunk):
            n = min(chunk, count - s)
            z = raw_u64(key, n, s) >> np.uint64(32)
            v = (z * np.uint64(span)) >> np.uint64(32)
            out[s:s + n] = (v.astype(np.int64) + lo).astype(dtype)
    return out.reshape(shape)


def permutation(seed: int, tag: int, n: int) -> np.ndarray:
    """Fisher-Yates shuffle of 0..n-1 driven by stream (seed, tag)."""
    p = np.arange(n, dtype=np.int64)
    if n <= 1:
        return p
    z = raw_u64(stream_key(seed, tag), n - 1) >> np.uint64(32)
    for idx, i in enumerate(range(n - 1, 0, -1)):
        j = int((int(z[idx]) * (i + 1)) >> 32)
        p[i], p[j] = p[j], p[i]
    return p


# --------------------------------------------------------------------------
# Workload recipes (shapes and value ranges of the paper-shaped workloads).
# --------------------------------------------------------------------------

def gemm_streams(seed: int, M: int, n: int, K: int, N: int, lo: int, hi: int):
    """M input streams c[M][n][K] and one shared operand G[K][N], both int8 range.

    Returns (c, G) as int8 arrays; G is row-major [K][N].
    """
    c = uniform_int(seed, 1, (M, n, K), lo, hi, dtype=np.int8)
    G = uniform_int(seed, 2, (K, N), lo, hi, dtype=np.int8)
    return c, G


def conv_streams(seed: int, M: int, N: int, c_lo: int, c_hi: int, g_lo: int, g_hi: int):
    """M streams c[M][N] (int64) and one shared filter g[N] (int8 range)."""
    c = uniform_int(seed, 3, (M, N), c_lo, c_hi, dtype=np.int64)
    g = uniform_int(seed, 4, (N,), g_lo, g_hi, dtype=np.int8)
    return c, g


def perm_scale_streams(seed: int, M: int, N: int, lo: int, hi: int):
    """M streams c[M][N], a bijection perm[N], per-position scale s[N] and
    additive constant a[N] (all in [lo, hi) except perm)."""
    c = uniform_int(seed, 5, (M, N), lo, hi, dtype=np.int64)
    perm = permutation(seed, 6, N)
    s = uniform_int(seed, 7, (N,), lo, hi, dtype=np.int64)
    a = uniform_int(seed, 8, (N,), lo, hi, dtype=np.int64)
    return c, perm, s, a


def bit_flip_trials(seed: int, trials: int, M: int, positions: int, w: int = 64):
    """Fault-injection plan: for each trial a (stream, position, bit) triple."""
    stream = uniform_int(seed, 11, (trials,), 0, M)
    pos = uniform_int(seed, 12, (trials,), 0, positions)
    bit = uniform_int(seed, 13, (trials,), 0, w)
    return stream, pos, bit


def batch_recipe(seed: int, count: int = 256, s_min: int = 64, s_max: int = 2048,
                 kinds=(0.6, 0.3, 0.1)):
    """Mixed batch of independent problems: M uniform in {3..8}; size
    s = round(s_min * (s_max / s_min) ** u), u uniform in [0, 1); operation
    GEMM / circular convolution / permute+scale with probabilities `kinds`;
    values uniform in [-128, 128).  GEMM: M streams s x K times a shared
    K x s operand, K = s rounded up to a multiple of 16.  Convolution: M
    streams and a filter of length s.  Permute+scale: s * s positions with a
    uniform random permutation (the SplitMix64 Fisher-Yates shuffle up to
    200000 positions, numpy's seeded generator above that, for speed),
    scale and add uniform in [-128, 128).
    Returns a list of dicts of host arrays (int8 inputs, int64 scale/add)."""
    M = uniform_int(seed, 31, (count,), 3, 9)
    u = uniform_int(seed, 32, (count,), 0, 1 << 30).astype(np.float64) / float(1 << 30)
    size = np.rint(s_min * (s_max / s_min) ** u).astype(np.int64)
    kind_u = uniform_int(seed, 33, (count,), 0, 1000)
    edges = np.cumsum(np.array(kinds) * 1000).astype(np.int64)
    out = []
    for i in range(count):
        k = int(np.searchsorted(edges, kind_u[i], side="right"))
        m, s = int(M[i]), int(size[i])
        sub = seed * 1009 + i
        if k == 0:
            K = (s + 15) // 16 * 16
            c = uniform_int(sub, 1, (m, s, K), -128, 128, dtype=np.int8)
            G = uniform_int(sub, 2, (K, s), -128, 128, dtype=np.int8)
            out.append(dict(op=0, M=m, c=c, G=G))
        elif k == 1:
            c = uniform_int(sub, 3, (m, s), -128, 128, dtype=np.int8)
            g = uniform_int(sub, 4, (s,), -128, 128, dtype=np.int8)
            out.append(dict(op=1, M=m, c=c, g=g))
        else:
            n = s * s
            c = uniform_int(sub, 5, (m, n), -128, 128, dtype=np.int8)
            perm = np.random.default_rng(sub).permutation(n).astype(np.int32) if n > 200000 \
                else permutation(sub, 6, n).astype(np.int32)
            scale = uniform_int(sub, 7, (n,), -128, 128)
            add = uniform_int(sub, 8, (n,), -128, 128)
            out.append(dict(op=2, M=m, c=c, perm=perm, scale=scale, add=add))
    return out
