"""Seeded synthetic inputs for the multisplit workloads.

This module only *draws* inputs: it holds none of the multisplit arithmetic
(no bucket identification, no counting, no permutation).  Both the CPU oracle
tests and the GPU path take their inputs from here, so the two sides see the
same bytes.

Generator: SplitMix64 (Steele, Lea and Flood, "Fast splittable pseudorandom
number generators", OOPSLA 2014).  It is counter based: draw ``i`` of the
stream with seed ``s`` is ``mix(s + (i + 1) * GAMMA)``, so any slice of a
stream can be produced independently and in parallel.  A uint32 draw is the
high 32 bits of the 64-bit output; a double in [0, 1) is the top 53 bits
times 2^-53.

Workload shapes follow the paper's experimental setup (Section 6: 32-bit keys
drawn uniformly so every bucket expects the same count; Section 6.4 binomial
and alpha-uniform bucket skews) plus the synthetic range/lognormal and batched
workloads that stand beside the plain method.
"""
from __future__ import annotations

import os
from concurrent.futures import ThreadPoolExecutor

import numpy as np

GAMMA = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)
_CHUNK = 1 << 22


def _mix(z: np.ndarray) -> np.ndarray:
    """SplitMix64 output function, in place on a uint64 array."""
    with np.errstate(over="ignore"):
        z ^= z >> np.uint64(30)
        z *= _M1
        z ^= z >> np.uint64(27)
        z *= _M2
        z ^= z >> np.uint64(31)
    return z


def splitmix64(seed: int, count: int, start: int = 0) -> np.ndarray:
    """Draws ``start .. start+count-1`` of the SplitMix64 stream for ``seed``."""
    out = np.empty(count, dtype=np.uint64)
    s = np.uint64(seed & 0xFFFFFFFFFFFFFFFF)
    with np.errstate(over="ignore"):
        for lo in range(0, count, _CHUNK):
            hi = min(count, lo + _CHUNK)
            z = np.arange(start + lo + 1, start + hi + 1, dtype=np.uint64)
            z *= GAMMA
            z += s
            out[lo:hi] = _mix(z)
    return out


def _threads() -> int:
    return max(1, min(16, os.cpu_count() or 1))


def _chunked(n: int, fill) -> None:
    """Calls fill(lo, hi) over chunks of [0, n), in parallel threads when n is
    large (numpy releases the interpreter lock inside its array loops).  The
    draws are counter based, so the result does not depend on the split."""
    spans = [(lo, min(n, lo + _CHUNK)) for lo in range(0, n, _CHUNK)]
    if len(spans) <= 1:
        for lo, hi in spans:
            fill(lo, hi)
        return
    with ThreadPoolExecutor(_threads()) as ex:
        list(ex.map(lambda sp: fill(*sp), spans))


def uniform_u32(seed: int, n: int) -> np.ndarray:
    """n uint32 keys uniform over [0, 2^32)."""
    out = np.empty(n, dtype=np.uint32)

    def fill(lo, hi):
        out[lo:hi] = (splitmix64(seed, hi - lo, lo) >> np.uint64(32)).astype(np.uint32)
    _chunked(n, fill)
    return out


def uniform_f64(seed: int, n: int, start: int = 0) -> np.ndarray:
    """n doubles in [0, 1) from the top 53 bits of each draw."""
    return (splitmix64(seed, n, start) >> np.uint64(11)).astype(np.float64) * (2.0 ** -53)


def index_values(n: int) -> np.ndarray:
    """Values equal to the original index (makes stability observable)."""
    return np.arange(n, dtype=np.uint32)


def lognormal_u32(seed: int, n: int, mu: float = 20.0, sigma: float = 2.0) -> np.ndarray:
    """floor(exp(mu + sigma*z)) saturated to [0, 2^32-1]; z standard normal.

    z comes from Box-Muller on draws 2i and 2i+1: z = sqrt(-2 ln(1-u1)) cos(2 pi u2).
    """
    out = np.empty(n, dtype=np.uint32)

    def fill(lo, hi):
        u = uniform_f64(seed, 2 * (hi - lo), 2 * lo)
        u1, u2 = u[0::2], u[1::2]
        z = np.sqrt(-2.0 * np.log1p(-u1)) * np.cos(2.0 * np.pi * u2)
        v = np.floor(np.exp(mu + sigma * z))
        v = np.minimum(v, 4294967295.0)
        out[lo:hi] = v.astype(np.uint32)
    _chunked(n, fill)
    return out


def quantile_splitters(sample: np.ndarray, m: int) -> np.ndarray:
    """m-1 ascending splitters at the i/m quantiles of a sorted sample.

    spl[i-1] = S[i * len(S) // m] for i = 1..m-1 (duplicates are kept).
    """
    s = np.sort(sample.astype(np.uint32), kind="stable")
    idx = (np.arange(1, m, dtype=np.int64) * len(s)) // m
    return s[idx].astype(np.uint32)


def skewed_bucket_keys(seed: int, n: int, m: int, dist: str, alpha: float = 0.25,
                       p: float = 0.5) -> np.ndarray:
    """Keys whose delta bucket k >> (32 - log2 m) follows a chosen distribution.

    dist = "uniform":   bucket uniform over [0, m)
    dist = "binomial":  bucket ~ B(m-1, p) (Section 6.4): for p = 1/2 the
                        number of set bits among m-1 uniform random bits
                        (ceil((m-1)/64) draws per key, draw W*i + w for
                        word w of key i, bits above m-1 cleared), otherwise
                        a sum of m-1 Bernoulli(p) trials
    dist = "alpha":     with probability alpha the bucket is uniform, else it
                        is one fixed bucket drawn from the seed (alpha-uniform)
    The low bits inside the bucket are uniform.  m must be a power of two.
    """
    r = int(m).bit_length() - 1
    assert 1 << r == m and 1 <= m <= 256
    shift = 32 - r
    low = uniform_u32(seed ^ 0x5A5A5A5A, n)
    low = low & np.uint32((1 << shift) - 1) if shift < 32 else low
    if dist == "uniform":
        b = (uniform_u32(seed, n).astype(np.uint64) * np.uint64(m)) >> np.uint64(32)
    elif dist == "binomial" and p == 0.5:
        trials = m - 1
        words = max(1, -(-trials // 64))
        top = trials - 64 * (words - 1)
        top_mask = np.uint64((1 << top) - 1) if top < 64 else np.uint64(0xFFFFFFFFFFFFFFFF)
        b = np.zeros(n, dtype=np.int64)

        def fill(lo, hi):
            w = splitmix64(seed + 7919, words * (hi - lo), words * lo).reshape(hi - lo, words)
            w[:, words - 1] &= top_mask
            b[lo:hi] = np.bitwise_count(w).sum(axis=1, dtype=np.int64)
        if trials > 0:
            _chunked(n, fill)
    elif dist == "binomial":
        b = np.zeros(n, dtype=np.int64)
        trials = m - 1
        for t in range(trials):
            u = uniform_f64(seed + 7919 * (t + 1), n)
            b += (u < p)
    elif dist == "alpha":
        u = uniform_f64(seed, n)
        unif = (uniform_u32(seed + 1, n).astype(np.uint64) * np.uint64(m)) >> np.uint64(32)
        fixed = int((int(uniform_u32(seed + 2, 1)[0]) * m) >> 32)
        b = np.where(u < alpha, unif, np.uint64(fixed))
    else:
        raise ValueError(dist)
    b = b.astype(np.uint64)
    if shift == 32:
        return low.astype(np.uint32)
    return ((b << np.uint64(shift)) | low.astype(np.uint64)).astype(np.uint32)


def batched_sizes(seed: int, num: int, lo_log2: int = 8, hi_log2: int = 20) -> np.ndarray:
    """Instance sizes log-uniform in [2^lo, 2^hi]: floor(2^(lo + (hi-lo) u)), clamped."""
    u = uniform_f64(seed, num)
    s = np.floor(np.exp2(lo_log2 + (hi_log2 - lo_log2) * u)).astype(np.int64)
    return np.clip(s, 1 << lo_log2, 1 << hi_log2)


def segment_offsets(sizes: np.ndarray) -> np.ndarray:
    """num+1 uint64 offsets of instances concatenated in index order."""
    seg = np.zeros(len(sizes) + 1, dtype=np.uint64)
    np.cumsum(sizes, out=seg[1:])
    return seg


def batched_pairs(seed: int, sizes: np.ndarray):
    """Concatenated keys (uniform) and values (index within instance)."""
    total = int(np.sum(sizes))
    keys = np.empty(total, dtype=np.uint32)
    vals = np.empty(total, dtype=np.uint32)
    starts = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)

    def fill(i):
        pos, s = int(starts[i]), int(sizes[i])
        keys[pos:pos + s] = uniform_u32(seed * 1000 + i, s)
        vals[pos:pos + s] = np.arange(s, dtype=np.uint32)
    with ThreadPoolExecutor(_threads()) as ex:
        list(ex.map(fill, range(len(sizes))))
    return keys, vals


def rmat_graph(seed: int, scale: int, n_edges: int, a: float = 0.5, b: float = 0.1,
               c: float = 0.1, max_weight: int = 1000):
    """Undirected R-MAT graph (Chakrabarti, Zhan and Faloutsos, SDM 2004) in
    directed CSR form, each edge stored in both directions.

    Edge e picks its endpoints by ``scale`` recursive quadrant choices on the
    2^scale x 2^scale adjacency matrix, most significant bit first, with draw
    ``l * n_edges + e`` of the stream at level l: top-left with probability
    a, top-right b, bottom-left c, bottom-right 1 - a - b - c.  Its weight is
    floor(u * (max_weight + 1)) for the draw ``scale * n_edges + e``, an
    integer uniform in [0, max_weight].  Self loops are dropped; repeated
    edges are kept.  Rows list their edges in generation order (forward
    directions first, then reverse ones).

    Returns (row uint64[nv + 1], col uint32[ne], wt uint32[ne]), nv = 2^scale.
    """
    nv = 1 << scale
    src = np.zeros(n_edges, dtype=np.int64)
    dst = np.zeros(n_edges, dtype=np.int64)
    for level in range(scale):
        r = uniform_f64(seed, n_edges, start=level * n_edges)
        src = 2 * src + (r >= a + b)
        dst = 2 * dst + (((r >= a) & (r < a + b)) | (r >= a + b + c))
    w = np.floor(uniform_f64(seed, n_edges, start=scale * n_edges) * (max_weight + 1))
    w = w.astype(np.int64)
    keep = src != dst
    s = np.concatenate([src[keep], dst[keep]])
    d = np.concatenate([dst[keep], src[keep]])
    ww = np.concatenate([w[keep], w[keep]])
    order = np.argsort(s, kind="stable")
    row = np.zeros(nv + 1, dtype=np.uint64)
    np.cumsum(np.bincount(s, minlength=nv), out=row[1:])
    return row, d[order].astype(np.uint32), ww[order].astype(np.uint32)
