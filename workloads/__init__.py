"""Seeded synthetic inputs shared by the tests, the smoke check and the bench.

This module holds data generators only: no sorting, no run detection, no
powers, no model.  Both the GPU path and the CPU oracle receive the same
arrays from here.  The shapes follow the paper's workloads (Section 5,
"Input permutations": presorted runs of geometric length) and the five
benchmark configurations of this project:

  uniform32      n = 2^16 uint32, uniform
  presorted64    n = 2^24 uint64, runs of length 1 + Geom(2^-10) (mean 2^10),
                 10% of runs descending, then floor(0.01 n) random swaps
  mixture64      n = 2^28 uint64: 50% uniform, 30% Zipf(s=1.1) over 2^20 ranks,
                 20% normal clusters (64 centres, sigma = 2^40)
  batch32        4096 uint32 arrays, lengths floor(2^(6+14U)) in [64, 2^20],
                 even arrays uniform, odd arrays Zipf(1.1)
  lognormal64    n = 2^28 uint64 keys floor(exp(2 N(0,1)) 2^40), saturated
  dup16_64       keys drawn uniformly from 16 distinct lognormal values
  paper(S)       the paper's generator: n ~ U[0.9N, N], values U[100, 1e9],
                 runs of geometric length with parameter 1/S
"""
from __future__ import annotations

import numpy as np

U64_MAX = np.uint64(0xFFFFFFFFFFFFFFFF)


def _rng(seed: int) -> np.random.Generator:
    return np.random.default_rng(seed)


def _finalize(x: np.ndarray) -> np.ndarray:
    """SplitMix64 output mixing (a bijection on 64-bit words)."""
    x = x.astype(np.uint64, copy=True)
    with np.errstate(over="ignore"):
        x ^= x >> np.uint64(30)
        x *= np.uint64(0xBF58476D1CE4E5B9)
        x ^= x >> np.uint64(27)
        x *= np.uint64(0x94D049BB133111EB)
        x ^= x >> np.uint64(31)
    return x


def uniform(n: int, bits: int, seed: int) -> np.ndarray:
    g = _rng(seed)
    if bits == 32:
        return g.integers(0, 2**32, size=n, dtype=np.uint64).astype(np.uint32)
    return g.integers(0, 2**64, size=n, dtype=np.uint64, endpoint=False)


def zipf_ranks(n: int, s: float, nranks: int, g: np.random.Generator) -> np.ndarray:
    """Ranks 1..nranks with P(r) proportional to r^-s (inverse CDF)."""
    w = np.arange(1, nranks + 1, dtype=np.float64) ** (-s)
    cdf = np.cumsum(w)
    cdf /= cdf[-1]
    u = g.random(n)
    return (np.searchsorted(cdf, u, side="right") + 1).astype(np.uint64)


def presorted(n: int, seed: int, mean_run: int = 1024, desc_frac: float = 0.1,
              swap_frac: float = 0.01, bits: int = 64) -> np.ndarray:
    g = _rng(seed)
    x = uniform(n, bits, seed + 1000003)
    pos = 0
    p = 1.0 / mean_run
    while pos < n:
        ln = int(g.geometric(p))  # numpy counts trials (>= 1): 1 + Geom0(p), mean 1/p
        end = min(n, pos + ln)
        seg = np.sort(x[pos:end], kind="stable")
        if g.random() < desc_frac:
            seg = seg[::-1]
        x[pos:end] = seg
        pos = end
    ns = int(swap_frac * n)
    if ns:
        a = g.integers(0, n, size=ns)
        b = g.integers(0, n, size=ns)
        for i, j in zip(a.tolist(), b.tolist()):
            x[i], x[j] = x[j], x[i]
    return x


def mixture(n: int, seed: int) -> np.ndarray:
    g = _rng(seed)
    comp = g.random(n)
    out = g.integers(0, 2**64, size=n, dtype=np.uint64, endpoint=False)
    zmask = (comp >= 0.5) & (comp < 0.8)
    nz = int(zmask.sum())
    if nz:
        out[zmask] = _finalize(zipf_ranks(nz, 1.1, 1 << 20, g))
    cmask = comp >= 0.8
    nc = int(cmask.sum())
    if nc:
        centres = g.integers(0, 2**64, size=64, dtype=np.uint64, endpoint=False)
        which = g.integers(0, 64, size=nc)
        off = np.rint(g.standard_normal(nc) * 2.0**40)
        # exact integer arithmetic for the offset, saturating at the ends
        c = centres[which]
        offi = off.astype(np.int64)
        neg = offi < 0
        mag = np.abs(offi).astype(np.uint64)
        res = c.copy()
        with np.errstate(over="ignore"):
            up = ~neg
            res[up] = np.where(c[up] > U64_MAX - mag[up], U64_MAX, c[up] + mag[up])
            res[neg] = np.where(c[neg] < mag[neg], np.uint64(0), c[neg] - mag[neg])
        out[cmask] = res
    return out


def lognormal(n: int, seed: int, sigma: float = 2.0, scale_log2: int = 40) -> np.ndarray:
    g = _rng(seed)
    v = np.exp(sigma * g.standard_normal(n)) * (2.0 ** scale_log2)
    out = np.empty(n, dtype=np.uint64)
    big = v >= 2.0**64
    out[big] = U64_MAX
    out[~big] = np.floor(v[~big]).astype(np.uint64)
    return out


def dup16(n: int, seed: int, every_16: bool = False) -> np.ndarray:
    """Adversarial input: 16 distinct values (uniform choice), or each value
    repeated exactly 16 times (every_16=True)."""
    g = _rng(seed)
    if every_16:
        vals = lognormal(max(1, n // 16 + 1), seed + 7)
        out = np.repeat(vals, 16)[:n]
        g.shuffle(out)
        return out
    vals = np.unique(lognormal(64, seed + 7))[:16]
    return vals[g.integers(0, vals.size, size=n)]


def batch_lengths(nseg: int, seed: int, lo_log2: int = 6, hi_log2: int = 20) -> np.ndarray:
    g = _rng(seed)
    u = g.random(nseg)
    L = np.floor(2.0 ** (lo_log2 + (hi_log2 - lo_log2) * u)).astype(np.int64)
    return np.clip(L, 1 << lo_log2, 1 << hi_log2)


def batch32(nseg: int, seed: int, lengths: np.ndarray | None = None):
    """(keys uint32, offsets int64[nseg+1]) for the segmented workload."""
    g = _rng(seed + 17)
    L = batch_lengths(nseg, seed) if lengths is None else np.asarray(lengths, dtype=np.int64)
    off = np.zeros(L.size + 1, dtype=np.int64)
    np.cumsum(L, out=off[1:])
    keys = np.empty(int(off[-1]), dtype=np.uint32)
    for i in range(L.size):
        a, b = int(off[i]), int(off[i + 1])
        if i % 2 == 0:
            keys[a:b] = g.integers(0, 2**32, size=b - a, dtype=np.uint64).astype(np.uint32)
        else:
            keys[a:b] = (_finalize(zipf_ranks(b - a, 1.1, 1 << 20, g)) & np.uint64(0xFFFFFFFF)).astype(np.uint32)
    return keys, off


def paper_workload(seed: int, S: int, N: int = 10**7, n: int | None = None) -> np.ndarray:
    """Section 5's generator with our own PRNG: n ~ U[0.9N, N], values
    U[100, 1e9] as uint32, presorted runs of geometric length (parameter 1/S)."""
    g = _rng(seed)
    if n is None:
        n = int(g.integers(int(0.9 * N), N + 1))
    x = g.integers(100, 10**9 + 1, size=n, dtype=np.int64).astype(np.uint32)
    pos = 0
    while pos < n:
        ln = int(g.geometric(1.0 / S)) if S > 1 else 1
        end = min(n, pos + ln)
        x[pos:end] = np.sort(x[pos:end])
        pos = end
    return x
