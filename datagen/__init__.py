"""Seeded synthetic inputs for the rANS coder: symbol arrays and their counts.

This module is shared by the tests, the benchmark and the smoke check.  It
holds none of the coder's arithmetic: it only draws i.i.d. symbols from
order-0 distributions (the paper's evaluation uses a static order-0 model per
file, Section 7) and counts them.  The paper's corpora are not used; Zipf,
"one dominant symbol", near-uniform and Dirichlet distributions over the
configured alphabets stand in for them, spanning about 0.05 to 12 bits per
symbol.

Sampling is inverse-CDF on float64 uniforms from numpy's PCG64, accelerated by
a bucket guide table; the result equals
``np.searchsorted(cdf, u, side="right")`` clipped to the alphabet.
"""
from __future__ import annotations

import math
import os
from concurrent.futures import ThreadPoolExecutor
from dataclasses import dataclass, field

import numpy as np

# ----------------------------------------------------------- distributions --


def zipf_probs(n: int, s: float) -> np.ndarray:
    """p_k proportional to (k+1)^-s, symbol 0 most frequent."""
    p = 1.0 / np.power(np.arange(1, n + 1, dtype=np.float64), s)
    return p / p.sum()


def dominant_probs(n: int, p0: float = 0.995) -> np.ndarray:
    """Symbol 0 has probability p0, the others share the rest uniformly."""
    if n == 1:
        return np.ones(1)
    p = np.full(n, (1.0 - p0) / (n - 1))
    p[0] = p0
    return p


def near_uniform_probs(n: int, rng: np.random.Generator) -> np.ndarray:
    """p_k proportional to 1 + 0.1*u_k with u_k ~ U(0,1)."""
    p = 1.0 + 0.1 * rng.random(n)
    return p / p.sum()


def gaussian_codes_probs(n: int = 256, sigma: float = 24.0) -> np.ndarray:
    """8-bit quantisation codes of normally distributed values (a symmetric
    weight tensor quantised to n levels around n/2): p_c is the normal mass
    of [c - 0.5, c + 0.5) about n/2 with standard deviation sigma (in code
    steps), the two end codes taking the tails."""
    c = np.arange(n, dtype=np.float64)
    lo = (c - 0.5 - n / 2) / (sigma * math.sqrt(2.0))
    hi = (c + 0.5 - n / 2) / (sigma * math.sqrt(2.0))
    erf = np.vectorize(math.erf)
    p = 0.5 * (erf(hi) - erf(lo))
    p[0] += 0.5 * (1.0 + math.erf(lo[0]))
    p[-1] += 0.5 * (1.0 - math.erf(hi[-1]))
    return p / p.sum()


def laplace_u16_probs(scale: float = 300.0) -> np.ndarray:
    """Signed integers d with p(d) proportional to exp(-|d| / scale) (prediction
    residuals, transform coefficients), stored as 16-bit values through the
    zigzag map d >= 0 -> 2d, d < 0 -> -2d - 1: p over 0..65535."""
    z = np.arange(65536, dtype=np.float64)
    d = np.where(z % 2 == 0, z / 2, (z + 1) / 2)
    p = np.exp(-d / scale)
    return p / p.sum()


def entropy_bits(p: np.ndarray) -> float:
    p = np.asarray(p, dtype=np.float64)
    p = p[p > 0]
    return float(-(p * np.log2(p)).sum())


# ----------------------------------------------------------------- sampling --

_BLOCK = 1 << 23
_GUIDE_BITS = 16


def _sample_block(u: np.ndarray, guide, cdf_ext, a: int, G: int) -> np.ndarray:
    s = guide[(u * G).astype(np.int64)]
    while True:
        adv = (s < a - 1) & (u >= cdf_ext[s])
        if not adv.any():
            return s
        s = s + adv


def sample(p: np.ndarray, n: int, rng: np.random.Generator, dtype=np.uint8,
           threads: int | None = None) -> np.ndarray:
    """Draws n i.i.d. symbols with probabilities p (inverse CDF).

    Block b of 2^23 symbols draws its uniforms from ``rng``'s bit generator
    jumped b+1 times, so the result does not depend on the thread count."""
    p = np.asarray(p, dtype=np.float64)
    a = len(p)
    cdf = np.cumsum(p)
    cdf /= cdf[-1]
    G = 1 << _GUIDE_BITS
    guide = np.searchsorted(cdf, np.arange(G, dtype=np.float64) / G, side="right")
    guide = np.minimum(guide, a - 1).astype(np.int64)
    cdf_ext = np.append(cdf, np.inf)
    out = np.empty(n, dtype=dtype)
    nblk = (n + _BLOCK - 1) // _BLOCK
    if nblk <= 1:
        if n:
            out[:] = _sample_block(rng.random(n), guide, cdf_ext, a, G)
        return out
    bg = rng.bit_generator

    def work(b):
        lo = b * _BLOCK
        m = min(_BLOCK, n - lo)
        g = np.random.Generator(bg.jumped(b + 1))
        out[lo:lo + m] = _sample_block(g.random(m), guide, cdf_ext, a, G)

    if threads is None:
        threads = min(8, os.cpu_count() or 1)
    with ThreadPoolExecutor(max_workers=max(1, threads)) as ex:
        list(ex.map(work, range(nblk)))
    return out


def counts(syms: np.ndarray, alphabet: int) -> np.ndarray:
    return np.bincount(np.asarray(syms).reshape(-1), minlength=alphabet).astype(np.uint64)


# ------------------------------------------------------------------ configs --


@dataclass
class Params:
    """Coder parameters: M = 2^k, b = 2^r, L = 2^l, w symbol bytes, N
    interleaved coders per chunk, C symbols per chunk (0 = one chunk)."""
    k: int
    r: int
    l: int
    w: int
    N: int
    C: int

    def astuple(self):
        return (self.k, self.r, self.l, self.w, self.N, self.C)


@dataclass
class Workload:
    name: str
    syms: np.ndarray
    alphabet: int
    params: Params
    probs: np.ndarray = field(repr=False)

    @property
    def counts(self) -> np.ndarray:
        return counts(self.syms, self.alphabet)

    @property
    def nbytes(self) -> int:
        return int(self.syms.nbytes)


def tiny_zipf(n: int = 1 << 20) -> Workload:
    """1 MiB of uint8, Zipf(1.1) over 256, M=2^12, b=L=2^16, 4 coders, one chunk."""
    rng = np.random.Generator(np.random.PCG64(1001))
    p = zipf_probs(256, 1.1)
    return Workload("zipf1.1-a256-1MiB-N4", sample(p, n, rng), 256,
                    Params(12, 16, 16, 1, 4, 0), p)


ZIPF_S = (0.8, 1.1, 1.5)


def zipf_buffer(s: float, n: int = 1 << 28) -> Workload:
    """256 MiB of uint8, Zipf(s) over 256, M=2^14, b=L=2^16, 64 KiB chunks, 64 coders."""
    idx = ZIPF_S.index(s)
    rng = np.random.Generator(np.random.PCG64(2001 + idx))
    p = zipf_probs(256, s)
    return Workload(f"zipf{s}-a256-{n >> 20}MiB-N64-C64K", sample(p, n, rng), 256,
                    Params(14, 16, 16, 1, 64, 65536), p)


SWEEP_ALPHABETS = (2, 16, 256, 4096)
SWEEP_K = (11, 15)
SWEEP_DISTS = ("dominant", "zipf1.1", "near_uniform")
SWEEP_RADIX = ((8, 23), (16, 16))
SWEEP_N = (32, 64)


def sweep_data(alphabet: int, dist: str, nbytes: int = 64 << 20):
    """64 MiB of symbol bytes (uint16 symbols for alphabets above 256)."""
    di = SWEEP_DISTS.index(dist)
    ai = SWEEP_ALPHABETS.index(alphabet)
    rng = np.random.Generator(np.random.PCG64(3000 + 3 * ai + di))
    if dist == "dominant":
        p = dominant_probs(alphabet, 0.995)
    elif dist == "zipf1.1":
        p = zipf_probs(alphabet, 1.1)
    else:
        p = near_uniform_probs(alphabet, rng)
    dt = np.uint8 if alphabet <= 256 else np.uint16
    n = nbytes // np.dtype(dt).itemsize
    return sample(p, n, rng, dt), p


def sweep_points():
    """The radix/precision sweep: 96 combinations, 12 of them infeasible
    (alphabet 4096 cannot be represented with M = 2^11)."""
    pts = []
    for a in SWEEP_ALPHABETS:
        for k in SWEEP_K:
            for dist in SWEEP_DISTS:
                for (r, l) in SWEEP_RADIX:
                    for N in SWEEP_N:
                        pts.append(dict(alphabet=a, k=k, dist=dist, r=r, l=l, N=N,
                                        w=1 if a <= 256 else 2,
                                        feasible=a <= (1 << k)))
    return pts


def dirichlet_streams(nstreams: int = 4096, lo_log2: float = 10.0, hi_log2: float = 22.0,
                    seed: int = 4001, alphabet: int = 256):
    """Independent uint8 streams with log-uniform lengths and per-stream
    Dirichlet(alpha) distributions, alpha log-uniform in [0.05, 5]."""
    ss = np.random.SeedSequence(seed)
    top = np.random.Generator(np.random.PCG64(ss))
    lens = np.floor(np.exp2(top.uniform(lo_log2, hi_log2, nstreams))).astype(np.int64)
    alphas = np.power(10.0, top.uniform(math.log10(0.05), math.log10(5.0), nstreams))
    children = ss.spawn(nstreams)

    def one(i):
        rng = np.random.Generator(np.random.PCG64(children[i]))
        p = rng.dirichlet(np.full(alphabet, alphas[i]))
        p = np.maximum(p, 0.0)
        p = p / p.sum()
        return sample(p, int(lens[i]), rng, threads=1), p

    # each stream has its own generator: the pool does not change the result
    with ThreadPoolExecutor(max_workers=min(8, os.cpu_count() or 1)) as ex:
        return list(ex.map(one, range(nstreams)))


def serving_requests(nreq: int = 1000, seed: int = 5001, lo_log2: float = 12.0,
                     hi_log2: float = 26.0):
    """Serving requests: sizes 2^U(12,26) bytes, encode/decode 50/50, per-request
    Zipf(s ~ U(0.7, 1.5)) over 256.  Returns a list of dicts with the data."""
    rng = np.random.Generator(np.random.PCG64(seed))
    sizes = np.floor(np.exp2(rng.uniform(lo_log2, hi_log2, nreq))).astype(np.int64)
    ops = rng.integers(0, 2, nreq)
    svals = rng.uniform(0.7, 1.5, nreq)
    reqs = []
    for i in range(nreq):
        p = zipf_probs(256, float(svals[i]))
        reqs.append(dict(id=i, op="encode" if ops[i] == 0 else "decode",
                         size=int(sizes[i]), s=float(svals[i]), probs=p))
    return reqs


def request_data(req: dict, seed: int = 5001) -> np.ndarray:
    rng = np.random.Generator(np.random.PCG64([seed, req["id"]]))
    return sample(req["probs"], req["size"], rng)


def requests_data(reqs, seed: int = 5001, threads: int | None = None):
    """request_data for every request, drawn on a thread pool (each request
    has its own generator, so the result does not depend on the pool)."""
    if threads is None:
        threads = min(8, os.cpu_count() or 1)
    with ThreadPoolExecutor(max_workers=max(1, threads)) as ex:
        return list(ex.map(lambda q: request_data(q, seed), reqs))
