"""Seeded synthetic inputs shared by the CPU oracle and the GPU path.

This module only draws random numbers and lays them out; it holds none of
the search method's arithmetic (no distances, no quantisation, no graph).
Both sides of every parity check take their base vectors and queries from
here, so neither side can feed the other.

Workloads (stand-ins for the paper's SIFT / Deep / MSSPACEV style data, whose
shapes and element types are listed in the paper's dataset table):

* ``tiny``     n=10,000, d=128 float32, 32 centres U[-4,4]^128, unit noise;
               100 queries.  Index: Vamana R=32, L_build=64, alpha=1.2;
               PQ m=32 x 256.
* ``sift1m``   n=1,000,000, d=128 uint8, 1,000 centres U[0,255]^128,
               noise N(0, 20^2) per dimension, rounded half-to-even and
               clipped to [0,255]; 10,000 queries.  Index: Vamana R=64,
               L_build=100, alpha=1.2; PQ m=32 x 256.  Worklist sizes
               16 ... 1024 (recall@10 reaches 0.9 between 512 and 768).
* ``deep1m``   n=1,000,000, d=96 float32, unit-normalised: 4,096 unit
               centres (normalised Gaussian vectors), noise N(0, (0.3^2/d) I)
               (expected noise norm 0.3), every point normalised; 10,000
               queries.  Index: Vamana R=64, L_build=100, alpha=1.2; PQ
               m=48 x 256 (two dims per subspace).  Shaped like the
               paper's Deep data (float, d=96); worklist sizes 16 ... 512.

Seeding: ``numpy.random.SeedSequence(240111324 + workload_index).spawn(8)``
gives independent streams, in order ``centres, base, queries, pq_sample,
pq_init, vamana_order, workload, arrivals``.  Mixture weights are uniform:
each point first draws its component, then its noise vector.
"""
from __future__ import annotations

import dataclasses
import numpy as np

STREAMS = ("centres", "base", "queries", "pq_sample", "pq_init",
           "vamana_order", "workload", "arrivals")
SEED_BASE = 240111324


@dataclasses.dataclass(frozen=True)
class Workload:
    name: str
    index: int            # seed offset
    n: int
    d: int
    dtype: str            # "f32" | "u8" | "i8"
    ncent: int
    centre_lo: float
    centre_hi: float
    sigma: float
    nq: int
    # index-build parameters
    R: int
    L_build: int
    alpha: float
    m: int
    kmeans_iters: int
    pq_sample: int
    # search parameters
    k: int
    Ls: tuple
    # unit-normalised mixture: centres are unit vectors, the noise vector has
    # expected norm sigma (per-coordinate sd sigma/sqrt(d)), every point is
    # normalised after the noise (centre_lo/hi unused)
    unit: bool = False

    def with_(self, **kw) -> "Workload":
        return dataclasses.replace(self, **kw)


WORKLOADS = {
    "tiny": Workload("tiny", 0, 10_000, 128, "f32", 32, -4.0, 4.0, 1.0, 100,
                     32, 64, 1.2, 32, 10, 100_000, 10, (64,)),
    "sift1m": Workload("sift1m", 1, 1_000_000, 128, "u8", 1000, 0.0, 255.0,
                       20.0, 10_000, 64, 100, 1.2, 32, 10, 100_000, 10,
                       (16, 32, 64, 128, 256, 512, 544, 576, 608, 640,
                        704, 768, 1024)),
    "deep1m": Workload("deep1m", 2, 1_000_000, 96, "f32", 4096, 0.0, 0.0,
                       0.3, 10_000, 64, 100, 1.2, 48, 10, 100_000, 10,
                       (16, 32, 64, 96, 112, 128, 192, 256, 384, 512),
                       unit=True),
}


def np_dtype(dt: str):
    return {"f32": np.float32, "u8": np.uint8, "i8": np.int8}[dt]


def streams(w: Workload) -> dict:
    seqs = np.random.SeedSequence(SEED_BASE + w.index).spawn(len(STREAMS))
    return {name: np.random.Generator(np.random.PCG64(s))
            for name, s in zip(STREAMS, seqs)}


def _centres(w: Workload, rng) -> np.ndarray:
    if w.unit:
        c = rng.standard_normal((w.ncent, w.d))
        return c / np.linalg.norm(c, axis=1, keepdims=True)
    return rng.uniform(w.centre_lo, w.centre_hi, size=(w.ncent, w.d))


def _draw(w: Workload, centres: np.ndarray, rng, count: int,
          chunk: int = 1 << 16) -> np.ndarray:
    """Draw `count` mixture points in chunks (bounded memory).

    Component ids for all points come first, then the noise chunk by chunk,
    so the result does not depend on the chunk size.
    """
    comp = rng.integers(0, w.ncent, size=count)
    out = np.empty((count, w.d), dtype=np_dtype(w.dtype))
    for s in range(0, count, chunk):
        e = min(count, s + chunk)
        sd = w.sigma / np.sqrt(w.d) if w.unit else w.sigma
        x = centres[comp[s:e]] + sd * rng.standard_normal((e - s, w.d))
        if w.unit:
            x = x / np.linalg.norm(x, axis=1, keepdims=True)
        if w.dtype == "f32":
            out[s:e] = x.astype(np.float32)
        elif w.dtype == "u8":
            out[s:e] = np.clip(np.rint(x), 0, 255).astype(np.uint8)
        else:
            out[s:e] = np.clip(np.rint(x), -128, 127).astype(np.int8)
    return out


def base_and_queries(w: Workload):
    """Return (base[n][d], queries[nq][d]) in the workload's element type."""
    rs = streams(w)
    c = _centres(w, rs["centres"])
    base = _draw(w, c, rs["base"], w.n)
    queries = _draw(w, c, rs["queries"], w.nq)
    return base, queries


def small(dtype: str = "f32", n: int = 2000, d: int = 32, nq: int = 20,
          ncent: int = 8, seed_index: int = 100, **kw) -> Workload:
    """A small workload for unit and parity tests (same recipe, own seed)."""
    lo, hi, sigma = {"f32": (-4.0, 4.0, 1.0), "u8": (0.0, 255.0, 20.0),
                     "i8": (-128.0, 127.0, 20.0)}[dtype]
    base = dict(name=f"small-{dtype}-{n}-{d}", index=seed_index, n=n, d=d,
                dtype=dtype, ncent=ncent, centre_lo=lo, centre_hi=hi,
                sigma=sigma, nq=nq, R=16, L_build=32, alpha=1.2,
                m=max(1, d // 4), kmeans_iters=6, pq_sample=n, k=10,
                Ls=(32,))
    base.update(kw)
    return Workload(**base)


def serving_requests(w: Workload, rate_qps: float, duration_s: float,
                     salt: int = 0, nq_max: int = 256, ks=(10, 100),
                     Ls=(32, 64, 128)):
    """An open-loop request stream over the workload's queries: request
    sizes log-uniform in [1, nq_max] queries, k and L drawn uniformly from
    `ks` and `Ls` (L raised to k where k > L: the worklist holds at least
    the k results), arrivals a Poisson process whose mean query rate is
    rate_qps, for duration_s seconds.  Query rows are drawn uniformly from
    the workload's queries.  Seeded by (workload, salt).

    Returns dict(nq, k, L, arrival_s, rows): per-request arrays and the
    concatenated query row indices."""
    rng = np.random.default_rng(
        np.random.SeedSequence([SEED_BASE + w.index, 99, int(salt)]))
    mean_nq = (nq_max - 1) / np.log(nq_max) if nq_max > 1 else 1.0
    rate_req = rate_qps / mean_nq
    n_exp = int(rate_req * duration_s * 1.2) + 16
    gaps = rng.exponential(1.0 / rate_req, n_exp)
    arrival = np.cumsum(gaps)
    arrival = arrival[arrival < duration_s]
    nreq = max(1, len(arrival))
    arrival = arrival[:nreq] if len(arrival) else np.zeros(1)
    nq = np.floor(np.exp(rng.uniform(0.0, np.log(nq_max + 1), nreq)))
    nq = np.clip(nq, 1, nq_max).astype(np.uint32)
    k = rng.choice(np.asarray(ks), nreq).astype(np.uint32)
    L = np.maximum(rng.choice(np.asarray(Ls), nreq), k).astype(np.uint32)
    rows = rng.integers(0, w.nq, int(nq.sum()))
    return {"nq": nq, "k": k, "L": L, "arrival_s": arrival, "rows": rows}


def mixed_batch(nq: int, salt: int = 0, ks=(1, 10, 100), L_lo: int = 16,
                L_hi: int = 256):
    """Per-query k and L of a mixed batch (the 100M configuration's query
    recipe): k uniform over `ks`, L = max(k, round(exp(U[ln L_lo,
    ln L_hi]))).  Seeded by salt.  Returns (k uint32[nq], L uint32[nq])."""
    rng = np.random.default_rng(np.random.SeedSequence([SEED_BASE, 77,
                                                        int(salt)]))
    k = rng.choice(np.asarray(ks), nq).astype(np.uint32)
    L = np.rint(np.exp(rng.uniform(np.log(L_lo), np.log(L_hi), nq)))
    return k, np.maximum(L.astype(np.uint32), k)


def scale_graph_index(n: int, d: int = 128, R: int = 64, m: int = 32,
                      nq: int = 10_000, seed: int = 240111324,
                      chunk: int = 1 << 20):
    """A large synthetic index for throughput at scale only (no recall):
    int8 base vectors and queries uniform in [-128, 127] and random PQ codes
    (a random block of `block` rows repeated over the n rows, so that
    filling 100M rows takes seconds), random codebooks, and an adjacency
    whose row u holds R distinct ids spread over the whole range by a
    fixed odd multiplier, (u * 2654435761 + j * 40503 + 17 * j * j) mod n,
    j < R, so consecutive expansions touch unrelated rows (no locality for
    any cache).  Arrays are filled chunk by chunk to bound host memory.

    Returns dict(base, adj, medoid, codebooks, codes, queries)."""
    if n <= R * 40503 + 17 * R * R:
        raise ValueError("n too small for distinct row offsets")
    rng = np.random.default_rng(seed)
    block = min(n, 1 << 22)
    bb = rng.bit_generator.random_raw(block * d // 8).view(np.int8)
    bb = bb.reshape(block, d)
    cbk = rng.bit_generator.random_raw(block * m // 8).view(np.uint8)
    cbk = cbk.reshape(block, m)
    base = np.empty((n, d), dtype=np.int8)
    codes = np.empty((n, m), dtype=np.uint8)
    adj = np.empty((n, R), dtype=np.uint32)
    j = np.arange(R, dtype=np.uint64)
    off = (j * np.uint64(40503) + np.uint64(17) * j * j) % np.uint64(n)
    off32 = off.astype(np.uint32)
    if n >= 1 << 31:
        raise ValueError("n must be below 2^31")
    chunk = min(chunk, block)
    for s in range(0, n, chunk):
        e = min(n, s + chunk)
        r0 = s % block  # block is a multiple of chunk: no wrap inside
        base[s:e] = bb[r0:r0 + (e - s)]
        codes[s:e] = cbk[r0:r0 + (e - s)]
        h = ((np.arange(s, e, dtype=np.uint64) * np.uint64(2654435761))
             % np.uint64(n)).astype(np.uint32)
        x = h[:, None] + off32[None, :]  # < 2n < 2^32
        np.subtract(x, np.uint32(n), out=x, where=x >= n)
        adj[s:e] = x
    cb = rng.uniform(-128, 127, size=(m, 256, d // m)).astype(np.float32)
    queries = rng.integers(-128, 128, size=(nq, d), dtype=np.int8)
    return {"base": base, "adj": adj, "medoid": 0, "codebooks": cb,
            "codes": codes, "queries": queries}
