"""CPU oracle for BANG's batched PQ greedy search (arXiv 2401.11324).

TEST INFRASTRUCTURE ONLY: the tests, the smoke check and the benchmark's
CPU-baseline leg use it; the product library never imports, links or calls
it, and it shares no code with the GPU path.

Contents (each routine cites the passage it follows in its own docstring or
in oracle.c):

* ``pq_tables``      stage 1, the PQ distance table, canonical FP32
* ``adc``            asymmetric distance, canonical FP32
* ``search``         stages 1-3: table (FP32, or the FP16 / u8 storage of
                     the precision form), greedy search (Algorithm 1, or
                     the filtered form of Algorithm 2), re-rank; or the
                     Exact-distance Version (no table, no re-rank)
* ``rerank``         stage 3 alone over given candidates
* ``pq_table_terms`` / ``bf16_table_bound``   the table in FP64 and the
                     error bound of its BF16-MFMA form (precision form)
* ``bruteforce``     exact k nearest (ground truth)
* ``train_pq`` / ``pq_encode``   PQ codebooks (k-means) and codes
* ``medoid`` / ``vamana_build`` / ``robust_prune`` / ``connect`` /
  ``reachable``      the graph index

Parity status: table, ADC, re-rank, search (every table form and the
exact-distance form) and brute force are pinned by the tests in
tests/test_oracle.py and tests/test_oracle_properties.py (closed forms,
brute force on tiny and random inputs, the paper's worked example).  The
graph build and the PQ training are inputs both paths consume; they are
pinned against plain re-statements on tiny inputs: RobustPrune by
hand-worked cases (the alpha rule, its <= boundary, ties) and the exact
greedy rule on random integer points, the whole Vamana build (sequential
insertion) against a plain re-statement, the connectivity repair and the
folding of coarse levels by hand-built graphs, and k-means by Lloyd's
algorithm written out plainly.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

from .pq import train_pq, pq_encode, kmeans_assign  # noqa: F401

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "_oracle.so")

DT = {"f32": 0, "u8": 1, "i8": 2, "f64": 3}
NONE = 0xFFFFFFFF

_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            from . import build as _b
            _b.build()
        L = ctypes.CDLL(LIB_PATH)
        P = ctypes.c_void_p
        u64, u32, f64 = ctypes.c_uint64, ctypes.c_uint32, ctypes.c_double
        L.or_pq_tables.argtypes = [P, ctypes.c_int, u64, u32, P, u32, P,
                                   ctypes.c_int]
        L.or_pq_tables.restype = None
        L.or_adc.argtypes = [P, P, u32, P, u64, P]
        L.or_adc.restype = None
        L.or_search.argtypes = [P, P, u64, u32, u32, u32, u32, ctypes.c_int,
                                ctypes.c_int, P, P, P, P, P, u32, P,
                                ctypes.c_int]
        L.or_quantize_tables.argtypes = [P, u64, u32, ctypes.c_int, P, P]
        L.or_quantize_tables.restype = None
        L.or_f32_to_f16.argtypes = [ctypes.c_float]
        L.or_f32_to_f16.restype = ctypes.c_uint16
        L.or_f16_to_f32.argtypes = [ctypes.c_uint16]
        L.or_f16_to_f32.restype = ctypes.c_float
        L.or_search.restype = ctypes.c_int
        L.or_fnv1a32.argtypes = [P, u64, u32]
        L.or_fnv1a32.restype = u32
        L.or_bloom_slots.argtypes = [u32, P, P]
        L.or_rerank.argtypes = [P, P, u64, P, u32, u32, P, P, ctypes.c_int]
        L.or_bf16_round.argtypes = [ctypes.c_float]
        L.or_bf16_round.restype = ctypes.c_float
        L.or_bf16_band.argtypes = [P, P, P, u64, P, P, P]
        L.or_rerank_bf16.argtypes = [P, P, u64, P, u32, u32, P, P, P]
        L.or_rerank.restype = ctypes.c_int
        L.or_bruteforce.argtypes = [P, ctypes.c_int, u64, u32, P, u64, u32,
                                    P, P, ctypes.c_int]
        L.or_bruteforce.restype = ctypes.c_int
        L.or_kmeans_assign.argtypes = [P, u64, u32, P, u32, P, ctypes.c_int]
        L.or_kmeans_assign.restype = f64
        L.or_pq_encode.argtypes = [P, ctypes.c_int, u64, u32, P, u32, P,
                                   ctypes.c_int]
        L.or_pq_encode.restype = None
        L.or_medoid.argtypes = [P, ctypes.c_int, u64, u32]
        L.or_medoid.restype = u32
        L.or_vamana_build.argtypes = [P, ctypes.c_int, u64, u32, u32, u32, P,
                                      ctypes.c_int, P, u32, f64, u32, P,
                                      ctypes.c_int]
        L.or_vamana_build.restype = ctypes.c_int
        L.or_robust_prune.argtypes = [P, ctypes.c_int, u64, u32, u32, P, u32,
                                      f64, u32, P]
        L.or_robust_prune.restype = ctypes.c_int64
        L.or_reachable.argtypes = [P, u64, u32, u32]
        L.or_reachable.restype = u64
        L.or_connect.argtypes = [P, ctypes.c_int, u64, u32, P, u32, u32,
                                 u32, ctypes.c_int]
        L.or_connect.restype = ctypes.c_int64
        L.or_max_threads.argtypes = []
        L.or_max_threads.restype = ctypes.c_int
        _lib = L
    return _lib


def default_threads() -> int:
    try:
        return max(1, len(os.sched_getaffinity(0)))
    except AttributeError:  # pragma: no cover
        return os.cpu_count() or 1


def _dtname(a: np.ndarray) -> str:
    return {np.dtype(np.float32): "f32", np.dtype(np.uint8): "u8",
            np.dtype(np.int8): "i8", np.dtype(np.float64): "f64"}[a.dtype]


def _p(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


class _OrIndex(ctypes.Structure):
    _fields_ = [("n", ctypes.c_uint64), ("d", ctypes.c_uint32),
                ("dtype", ctypes.c_int32), ("base", ctypes.c_void_p),
                ("R", ctypes.c_uint32), ("adj", ctypes.c_void_p),
                ("medoid", ctypes.c_uint32), ("m", ctypes.c_uint32),
                ("codebooks", ctypes.c_void_p), ("codes", ctypes.c_void_p)]


class Index:
    """Host-resident index as the oracle sees it (numpy arrays)."""

    def __init__(self, base, adj, medoid, codebooks, codes):
        self.base = np.ascontiguousarray(base)
        self.adj = np.ascontiguousarray(adj, dtype=np.uint32)
        self.medoid = int(medoid)
        self.codebooks = np.ascontiguousarray(codebooks, dtype=np.float32)
        self.codes = np.ascontiguousarray(codes, dtype=np.uint8)
        n, d = self.base.shape
        self.n, self.d = n, d
        self.R = self.adj.shape[1]
        self.m = self.codes.shape[1]
        assert self.adj.shape[0] == n and self.codes.shape[0] == n
        assert self.codebooks.shape == (self.m, 256, d // self.m)
        self.dtype = _dtname(self.base)
        self._c = _OrIndex(n, d, DT[self.dtype], self.base.ctypes.data, self.R,
                           self.adj.ctypes.data, self.medoid, self.m,
                           self.codebooks.ctypes.data, self.codes.ctypes.data)

    @property
    def cptr(self):
        return ctypes.byref(self._c)


def pq_tables(queries: np.ndarray, codebooks: np.ndarray, nthreads: int = 0):
    """Stage 1 (section "Construction of PQDistTable in Parallel"):
    T[q][j][c] = sum_t (q[j*d/m+t] - cb[j][c][t])^2, FP32 left to right."""
    q = np.ascontiguousarray(queries)
    cb = np.ascontiguousarray(codebooks, dtype=np.float32)
    nq, d = q.shape
    m = cb.shape[0]
    T = np.empty((nq, m, 256), dtype=np.float32)
    lib().or_pq_tables(_p(q), DT[_dtname(q)], nq, d, _p(cb), m, _p(T),
                       nthreads or default_threads())
    return T


def adc(table: np.ndarray, codes: np.ndarray, ids: np.ndarray) -> np.ndarray:
    """Asymmetric distance (section "Parallel Neighbour Distance
    Computation"): sum_j T[j][code[j]], FP32 left to right."""
    T = np.ascontiguousarray(table, dtype=np.float32)
    c = np.ascontiguousarray(codes, dtype=np.uint8)
    ids = np.ascontiguousarray(ids, dtype=np.uint32)
    out = np.empty(len(ids), dtype=np.float32)
    lib().or_adc(_p(T), _p(c), c.shape[1], _p(ids), len(ids), _p(out))
    return out


# "exact": no table; the search ranks by exact distances and returns the
# k first worklist entries with no re-rank (the Exact-distance Version)
TABLES = {"f32": 0, "f16": 1, "u8": 2, "exact": 3}


def iter_cap_for(L: int) -> int:
    """Safety cap on iterations per query, identical on both sides: above
    the iteration counts of the paper's worklist-size table (I <= 3.1 t)
    and of the workloads here (I ~ 1.2 L on average, 3.3 L at most)."""
    return max(4 * L, L + 64)


def quantize_tables(T: np.ndarray, table: str):
    """Reduced-precision storage of canonical FP32 tables [nq][m][256]:
    'f16' -> uint16 half bit patterns, 'u8' -> uint8 (see oracle.c)."""
    T = np.ascontiguousarray(T, dtype=np.float32)
    nq, m, _ = T.shape
    nul = ctypes.c_void_p(0)
    if table == "f16":
        out = np.empty(T.shape, dtype=np.uint16)
        lib().or_quantize_tables(_p(T), nq, m, 1, _p(out), nul)
    elif table == "u8":
        out = np.empty(T.shape, dtype=np.uint8)
        lib().or_quantize_tables(_p(T), nq, m, 2, nul, _p(out))
    else:
        raise ValueError(table)
    return out


# visited filters of the search (oracle.c greedy_search): Algorithm 1's
# set union, Algorithm 2 with an exact seen-set, Algorithm 2 with the
# paper's Bloom filter
MODES = {"union": 0, "exact": 1, "bloom": 2}
BLOOM_Z = 399887


def fnv1a32(data: bytes, basis: int = 0x811C9DC5) -> int:
    """FNV-1a-32 of a byte string (oracle.c or_fnv1a32)."""
    buf = ctypes.create_string_buffer(bytes(data), max(1, len(data)))
    return int(lib().or_fnv1a32(ctypes.cast(buf, ctypes.c_void_p),
                                len(data), basis))


def bloom_slots(x: int):
    """The two Bloom-filter entries of node x (oracle.c or_bloom_slots)."""
    h1, h2 = ctypes.c_uint32(), ctypes.c_uint32()
    lib().or_bloom_slots(x, ctypes.byref(h1), ctypes.byref(h2))
    return int(h1.value), int(h2.value)


def search(index: Index, queries: np.ndarray, k: int, L: int,
           c_max: int | None = None, iter_cap: int | None = None,
           mode: int = 0, want_pq: bool = False, want_cand: bool = False,
           table: str = "f32", nthreads: int = 0):
    """Stages 1-3 for a batch (Algorithms 1 and 2, sections on the PQ
    table, re-ranking).  `table` picks the table storage the search ranks
    by: "f32" (canonical), "f16" or "u8" (the precision form, oracle.c),
    or "exact": exact distances in the search and no re-rank (section
    "Implementation Variants", Exact-distance Version).  `mode` picks
    the visited filter (MODES: 0 Algorithm 1's set union, 1 Algorithm 2
    with an exact seen-set, 2 Algorithm 2 with the paper's Bloom filter).
    Returns a dict with ids, dists and, on request,
    pq_ids/pq_dists (Algorithm 1's own top-k), cand (expanded nodes in
    expansion order, NONE padded) and counters [I, status, added]."""
    q = np.ascontiguousarray(queries, dtype=index.base.dtype)
    nq = q.shape[0]
    c_max = 4 * L if c_max is None else c_max
    iter_cap = iter_cap_for(L) if iter_cap is None else iter_cap
    ids = np.empty((nq, k), dtype=np.uint32)
    dists = np.empty((nq, k), dtype=np.float32)
    pq_ids = np.empty((nq, k), dtype=np.uint32) if want_pq else None
    pq_d = np.empty((nq, k), dtype=np.float32) if want_pq else None
    cand = np.empty((nq, iter_cap), dtype=np.uint32) if want_cand else None
    counters = np.empty((nq, 4), dtype=np.uint32)
    nul = ctypes.c_void_p(0)
    rc = lib().or_search(
        index.cptr, _p(q), nq, k, L, c_max, iter_cap, mode, TABLES[table],
        _p(ids),
        _p(dists), _p(pq_ids) if want_pq else nul,
        _p(pq_d) if want_pq else nul, _p(cand) if want_cand else nul,
        iter_cap, _p(counters), nthreads or default_threads())
    if rc != 0:
        raise ValueError(f"or_search failed ({rc})")
    out = {"ids": ids, "dists": dists,
           "iters": counters[:, 0].copy(), "status": counters[:, 1].copy(),
           "added": counters[:, 2].astype(np.uint64)
           | (counters[:, 3].astype(np.uint64) << np.uint64(32))}
    if want_pq:
        out["pq_ids"], out["pq_dists"] = pq_ids, pq_d
    if want_cand:
        out["cand"] = cand
    return out


def rerank(index: Index, queries: np.ndarray, cand: np.ndarray, k: int,
           nthreads: int = 0):
    """Stage 3 alone (section "Re-ranking"): exact distances of the given
    candidates, sorted by (distance, id), top-k; NONE or ids >= n skipped."""
    q = np.ascontiguousarray(queries, dtype=index.base.dtype)
    cand = np.ascontiguousarray(cand, dtype=np.uint32)
    nq, cm = cand.shape
    ids = np.empty((nq, k), dtype=np.uint32)
    dists = np.empty((nq, k), dtype=np.float32)
    lib().or_rerank(index.cptr, _p(q), nq, _p(cand), cm, k, _p(ids),
                    _p(dists), nthreads or default_threads())
    return ids, dists


def bf16_round(x: float) -> float:
    """x rounded to bfloat16 (nearest, ties to even), as a float."""
    return float(lib().or_bf16_round(float(x)))


def bf16_round_array(x: np.ndarray) -> np.ndarray:
    """Every element rounded to bfloat16 (nearest, ties to even), as FP64:
    the nearest number with an 8-bit significand, found from the FP64
    significand scaled to 8 integer bits and rounded half to even.  Finite
    inputs in the normal range of bfloat16 (every table input here)."""
    x = np.asarray(x, dtype=np.float64)
    m, e = np.frexp(x)                 # x = m * 2^e, 0.5 <= |m| < 1
    return np.ldexp(np.rint(np.ldexp(m, 8)), e - 8)


# unit roundoffs: bfloat16 (8-bit significand) and FP32 (24-bit)
BF16_U = 2.0 ** -8
FP32_U = 2.0 ** -24


def pq_table_terms(queries: np.ndarray, codebooks: np.ndarray):
    """The PQ table of section "Construction of PQDistTable in Parallel" in
    FP64 with the sums its error bounds need, per (query, subspace j,
    centroid c) with t over the subspace's coordinates: T = sum (q_t -
    c_t)^2 (exact to FP64 rounding), S_qc = sum |q_t c_t|, S_qq = sum q_t^2,
    S_cc = sum c_t^2, and T_b = |q|^2 + |c|^2 - 2 sum bf16(q_t) bf16(c_t),
    the table with both factors of the inner product rounded to bfloat16.
    Each [nq][m][256]."""
    q = np.asarray(queries, dtype=np.float64)
    cb = np.asarray(codebooks, dtype=np.float64)      # [m][256][ds]
    m, _, ds = cb.shape
    qs = q.reshape(q.shape[0], m, 1, ds)
    cs = cb[None]
    T = ((qs - cs) ** 2).sum(-1)
    S_qc = np.abs(qs * cs).sum(-1)
    S_qq = (qs ** 2).sum(-1) + 0.0 * S_qc
    S_cc = (cs ** 2).sum(-1) + 0.0 * S_qc
    Tb = S_qq + S_cc - 2.0 * (bf16_round_array(qs) *
                              bf16_round_array(cs)).sum(-1)
    return T, S_qc, S_qq, S_cc, Tb


def bf16_table_bound(queries: np.ndarray, codebooks: np.ndarray):
    """(T, E): the exact table and a bound E on |T~ - T| for the table
    built by BF16 MFMA with FP32 accumulation, T~ = fl(fl(|q|^2 + |c|^2) -
    2 X~), where |q|^2 and |c|^2 are FP32 sums of the unrounded
    coordinates and X~ the FP32-accumulated inner product of the
    coordinates rounded to bfloat16.  With u = 2^-8 and v = 2^-24:
      * rounding both factors: |bf16(q)bf16(c) - qc| <= (2u + u^2)|qc|;
      * the products are exact in FP32 (8-bit significands) and their
        ds-term sum, in any order, errs by at most g S~ with g = (ds+1) v
        and S~ <= (1 + u)^2 S_qc;
      * each norm errs by at most g times itself, their sum and the last
        subtraction by v times their magnitudes (<= S_qq + S_cc + 2 S~).
    So E = 2 (2u + u^2 + g (1 + u)^2) S_qc + g (S_qq + S_cc)
           + 2 v (S_qq + S_cc + 2 (1 + u)^2 S_qc), doubled for margin in
    the FP32 terms only."""
    T, S_qc, S_qq, S_cc, _ = pq_table_terms(queries, codebooks)
    ds = np.asarray(codebooks).shape[2]
    u, v = BF16_U, FP32_U
    g = (ds + 1) * v
    w = (1.0 + u) ** 2
    E = (2.0 * (2.0 * u + u * u) * S_qc
         + 2.0 * (2.0 * g * w * S_qc + g * (S_qq + S_cc)
                  + 2.0 * v * (S_qq + S_cc + 2.0 * w * S_qc)))
    return T, E


def bf16_band(index: Index, query: np.ndarray, ids: np.ndarray):
    """The BF16 re-rank's terms for candidates `ids` of one float query:
    (D~ the FP32 distance over BF16-rounded rows, lower, upper) with the
    canonical FP32 distance guaranteed inside [lower, upper]."""
    q = np.ascontiguousarray(query, dtype=np.float32)
    ids = np.ascontiguousarray(ids, dtype=np.uint32)
    n = len(ids)
    out = [np.empty(n, dtype=np.float32) for _ in range(3)]
    lib().or_bf16_band(index.cptr, _p(q), _p(ids), n, *(_p(a) for a in out))
    return tuple(out)


def rerank_bf16(index: Index, queries: np.ndarray, cand: np.ndarray, k: int):
    """The precision form's re-rank of float data: BF16 rows and FP32 sums,
    then the canonical FP32 distance for every candidate whose lower bound
    is within the k-th smallest upper bound.  Returns (ids, dists,
    rechecked per query); ids and dists equal rerank()'s."""
    q = np.ascontiguousarray(queries, dtype=np.float32)
    cand = np.ascontiguousarray(cand, dtype=np.uint32)
    nq, cm = cand.shape
    ids = np.empty((nq, k), dtype=np.uint32)
    dists = np.empty((nq, k), dtype=np.float32)
    rc = np.empty(nq, dtype=np.uint32)
    if lib().or_rerank_bf16(index.cptr, _p(q), nq, _p(cand), cm, k, _p(ids),
                            _p(dists), _p(rc)) != 0:
        raise ValueError("the BF16 re-rank needs float data")
    return ids, dists, rc


def bruteforce(base: np.ndarray, queries: np.ndarray, k: int,
               nthreads: int = 0):
    """Exact k nearest by (squared L2, id): int64-exact for integer data,
    FP64 for float data.  Returns (ids uint32, dists float64)."""
    b = np.ascontiguousarray(base)
    q = np.ascontiguousarray(queries, dtype=b.dtype)
    n, d = b.shape
    nq = q.shape[0]
    ids = np.empty((nq, k), dtype=np.uint32)
    dists = np.empty((nq, k), dtype=np.float64)
    rc = lib().or_bruteforce(_p(b), DT[_dtname(b)], n, d, _p(q), nq, k,
                             _p(ids), _p(dists), nthreads or default_threads())
    if rc != 0:
        raise ValueError("or_bruteforce failed")
    return ids, dists


def medoid(base: np.ndarray) -> int:
    """Start node: the point nearest the mean (FP64), ties to the lowest id
    (the paper only says it is fixed at build time)."""
    b = np.ascontiguousarray(base)
    n, d = b.shape
    return int(lib().or_medoid(_p(b), DT[_dtname(b)], n, d))


def vamana_build(base: np.ndarray, R: int, L_build: int, alpha: float,
                 perm: np.ndarray, start: int, passes: int = 2,
                 slack: float = 1.3, max_batch_frac: float = 0.02,
                 nthreads: int = 0) -> np.ndarray:
    """Vamana graph: pass 1 with alpha=1, pass 2 with the given alpha, over
    the insertion order `perm`.  Returns adj[n][R] uint32, NONE padded."""
    b = np.ascontiguousarray(base)
    n, d = b.shape
    alphas = np.array([1.0, alpha][-passes:] if passes <= 2 else
                      [1.0] * (passes - 1) + [alpha], dtype=np.float64)
    perm = np.ascontiguousarray(perm, dtype=np.uint32)
    assert perm.shape == (n,)
    adj = np.empty((n, R), dtype=np.uint32)
    max_batch = max(1, int(n * max_batch_frac))
    rc = lib().or_vamana_build(_p(b), DT[_dtname(b)], n, d, R, L_build,
                               _p(alphas), len(alphas), _p(perm), start,
                               slack, max_batch, _p(adj),
                               nthreads or default_threads())
    if rc != 0:
        raise MemoryError("or_vamana_build failed")
    return adj


def robust_prune(base: np.ndarray, p: int, cand, alpha: float,
                 R: int) -> np.ndarray:
    """RobustPrune(p, cand, alpha, R) of the Vamana build (oracle.c
    robust_prune): candidates in (distance to p, id) order, p and repeats
    dropped; the nearest remaining one is kept and every remaining p' with
    alpha * d(p*, p') <= d(p, p') (plain Euclidean distances) is dropped,
    until R are kept.  Returns the kept ids in selection order."""
    b = np.ascontiguousarray(base)
    n, d = b.shape
    c = np.ascontiguousarray(cand, dtype=np.uint32)
    out = np.empty(max(1, R), dtype=np.uint32)
    no = lib().or_robust_prune(_p(b), DT[_dtname(b)], n, d, int(p), _p(c),
                               len(c), float(alpha), R, _p(out))
    if no < 0:
        raise MemoryError("or_robust_prune failed")
    return out[:no].copy()


def connect(base: np.ndarray, adj: np.ndarray, start: int, L_build: int,
            max_rounds: int = 8) -> int:
    """Connectivity repair in place (oracle.c or_connect): every node not
    reachable from `start` gets an in-edge from the nearest node that the
    build's greedy search toward it expands.  Returns the edges added."""
    b = np.ascontiguousarray(base)
    assert adj.flags["C_CONTIGUOUS"] and adj.dtype == np.uint32
    n, R = adj.shape
    return int(lib().or_connect(_p(b), DT[_dtname(b)], n, b.shape[1],
                                _p(adj), R, start, L_build, max_rounds))


def reachable(adj: np.ndarray, start: int) -> int:
    a = np.ascontiguousarray(adj, dtype=np.uint32)
    n, R = a.shape
    return int(lib().or_reachable(_p(a), n, R, start))
