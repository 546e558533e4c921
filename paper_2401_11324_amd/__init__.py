"""MI355X-native batched PQ graph search (BANG, arXiv 2401.11324).

Thin Python binding over the C ABI in include/bang.h (library
``_bang.so`` next to this file).  Every step of the search runs in the
library's HIP kernels; this module only marshals arguments: numpy arrays
for the index description, torch CUDA tensors for queries and outputs, and
the current torch stream.  There is no fallback: if the library is missing
or no GPU is usable, calls raise.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "_bang.so")

BANG_NONE = 0xFFFFFFFF
MAX_L = 1024
MAX_R = 64
DTYPES = {"f32": 0, "u8": 1, "i8": 2}
TABLES = {"f32": 0, "f16": 1, "u8": 2, "exact": 3}
INDEX_HOST_ADJ = 1
INDEX_BF16_BASE = 2
# re-rank forms (bang.h BANG_RERANK_*)
RERANKS = {"exact": 0, "bf16": 1}
# visited filters (bang.h BANG_FILTER_*)
FILTERS = {"exact": 0, "bloom": 1, "seen": 2}
ERRORS = {-1: "EINVAL", -2: "ENOMEM", -3: "EDEVICE", -4: "EUNSUPPORTED",
          -5: "EABORTED"}
EXPORTS = ("bang_index_create", "bang_index_destroy", "bang_build_pq_tables",
           "bang_build_pq_tables_bf16", "bang_search", "bang_search_noalloc",
           "bang_rerank",
           "bang_index_probe",
           "bang_server_create",
           "bang_server_destroy", "bang_server_submit", "bang_server_wait",
           "bang_server_replay", "bang_server_stats", "bang_abort_create",
           "bang_abort_destroy", "bang_abort_set", "bang_abort_clear",
           "bang_abort_status", "bang_last_error")


class BangError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{ERRORS.get(code, code)}: {msg}")
        self.code = code


class IndexDesc(ctypes.Structure):
    _fields_ = [("n", ctypes.c_uint64), ("d", ctypes.c_uint32),
                ("dtype", ctypes.c_int32), ("base", ctypes.c_void_p),
                ("R", ctypes.c_uint32), ("adj", ctypes.c_void_p),
                ("medoid", ctypes.c_uint32), ("m", ctypes.c_uint32),
                ("codebooks", ctypes.c_void_p), ("codes", ctypes.c_void_p),
                ("flags", ctypes.c_uint32)]


class SearchOpts(ctypes.Structure):
    _fields_ = [("c_max", ctypes.c_uint32), ("iter_cap", ctypes.c_uint32),
                ("out_cand", ctypes.c_void_p), ("cand_stride", ctypes.c_uint32),
                ("out_counters", ctypes.c_void_p),
                ("out_times", ctypes.c_void_p),
                ("table", ctypes.c_uint32), ("flags", ctypes.c_uint32),
                ("query_L", ctypes.c_void_p), ("query_k", ctypes.c_void_p),
                ("filter", ctypes.c_uint32), ("out_phases", ctypes.c_void_p),
                ("abort", ctypes.c_void_p), ("rerank", ctypes.c_uint32),
                ("tables", ctypes.c_void_p), ("order", ctypes.c_void_p),
                ("waves_per_cu", ctypes.c_uint32)]


class ServerOpts(ctypes.Structure):
    _fields_ = [("max_batch", ctypes.c_uint32), ("slots", ctypes.c_uint32),
                ("max_k", ctypes.c_uint32), ("max_L", ctypes.c_uint32),
                ("table", ctypes.c_uint32),
                ("hbm_budget_bytes", ctypes.c_uint64),
                ("flags", ctypes.c_uint32)]


_lib = None


def lib():
    """Load the HIP library; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(
                f"{LIB_PATH} is missing: build it with "
                "`python -c 'import __graft_entry__ as g; g.build()'`")
        L = ctypes.CDLL(LIB_PATH)
        P, u32, u64 = ctypes.c_void_p, ctypes.c_uint32, ctypes.c_uint64
        L.bang_index_create.argtypes = [ctypes.POINTER(IndexDesc),
                                        ctypes.POINTER(P)]
        L.bang_index_destroy.argtypes = [P]
        L.bang_build_pq_tables.argtypes = [P, P, u64, P, P]
        L.bang_build_pq_tables_bf16.argtypes = [P, P, u64, P, P]
        L.bang_search.argtypes = [P, P, u64, u32, u32, P, P,
                                  ctypes.POINTER(SearchOpts), P]
        L.bang_search_noalloc.argtypes = L.bang_search.argtypes
        L.bang_rerank.argtypes = [P, P, u64, P, u32, u32, P, P, P]
        L.bang_index_probe.argtypes = [P, u64, u64, P, ctypes.POINTER(u32), P]
        L.bang_server_create.argtypes = [P, ctypes.POINTER(ServerOpts),
                                         ctypes.POINTER(P)]
        L.bang_server_destroy.argtypes = [P]
        L.bang_server_submit.argtypes = [P, P, u32, u32, u32,
                                         ctypes.POINTER(u64)]
        L.bang_server_wait.argtypes = [P, u64, P, P, ctypes.c_int]
        L.bang_server_replay.argtypes = [P, P, u32, P, P, P, P, u32, P, P, P]
        L.bang_server_stats.argtypes = [P, P, u32]
        L.bang_abort_create.argtypes = [ctypes.POINTER(P)]
        for f in ("bang_abort_destroy", "bang_abort_set", "bang_abort_clear",
                  "bang_abort_status"):
            getattr(L, f).argtypes = [P]
        for f in EXPORTS[:-1]:
            getattr(L, f).restype = ctypes.c_int
        L.bang_last_error.argtypes = []
        L.bang_last_error.restype = ctypes.c_char_p
        _lib = L
    return _lib


def _check(rc: int):
    if rc != 0:
        raise BangError(rc, lib().bang_last_error().decode())


def _stream(stream):
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def _check_out(ids, dists, nq, k, device):
    """Caller-supplied outputs must be exactly [nq][k] on the queries' device
    (the kernels write every element of both)."""
    import torch
    for t, dt, nm in ((ids, torch.int32, "ids"), (dists, torch.float32,
                                                   "dists")):
        if tuple(t.shape) != (nq, k):
            raise ValueError(f"{nm} must have shape ({nq}, {k}), got "
                             f"{tuple(t.shape)}")
        if t.device != device:
            raise ValueError(f"{nm} must be on {device}")
        _dev_ptr(t, dt, nm)


def _dev_ptr(t, dtype=None, name="tensor"):
    import torch
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a CUDA tensor")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if dtype is not None and t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}, got {t.dtype}")
    return ctypes.c_void_p(t.data_ptr())


class Index:
    """Index.  Host numpy arrays in, copies in HBM.

    base [n][d] (float32 / uint8 / int8), adj [n][R] uint32 (BANG_NONE for
    empty slots), medoid, codebooks [m][256][d/m] float32, codes [n][m]
    uint8.  host_adj=True keeps the adjacency in pinned host memory, read
    by the search across the host link (BANG_INDEX_HOST_ADJ); bf16_base=True
    (float data) also keeps the base in bfloat16 for the BF16 re-rank
    (BANG_INDEX_BF16_BASE)."""

    def __init__(self, base, adj, medoid, codebooks, codes,
                 host_adj: bool = False, bf16_base: bool = False):
        self._h = None
        self._sink = None  # device word the probe kernel may write
        base = np.ascontiguousarray(base)
        adj = np.ascontiguousarray(adj, dtype=np.uint32)
        cb = np.ascontiguousarray(codebooks, dtype=np.float32)
        codes = np.ascontiguousarray(codes, dtype=np.uint8)
        dt = {np.dtype(np.float32): "f32", np.dtype(np.uint8): "u8",
              np.dtype(np.int8): "i8"}.get(base.dtype)
        if dt is None:
            raise TypeError(f"unsupported base dtype {base.dtype}")
        n, d = base.shape
        self.n, self.d, self.dtype = n, d, dt
        self.R = adj.shape[1]
        self.m = codes.shape[1]
        self.torch_dtype = {"f32": "float32", "u8": "uint8", "i8": "int8"}[dt]
        self.host_adj = bool(host_adj)
        desc = IndexDesc(n, d, DTYPES[dt], base.ctypes.data, adj.shape[1],
                         adj.ctypes.data, int(medoid), codes.shape[1],
                         cb.ctypes.data, codes.ctypes.data,
                         (INDEX_HOST_ADJ if host_adj else 0) |
                         (INDEX_BF16_BASE if bf16_base else 0))
        if adj.shape[0] != n or codes.shape[0] != n:
            raise ValueError("adj and codes need one row per base vector")
        if cb.shape != (self.m, 256, d // max(1, self.m)):
            raise ValueError("codebooks must be [m][256][d/m]")
        h = ctypes.c_void_p()
        _check(lib().bang_index_create(ctypes.byref(desc), ctypes.byref(h)))
        self._h = h

    def close(self):
        if self._h is not None and _lib is not None:
            lib().bang_index_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _queries(self, q):
        import torch
        want = getattr(torch, self.torch_dtype)
        if q.dim() != 2 or q.shape[1] != self.d:
            raise ValueError(f"queries must be [nq][{self.d}]")
        return _dev_ptr(q, want, "queries")

    def build_pq_tables(self, q, out=None, stream=None, bf16: bool = False):
        """Stage 1: tables [nq][m][256] float32 on the queries' device;
        bf16=True builds them by BF16 MFMA with FP32 accumulation
        (bang_build_pq_tables_bf16)."""
        import torch
        qp = self._queries(q)
        if out is None:
            out = torch.empty((q.shape[0], self.m, 256), dtype=torch.float32,
                              device=q.device)
        elif tuple(out.shape) != (q.shape[0], self.m, 256):
            raise ValueError(f"out must have shape ({q.shape[0]}, {self.m}, 256)")
        fn = (lib().bang_build_pq_tables_bf16 if bf16
              else lib().bang_build_pq_tables)
        _check(fn(self._h, qp, q.shape[0], _dev_ptr(out, torch.float32, "out"),
                  _stream(stream)))
        return out

    def search(self, q, k: int, L: int, c_max: int = 0, iter_cap: int = 0,
               want_cand: int = 0, want_counters: bool = False,
               want_times: bool = False, table: str = "f32",
               rerank_global: bool = False, query_L=None, query_k=None,
               filter: str = "exact", want_phases: bool = False, out=None,
               abort=None, rerank: str = "exact", stream=None,
               seen_log_short: bool = False, tables=None, order=None,
               waves_per_cu: int = 0, seen_cache: bool = True,
               _entry: str = "bang_search"):
        """Stages 1-3.  Returns (ids uint32-as-int32 [nq][k], dists
        float32 [nq][k]) and, on request, the expanded nodes [nq][want_cand]
        `table` is the PQ table storage the search ranks by: "f32", the
        precision form's "f16" / "u8", or "exact" (no table: exact
        distances, no re-rank).  query_L / query_k (int32 CUDA tensors
        [nq]) make a mixed batch: query i with its own L_i <= L and
        k_i <= min(k, L_i), row i holding k_i results then padding.
        and counters [nq][4] (iterations, status) and device wall-clock
        ticks [nq][2] (begin, end).  `filter` is the visited filter:
        "exact" (set union, the default), "bloom" (the paper's Bloom
        filter, BANG_FILTER_BLOOM) or "seen" (an exact seen bitmap,
        BANG_FILTER_SEEN: the same results as "exact").  want_phases adds per-query cycles of
        the search's seven phases [nq][7] (bang_search_opts.out_phases;
        a timed copy of the search).  abort: a StopRequest the search
        obeys (bang_search_opts.abort).  rerank: "exact" or "bf16" (float
        data on an index with bf16_base; the same answer, counters[:, 2]
        the candidates recomputed in FP32).  tables: float32 CUDA tensor
        [nq][m][256] of PQ tables built beforehand (build_pq_tables,
        optionally bf16=True) that the search ranks by instead of building
        its own.  order (int32 CUDA tensor [nq], a permutation): the order
        in which the persistent waves take the queries; waves_per_cu: a
        cap on resident waves per CU (0: as many as fit); neither changes
        results.  seen_log_short: with the
        "seen" filter, stop setting bits after 64 logged ids and only test
        from then on (BANG_SEARCH_SEEN_LOG_SHORT; for testing).
        seen_cache=False: the exact-distance search without its seen-id
        cache (BANG_SEARCH_NO_SEEN_CACHE; same results)."""
        import torch
        qp = self._queries(q)
        nq = q.shape[0]
        if out is None:
            ids = torch.empty((nq, k), dtype=torch.int32, device=q.device)
            dists = torch.empty((nq, k), dtype=torch.float32, device=q.device)
        else:
            ids, dists = out
            _check_out(ids, dists, nq, k, q.device)
        opts = SearchOpts(c_max, iter_cap, None, 0, None, None, TABLES[table],
                          (1 if rerank_global else 0)
                          | (2 if seen_log_short else 0)
                          | (0 if seen_cache else 4))
        opts.filter = FILTERS[filter]
        if abort is not None:
            opts.abort = abort._h.value
        opts.rerank = RERANKS[rerank]
        if order is not None:
            if tuple(order.shape) != (nq,):
                raise ValueError(f"order must have shape ({nq},)")
            opts.order = _dev_ptr(order, torch.int32, "order").value
        opts.waves_per_cu = int(waves_per_cu)
        if tables is not None:
            if tuple(tables.shape) != (nq, self.m, 256):
                raise ValueError(f"tables must have shape ({nq}, {self.m}, 256)")
            opts.tables = _dev_ptr(tables, torch.float32, "tables").value
        for t, nm in ((query_L, "query_L"), (query_k, "query_k")):
            if t is not None:
                if tuple(t.shape) != (nq,):
                    raise ValueError(f"{nm} must have shape ({nq},)")
                setattr(opts, nm, _dev_ptr(t, torch.int32, nm).value)
        cand = cnt = times = None
        if want_cand:
            cand = torch.empty((nq, want_cand), dtype=torch.int32,
                               device=q.device)
            opts.out_cand = cand.data_ptr()
            opts.cand_stride = want_cand
        if want_counters:
            cnt = torch.empty((nq, 4), dtype=torch.int32, device=q.device)
            opts.out_counters = cnt.data_ptr()
        if want_times:
            times = torch.empty((nq, 2), dtype=torch.int64, device=q.device)
            opts.out_times = times.data_ptr()
        phases = None
        if want_phases:
            phases = torch.empty((nq, 7), dtype=torch.int32, device=q.device)
            opts.out_phases = phases.data_ptr()
        _check(getattr(lib(), _entry)(
            self._h, qp, nq, k, L, _dev_ptr(ids, torch.int32, "ids"),
            _dev_ptr(dists, torch.float32, "dists"), ctypes.byref(opts),
            _stream(stream)))
        res = (ids, dists)
        if want_cand:
            res += (cand,)
        if want_counters:
            res += (cnt,)
        if want_times:
            res += (times,)
        if want_phases:
            res += (phases,)
        return res

    def search_noalloc(self, q, k: int, L: int, out, table: str = "f32",
                       query_L=None, query_k=None, rerank: str = "exact",
                       abort=None, stream=None):
        """bang_search_noalloc: the search with no device allocation into
        the caller's `out` = (ids int32 [nq][k], dists float32 [nq][k])
        CUDA tensors; the other arguments as in search.  Returns out."""
        return self.search(q, k, L, out=out, table=table, query_L=query_L,
                           query_k=query_k, rerank=rerank, abort=abort,
                           stream=stream, _entry="bang_search_noalloc")

    def probe(self, nreads: int, seed: int = 0, stream=None) -> int:
        """Launch the random-row read probe (bang_index_probe) on `stream`
        (default: torch's current stream): nreads adjacency rows read the
        way the search reads them.  Returns the bytes read per row; the
        caller times the launch."""
        import torch
        if self._sink is None:
            self._sink = torch.zeros(1, dtype=torch.int64, device="cuda")
        rb = ctypes.c_uint32(0)
        _check(lib().bang_index_probe(self._h, nreads, seed,
                                      self._sink.data_ptr(),
                                      ctypes.byref(rb), _stream(stream)))
        return int(rb.value)

    def rerank(self, q, cand, k: int, out=None, stream=None):
        """Stage 3 alone over cand [nq][c_max] (int32 view of uint32 ids;
        -1 = BANG_NONE padding)."""
        import torch
        qp = self._queries(q)
        nq = q.shape[0]
        if cand.shape[0] != nq:
            raise ValueError("one candidate row per query")
        if out is None:
            ids = torch.empty((nq, k), dtype=torch.int32, device=q.device)
            dists = torch.empty((nq, k), dtype=torch.float32, device=q.device)
        else:
            ids, dists = out
            _check_out(ids, dists, nq, k, q.device)
        _dev_ptr(cand, torch.int32, "cand")
        if cand.device != q.device:
            raise ValueError("cand must be on the queries' device")
        _check(lib().bang_rerank(
            self._h, qp, nq, _dev_ptr(cand, torch.int32, "cand"),
            cand.shape[1], k, _dev_ptr(ids, torch.int32, "ids"),
            _dev_ptr(dists, torch.float32, "dists"), _stream(stream)))
        return ids, dists


class StopRequest:
    """A stop request (bang_abort_*): set() asks every search that carries
    it to stop soon (each wave leaves after its current expansion; rows of
    stopped or unstarted queries are padding with status 2); stopped()
    tells, after the search's stream has been synchronised, whether a
    search stopped a query because of it; clear() re-arms it."""

    def __init__(self):
        self._h = None
        h = ctypes.c_void_p()
        _check(lib().bang_abort_create(ctypes.byref(h)))
        self._h = h

    def set(self):
        _check(lib().bang_abort_set(self._h))

    def clear(self):
        _check(lib().bang_abort_clear(self._h))

    def stopped(self) -> bool:
        rc = lib().bang_abort_status(self._h)
        if rc == -5:
            return True
        _check(rc)
        return False

    def close(self):
        if self._h is not None and _lib is not None:
            lib().bang_abort_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Server:
    """Continuous-batching request loop over an Index (bang_server_*).

    submit(q, k, L) queues a request of host queries (numpy [nq][d]) and
    returns a ticket; wait(ticket) returns (ids uint32 [nq][k], dists
    float32 [nq][k]).  replay() drives an open-loop arrival schedule from
    native code and returns results and per-request latencies.  graphs:
    each slot replays its batches from captured HIP graphs
    (BANG_SERVER_GRAPHS)."""

    def __init__(self, index: Index, max_batch: int = 4096, slots: int = 2,
                 max_k: int = 100, max_L: int = 256, table: str = "f32",
                 hbm_budget_bytes: int = 0, graphs: bool = False):
        self._h = None
        self.index = index  # the index must outlive the server
        o = ServerOpts(max_batch, slots, max_k, max_L, TABLES[table],
                       hbm_budget_bytes, 1 if graphs else 0)
        h = ctypes.c_void_p()
        _check(lib().bang_server_create(index._h, ctypes.byref(o),
                                        ctypes.byref(h)))
        self._h = h
        self.dtype = np.dtype(index.torch_dtype)
        self._shapes = {}  # ticket -> (nq, k); dict updates are atomic

    def _q(self, q):
        q = np.ascontiguousarray(q, dtype=self.dtype)
        if q.ndim != 2 or q.shape[1] != self.index.d:
            raise ValueError(f"queries must be [nq][{self.index.d}]")
        return q

    def submit(self, q, k: int, L: int) -> int:
        q = self._q(q)
        t = ctypes.c_uint64()
        _check(lib().bang_server_submit(self._h, q.ctypes.data, q.shape[0], k,
                                        L, ctypes.byref(t)))
        self._shapes[t.value] = (q.shape[0], k)
        return t.value

    def wait(self, ticket: int, timeout_ms: int = -1):
        if ticket not in self._shapes:
            raise BangError(-1, f"unknown ticket {ticket}")
        nq, k = self._shapes[ticket]
        ids = np.empty((nq, k), dtype=np.uint32)
        d = np.empty((nq, k), dtype=np.float32)
        _check(lib().bang_server_wait(self._h, ticket, ids.ctypes.data,
                                      d.ctypes.data, timeout_ms))
        self._shapes.pop(ticket, None)
        return ids, d

    def replay(self, queries, nq, k, L, arrival_s, kstride: int | None = None):
        """Open loop: request j arrives at arrival_s[j] (seconds from the
        call) with nq[j] consecutive query rows, k[j], L[j].  Returns
        (ids [sum nq][kstride], dists, latency_s [nreq])."""
        q = self._q(queries)
        nq = np.ascontiguousarray(nq, dtype=np.uint32)
        k = np.ascontiguousarray(k, dtype=np.uint32)
        L = np.ascontiguousarray(L, dtype=np.uint32)
        arr = np.ascontiguousarray(arrival_s, dtype=np.float64)
        if int(nq.sum()) > q.shape[0]:
            raise ValueError("fewer query rows than the requests hold")
        ks = int(kstride or k.max())
        tot = int(nq.sum())
        ids = np.empty((tot, ks), dtype=np.uint32)
        d = np.empty((tot, ks), dtype=np.float32)
        lat = np.empty(len(nq), dtype=np.float64)
        _check(lib().bang_server_replay(
            self._h, q.ctypes.data, len(nq), nq.ctypes.data, k.ctypes.data,
            L.ctypes.data, arr.ctypes.data, ks, ids.ctypes.data,
            d.ctypes.data, lat.ctypes.data))
        return ids, d, lat

    def stats(self) -> dict:
        out = np.zeros(5, dtype=np.uint64)
        _check(lib().bang_server_stats(self._h, out.ctypes.data, 5))
        return dict(zip(("requests", "launches", "queries", "max_in_flight",
                         "slots"), (int(x) for x in out)))

    def close(self):
        if self._h is not None and _lib is not None:
            lib().bang_server_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
