"""Benchmark: QPS of the whole hot path (PQ table + greedy search + re-rank)
on one MI355X for the 1M uint8 workload, plain FP32 tables vs the precision
form (FP16 / u8 tables), each at the smallest worklist size L whose mean
10-recall@10 reaches 0.9 (or, if none does, the L with the best recall),
with p50/p99 per-query completion latency, the search kernel's fraction of
the HBM roofline, and the CPU oracle timed on the host.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--L L]

Prints one JSON line; `value` is the plain FP32 form's QPS and
`precision_form` holds the reduced-precision measurements (FP16 / u8 table
storage, and each form ranking by tables built with BF16 MFMA).  A step is
one bang_search call over the 10,000 resident queries (with BF16-MFMA
tables: their build, then the search); each form's timed region
holds exactly K steps, bracketed by a device synchronisation on both sides,
each step bracketed by HIP events on the stream the kernel runs on.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = ("QPS at recall@10>=0.9 on 1 GPU, plain FP32 vs reduced-precision "
          "form; p50/p99 ms")
WORKLOAD = "sift1m"
HBM_PEAK_GBS = 8000.0
BF16_PEAK_TFLOPS = 2500.0  # MI355X dense BF16 MFMA
# MI355X's host link: PCIe 5.0 x16, 64 GB/s per direction
HOST_LINK_PEAK_GBS = 64.0
TARGET_RECALL = 0.9
TABLES = ("f32", "f16", "u8")
# the unseen-neighbour count of the method's bytes runs on every 5th query
NPRIME_EVERY = 5
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "search_sift1m_traffic.json")
KERNEL_SOURCES = [os.path.join(ROOT, "paper_2401_11324_amd", "csrc", f)
                  for f in ("search_kernel.h", "search_variants.hip",
                            "bang_kernels.hip", "bang_api.cpp", "internal.h")]


def kernel_hash() -> str:
    h = hashlib.sha256()
    for p in KERNEL_SOURCES:
        with open(p, "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def recall_at_k(ids: np.ndarray, gt: np.ndarray, k: int) -> float:
    """Mean k-recall@k = |S ∩ S~| / k (section "Algorithm Parameters")."""
    hits = [len(set(a[:k].tolist()) & set(b[:k].tolist())) for a, b in
            zip(ids, gt)]
    return float(np.mean(hits)) / k


def iteration_overhead(I: float, t: int) -> float:
    """lambda = (I - t) / t * 100: iterations above the lower bound t (the
    worklist size), section "Effect of Varying Worklist Size (t)"."""
    return (I - t) / t * 100.0


def packed_row_bytes(adj_deg, R, m, d, elem, k, iters, cand, c_max,
                     exact=False):
    """Bytes this design's search reads, from the per-query counters: per
    expansion the packed row, i.e. the adjacency ids (4R) and the m code
    bytes of EVERY neighbour (the row carries them, seen or not); per query
    the query vector, the base rows of the re-ranked candidates and the k
    (id, distance) results.  Exact-distance search: the base row (d
    elements) of every neighbour instead of its codes, and no re-rank."""
    I = iters.astype(np.int64)
    valid = cand != 0xFFFFFFFF
    deg_sum = np.where(valid, adj_deg[np.where(valid, cand, 0)], 0).sum()
    if exact:
        return int(I.sum() * 4 * R + deg_sum * d * elem + len(I) * d * elem
                   + len(I) * 8 * k)
    rr = np.minimum(I, c_max).sum()
    return int(I.sum() * 4 * R + deg_sum * m + len(I) * d * elem
               + rr * d * elem + len(I) * 8 * k)


def unseen_neighbours(adj, medoid, iters, cand):
    """Per query, the sum over its expansions of |N'|, the neighbours not
    seen before (Algorithm 2 with an exact visited set: the seen set starts
    as {s} and takes each row's unseen neighbours).  Every id enters the
    seen set once, so the sum is the number of distinct ids in the rows of
    the expanded nodes, the start node and empty slots excluded.  cand
    holds the expanded nodes in expansion order."""
    # distinct count without a sort: after pos[ids] = 0..len-1, exactly one
    # position per distinct id holds its own index (whichever repeat won)
    pos = np.zeros(adj.shape[0], dtype=np.int64)
    out = np.zeros(len(iters), dtype=np.int64)
    for qi in range(len(iters)):
        ids = adj[cand[qi, :int(iters[qi])]].ravel()
        ids = ids[(ids != 0xFFFFFFFF) & (ids != medoid)]
        at = np.arange(ids.size)
        pos[ids] = at
        out[qi] = np.count_nonzero(pos[ids] == at)
    return out


def method_bytes(nprime, R, m, d, elem, k, iters, c_max, exact=False):
    """HBM bytes the method itself must move per launch: per expansion the
    adjacency row (4R), the visited-set probes (8 bytes per neighbour slot)
    and the codes of the unseen neighbours only (m bytes each); per query
    the base rows re-ranked (the expanded nodes, at most c_max), the query
    and the k results.  Exact-distance search: the base row of each unseen
    neighbour instead of its codes, and no re-rank.  nprime[q] is the
    query's sum of |N'| over its expansions (unseen_neighbours, or an
    estimate from a sample of the batch).  Returns
    (total, parts) with the terms listed separately."""
    I = iters.astype(np.int64)
    npr = np.asarray(nprime, dtype=np.float64).sum()
    parts = {"adjacency": int(I.sum() * 4 * R),
             "visited_probes": int(I.sum() * 8 * R),
             "codes_unseen" if not exact else "base_rows_unseen":
                 int(npr * (d * elem if exact else m)),
             "rerank_rows": 0 if exact else
                 int(np.minimum(I, c_max).sum() * d * elem),
             "queries_and_results": int(len(I) * (d * elem + 8 * k))}
    return sum(parts.values()), parts


def cpu_model() -> str:
    """The host CPU's model name (/proc/cpuinfo), or "unknown"."""
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(idx_np, queries, k, L, budget_s=15.0, budget1_s=8.0):
    """The CPU oracle (test infrastructure) on a bounded sample of the same
    queries, on every host thread this process may use: 64 queries to
    estimate the rate, then enough for ~budget_s; then on one thread for
    ~budget1_s."""
    import oracle
    threads = oracle.default_threads()
    ix = oracle.Index(idx_np["base"], idx_np["adj"], idx_np["medoid"],
                      idx_np["codebooks"], idx_np["codes"])

    def timed(nthreads, budget):
        t = time.perf_counter()
        probe = 64 if nthreads > 1 else 8
        oracle.search(ix, queries[:probe], k, L, nthreads=nthreads)
        rate = probe / max(1e-9, time.perf_counter() - t)
        n = int(min(len(queries), max(probe, rate * budget)))
        t = time.perf_counter()
        oracle.search(ix, queries[:n], k, L, nthreads=nthreads)
        return n, time.perf_counter() - t

    n, dt = timed(threads, budget_s)
    n1, dt1 = timed(1, budget1_s)
    return {"value": round(n / dt, 1), "unit": "queries/s", "cores": threads,
            "kind": "oracle", "cpu_model": cpu_model(),
            "sample": f"first {n} of {len(queries)} queries, k={k}, L={L}, "
                      f"{dt:.1f} s; table + Algorithm 1 + re-rank, "
                      f"{threads} threads",
            "one_thread": {"value": round(n1 / dt1, 1), "unit": "queries/s",
                           "sample": f"first {n1} queries, {dt1:.1f} s"}}


# offered queries/s: 10^4 to 10^6 in half decades
SERVE_RATES = (1e4, 10 ** 4.5, 1e5, 10 ** 5.5, 1e6)
SERVE_P99_TARGET_MS = 50.0
SERVE_CANDIDATES = ((1024, 2, False), (4096, 2, False), (4096, 4, False),
                    (16384, 2, False), (4096, 2, True), (16384, 2, True))


def serving_section(gi, d, w, gt):
    """The serving loop on the resident index: the autotuner picks batch
    size and slot count on a calibration stream, then open-loop Poisson
    streams at each offered rate (requests of 1-256 queries, k in {10,
    100}, L in {32, 64, 128}) report sustained rate, p50/p99 request
    latency and recall@10 of every served query."""
    import synth
    from paper_2401_11324_amd import serving
    qnp = d["queries"]
    max_k, max_L = 100, 128
    # calibrate near the highest offered rate, where the candidates differ
    calib = synth.serving_requests(w, SERVE_RATES[-1], 0.2, salt=1)
    (mb, sl, gr), trials = serving.autotune(gi, qnp, calib, SERVE_CANDIDATES,
                                            max_k, max_L, SERVE_P99_TARGET_MS)
    rates = []
    for i, rate in enumerate(SERVE_RATES):
        req = synth.serving_requests(w, rate, min(1.0, 2e5 / rate),
                                     salt=10 + i)
        s, ids, _ = serving.run_load(gi, qnp, req, mb, sl, max_k, max_L,
                                     graphs=gr)
        s["recall10"] = round(recall_at_k(ids[:, :10], gt[req["rows"]], 10), 4)
        rates.append(s)
    # the same streams at the lowest and highest rate, with and without the
    # slots replaying captured HIP graphs
    graphs = []
    for i, rate in ((0, SERVE_RATES[0]), (len(SERVE_RATES) - 1,
                                          SERVE_RATES[-1])):
        req = synth.serving_requests(w, rate, min(1.0, 2e5 / rate),
                                     salt=10 + i)
        for g in (False, True):
            s, _, _ = serving.run_load(gi, qnp, req, mb, sl, max_k, max_L,
                                       graphs=g)
            graphs.append(s)
    return {"table": "f32",
            "requests": "sizes log-uniform 1-256 queries, k in {10,100}, "
                        "L in {32,64,128} raised to k, Poisson arrivals",
            "autotune": {"chosen": {"max_batch": mb, "slots": sl,
                                    "graphs": gr},
                         "p99_target_ms": SERVE_P99_TARGET_MS,
                         "trials": trials},
            "rates": rates,
            "graphs_vs_direct": graphs}


DEEP_WORKLOAD = "deep1m"


def deep_section(a, bang, torch):
    """Plain FP32 vs the precision form (FP16 / u8 tables) and the exact-
    distance search on the unit-normalised float index shaped like the
    paper's Deep data (d=96, m=48: a 48 KB FP32 table), each at its
    smallest swept L with recall@10 >= 0.9; recall lost against FP32 at
    the same L and the distance error against FP64 ground truth."""
    import synth
    from synth import store
    w = synth.WORKLOADS[DEEP_WORKLOAD]
    if not store.exists(w):
        return {"skipped": f"index files for {w.name} are missing; write "
                           f"them with `python -m oracle.build_index "
                           f"{w.name}`"}
    run = Runner(w, a, bang, torch, bf16_base=True)
    forms = TABLES + ("exact",)
    rows = run.sweep(forms)
    by = {(r["table"], r["L"]): r["recall10"] for r in rows}
    out = {"workload": "unit-normalised Gaussian mixture: n=1,000,000 d=96 "
                       "float32, 4,096 unit centres, noise norm 0.3; 10,000 "
                       "queries; graph R=64 L_build=100 alpha=1.2; PQ m=48",
           "sweep": rows, "forms": {}}
    for t in forms:
        rec = run.measure(t, run.pick_L(t))
        if t in ("f16", "u8"):
            rec["recall_lost_vs_f32_same_L"] = round(
                by[("f32", rec["L"])] - by[(t, rec["L"])], 4)
        out["forms"][t] = rec
    # the BF16 re-rank with the FP32 recheck, at each PQ form's point
    for t in TABLES:
        rec = run.measure(t, out["forms"][t]["L"], rerank="bf16")
        rec["recall_equal_to_exact_rerank"] = rec["recall10"] == \
            out["forms"][t]["recall10"]
        out["forms"][t + "+bf16_rerank"] = rec
    # the tables by BF16 MFMA with FP32 accumulation (a step builds them,
    # then searches by them), each PQ form at its point; and the whole
    # precision form: BF16-MFMA tables stored as FP16 / u8, then the BF16
    # re-rank with the FP32 recheck
    for t in TABLES:
        rec = run.measure(t, out["forms"][t]["L"], bf16_tables=True)
        rec["recall_lost_vs_fp32_tables_same_L"] = round(
            out["forms"][t]["recall10"] - rec["recall10"], 4)
        out["forms"][t + "+bf16_mfma_tables"] = rec
    for t in ("f16", "u8"):
        rec = run.measure(t, out["forms"][t]["L"], bf16_tables=True,
                          rerank="bf16")
        rec["recall_lost_vs_f32_same_L"] = round(
            by[("f32", rec["L"])] - rec["recall10"], 4)
        out["forms"][t + "+bf16_mfma_tables+bf16_rerank"] = rec
    out["table_build"] = table_build_section(run)
    base = out["forms"]["f32"]["qps"]
    for t in out["forms"]:
        out["forms"][t]["speedup_vs_f32"] = round(
            out["forms"][t]["qps"] / base, 3)
    run.gi.close()
    return out


def table_build_section(run, reps=20):
    """Stage 1 alone for the whole query batch: the FP32 table kernel
    against the BF16-MFMA one (bang_build_pq_tables_bf16), each as time,
    table bytes written per second and, for the MFMA build, its inner-
    product FLOP rate against the BF16 dense peak (2 nq m 256 ds FLOP,
    d/m padded to the MFMA's K of 4)."""
    torch, gi, q = run.torch, run.gi, run.q
    stream = torch.cuda.current_stream()
    nq, m = q.shape[0], run.w.m
    ds = run.w.d // m
    out = {"queries": nq, "table_bytes": nq * m * 256 * 4}
    for name, bf in (("fp32", False), ("bf16_mfma", True)):
        T = gi.build_pq_tables(q, bf16=bf)
        torch.cuda.synchronize()
        ts = []
        for _ in range(reps):
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            gi.build_pq_tables(q, out=T, bf16=bf)
            e1.record(stream)
            torch.cuda.synchronize()
            ts.append(e0.elapsed_time(e1))
        ms = float(np.mean(ts))
        rec = {"ms": round(ms, 4),
               "written_gbs": round(out["table_bytes"] / (ms / 1e3) / 1e9, 1)}
        if bf:
            kpad = -(-ds // 4) * 4
            fl = 2.0 * nq * m * 256 * kpad
            rec["mfma_tflops"] = round(fl / (ms / 1e3) / 1e12, 4)
            rec["mfma_frac_of_bf16_peak"] = round(
                fl / (ms / 1e3) / 1e12 / BF16_PEAK_TFLOPS, 6)
            rec["k_used_of_padded"] = f"{ds}/{kpad}"
        out[name] = rec
    return out


BATCH_SIZES = (1, 10, 100, 500, 1000, 2000, 4000, 10000, 20000)
SCALE_MIXED_NQ = 100_000
M_SWEEP = (16, 32, 64)


def batch_section(run, L):
    """QPS of the plain FP32 search at the bench point against the size of
    the query batch (the paper's batch-size study): one launch per batch,
    the mean of several; past 10,000 the queries repeat."""
    torch, gi, q, k = run.torch, run.gi, run.q, run.w.k
    stream = torch.cuda.current_stream()
    rows = []
    for nq in BATCH_SIZES:
        reps = -(-nq // q.shape[0])
        qb = q.repeat(reps, 1)[:nq].contiguous() if reps > 1 else q[:nq]
        ids = torch.empty((nq, k), dtype=torch.int32, device=q.device)
        dist = torch.empty((nq, k), dtype=torch.float32, device=q.device)
        gi.search(qb, k, L, out=(ids, dist))
        torch.cuda.synchronize()
        n = 5
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(n):
            gi.search(qb, k, L, out=(ids, dist))
        e1.record(stream)
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / n
        rows.append({"batch": nq, "ms_per_launch": round(ms, 4),
                     "qps": round(nq / (ms / 1e3), 1)})
    top = max(r["qps"] for r in rows)
    sat = next(r["batch"] for r in rows if r["qps"] >= 0.9 * top)
    return {"table": "f32", "L": L, "rows": rows,
            "saturation_batch_90pct": sat,
            "waves_resident": "CUs x waves per CU set by the table's LDS"}


def gather_probe(gi, torch, nreads, reps=3):
    """Random-row read rate of the index's adjacency (bang_index_probe):
    rows read the way the search reads an expanded node's row, as many in
    flight as 32 waves per CU allow.  Returns {row_bytes, reads, gbs}."""
    stream = torch.cuda.current_stream()
    gi.probe(nreads, seed=1)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for i in range(reps):
        rb = gi.probe(nreads, seed=2 + i)
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    return {"row_bytes": rb, "reads": nreads,
            "gbs": round(nreads * rb / (ms / 1e3) / 1e9, 2)}


PHASES = ("table_and_start", "row_wait", "scoring", "rank", "next_node",
          "merge", "rerank")


def phase_section(run, points):
    """Where a query's time goes (the fused kernel's counterpart of the
    paper's per-kernel time table): one launch of the timed copy of the
    search (bang_search_opts.out_phases) per (table form, L) point.  Cycles
    are per query for the table and the re-rank, per expansion for the
    loop's phases, and each phase's share of all cycles."""
    torch, q, k = run.torch, run.q, run.w.k
    stream = torch.cuda.current_stream()
    out = []
    for table, L in points:
        ids, dist, cnt, ph = run.gi.search(q, k, L, table=table,
                                           want_counters=True,
                                           want_phases=True)
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        run.gi.search(q, k, L, table=table, want_phases=True)
        e1.record(stream)
        torch.cuda.synchronize()
        c = ph.cpu().numpy().view(np.uint32).astype(np.float64)
        it = float(cnt.cpu().numpy()[:, 0].astype(np.float64).sum())
        tot = c.sum(0)
        rec = {"table": table, "L": L,
               "timed_kernel_ms": round(e0.elapsed_time(e1), 3),
               "share": {n: round(float(v / tot.sum()), 4)
                         for n, v in zip(PHASES, tot)},
               "cycles_per_query": {n: round(float(tot[i] / len(c)), 1)
                                    for i, n in enumerate(PHASES)
                                    if n in ("table_and_start", "rerank")},
               "cycles_per_expansion": {n: round(float(tot[i] / it), 1)
                                        for i, n in enumerate(PHASES)
                                        if n not in ("table_and_start",
                                                     "rerank")}}
        out.append(rec)
    return out


def bloom_section(run, points):
    """The paper's Bloom filter as the visited test (BANG_FILTER_BLOOM)
    against the exact set union, at the given (table form, L) points:
    QPS, recall@10 and iterations with each filter."""
    out = {"z": 399887, "hashes": "FNV-1a-32 x2", "points": []}
    for table, L, exact in points:
        rec = run.measure(table, L, filter="bloom")
        rec["vs_exact_filter"] = {
            "qps_ratio": round(rec["qps"] / exact["qps"], 4),
            "recall10_delta": round(rec["recall10"] - exact["recall10"], 4),
            "iterations_delta": round(rec["mean_iterations"]
                                      - exact["mean_iterations"], 2)}
        out["points"].append(rec)
    return out


def m_section(run, bang):
    """Recall and QPS against the number m of PQ subspaces (the paper's
    compression-ratio study): the same base, graph and queries encoded with
    m = 16, 32, 64 (m/d = 0.125, 0.25, 0.5 code bytes per base byte), FP32
    tables, every swept L; per m also the smallest L with recall@10 >= 0.9.
    The extra encodings sit beside the index (written by
    `python -m oracle.build_index <workload> --extra-m 16 64`)."""
    from synth import store
    torch, w, d, q, k = run.torch, run.w, run.d, run.q, run.w.k
    stream = torch.cuda.current_stream()
    have = store.extra_names(w)
    out = {"table": "f32", "per_m": []}
    for m in M_SWEEP:
        if m == w.m:
            cb, codes = d["codebooks"], d["codes"]
        elif f"codes_m{m}" in have:
            ex = store.load_extra(w, [f"codebooks_m{m}", f"codes_m{m}"])
            cb, codes = ex[f"codebooks_m{m}"], ex[f"codes_m{m}"]
        else:
            out["per_m"].append({"m": m, "skipped": "encoding missing"})
            continue
        gi = bang.Index(d["base"], d["adj"], d["medoid"], cb, codes)
        rows = []
        for L in w.Ls:
            ids, dist = gi.search(q, k, L)
            torch.cuda.synchronize()
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            gi.search(q, k, L, out=(ids, dist))
            e1.record(stream)
            torch.cuda.synchronize()
            rec = recall_at_k(ids.cpu().numpy().view(np.uint32), run.gt, k)
            rows.append({"L": L, "recall10": round(rec, 4),
                         "qps": round(q.shape[0] / (e0.elapsed_time(e1)
                                                    / 1e3))})
        gi.close()
        ok = [r for r in rows if r["recall10"] >= TARGET_RECALL]
        out["per_m"].append({
            "m": m, "code_bytes_per_vector": m,
            "compression_ratio": round(m / (w.d * (1 if w.dtype in
                                                   ("u8", "i8") else 4)), 4),
            "fp32_table_kb": m, "sweep": rows,
            "at_target": ok[0] if ok else None,
            "best_recall10": max(r["recall10"] for r in rows)})
    return out


def scale_host(a) -> int:
    """Host-resident adjacency at scale: a synthetic graph of a.scale_host
    int8 points (synth.scale_graph_index: R=64 ids per row spread over the
    whole range, so no cache helps), adjacency in pinned host memory, codes
    and base vectors in HBM; 10,000 queries, k=10.  Reports QPS, mean
    iterations and the adjacency bytes that crossed the host link per
    second.  Recall is not defined on this graph."""
    import torch
    import synth
    import paper_2401_11324_amd as bang
    n = a.scale_host
    t0 = time.perf_counter()

    def log(msg):
        print(f"[scale-host {time.perf_counter() - t0:6.1f}s] {msg}",
              file=sys.stderr, flush=True)

    log(f"generating {n:,} nodes")
    d = synth.scale_graph_index(n, nq=SCALE_MIXED_NQ)
    log("index (validate, pin adjacency, upload)")
    gi = bang.Index(d["base"], d["adj"], d["medoid"], d["codebooks"],
                    d["codes"], host_adj=True)
    R = d["adj"].shape[1]
    del d["adj"]
    qall = torch.from_numpy(d["queries"]).cuda()
    q = qall[:10_000]
    nq, k = q.shape[0], 10
    stream = torch.cuda.current_stream()
    rows = []
    for L in (64, 128):
        ids, dist, cnt = gi.search(q, k, L, want_counters=True)
        torch.cuda.synchronize()
        iters = cnt.cpu().numpy()[:, 0].astype(np.int64)
        ev = [(torch.cuda.Event(enable_timing=True),
               torch.cuda.Event(enable_timing=True)) for _ in range(a.steps)]
        for e0, e1 in ev:
            e0.record(stream)
            gi.search(q, k, L, out=(ids, dist))
            e1.record(stream)
        torch.cuda.synchronize()
        ms = float(np.mean([e0.elapsed_time(e1) for e0, e1 in ev]))
        link = iters.sum() * 4 * R / (ms / 1e3) / 1e9
        rows.append({"L": L, "k": k, "qps": round(nq / (ms / 1e3), 1),
                     "kernel_ms_mean": round(ms, 3),
                     "mean_iterations": round(float(iters.mean()), 2),
                     "host_link_gbs": round(link, 2),
                     "host_link_frac": round(link / HOST_LINK_PEAK_GBS, 4)})
        log(f"L={L}: {rows[-1]}")
    # one persistent launch of the 100M configuration's mixed batch: 100,000
    # queries, k in {1, 10, 100}, L = max(k, round(exp(U[ln 16, ln 256])))
    kq, Lq = synth.mixed_batch(SCALE_MIXED_NQ, salt=3)
    from paper_2401_11324_amd import tuning
    tiles, tile_trials = tuning.launch_tiles(gi, qall, kq, Lq)
    log(f"tiles: {tiles}")
    mixed = mixed_launch(gi, qall, kq, Lq, tiles, a.steps, R)
    mixed["tiles"] = {"chosen": tiles, "trials": tile_trials}
    mixed["untuned"] = mixed_launch(gi, qall, kq, Lq, None, a.steps, R)
    for m_ in (mixed, mixed["untuned"]):
        m_["host_link_frac"] = round(m_["adjacency_gbs"] /
                                     HOST_LINK_PEAK_GBS, 4)
    log(f"mixed batch: {mixed}")
    del ids, dist, cnt
    # the serving loop on the same host-resident index (configuration 4's
    # request recipe; results are not checked here, recall is undefined)
    from paper_2401_11324_amd import serving
    w = synth.WORKLOADS["sift1m"].with_(name="scale", nq=nq)
    serve = []
    for i, rate in enumerate(SERVE_RATES):
        req = synth.serving_requests(w, rate, min(1.0, 2e5 / rate),
                                     salt=20 + i)
        sm, _, _ = serving.run_load(gi, d["queries"][:nq], req, 16384, 2,
                                    100, 128)
        serve.append(sm)
        log(f"serving {rate:.0e}: {sm}")
    gi.close()
    print(json.dumps({"scale_host": {
        "workload": f"synthetic graph: n={n:,} int8 d=128, R={R} ids per "
                    f"row spread over the range (no locality), PQ m=32; "
                    f"adjacency {n * R * 4 / 1e9:.1f} GB in pinned host "
                    f"memory; {nq:,} queries",
        "steps": a.steps, "rows": rows, "mixed_batch": mixed,
        "host_link_peak_gbs": HOST_LINK_PEAK_GBS,
        "serving": {"max_batch": 16384, "slots": 2,
                    "requests": "sizes log-uniform 1-256 queries, k in "
                                "{10,100}, L in {32,64,128} raised to k, "
                                "Poisson arrivals", "rates": serve}}}),
          flush=True)
    return 0


def mixed_launch(gi, q, kq, Lq, tiles, steps, R, gt=None):
    """One persistent launch of a mixed batch (per-query k and L) with
    the take order and waves per CU of `tiles` (None: the batch's order,
    full occupancy): QPS, iterations, adjacency bytes per second and,
    given ground truth for the rows, recall@10 of the queries with k >= 10."""
    import torch
    from paper_2401_11324_amd import tuning
    nq = q.shape[0]
    qk = torch.from_numpy(kq.astype(np.int32)).cuda()
    qL = torch.from_numpy(Lq.astype(np.int32)).cuda()
    kmax, Lmax = int(kq.max()), int(Lq.max())
    order, w = None, 0
    if tiles is not None:
        o = tuning.order_of(tiles["order"], Lq)
        order = None if o is None else torch.from_numpy(o).cuda()
        w = tiles["waves_per_cu"]
    kw = dict(query_L=qL, query_k=qk, order=order, waves_per_cu=w)
    ids, dist, cnt = gi.search(q, kmax, Lmax, want_counters=True, **kw)
    torch.cuda.synchronize()
    iters = cnt.cpu().numpy()[:, 0].astype(np.int64)
    stream = torch.cuda.current_stream()
    ev = [(torch.cuda.Event(enable_timing=True),
           torch.cuda.Event(enable_timing=True)) for _ in range(steps)]
    for e0, e1 in ev:
        e0.record(stream)
        gi.search(q, kmax, Lmax, out=(ids, dist), **kw)
        e1.record(stream)
    torch.cuda.synchronize()
    ms = float(np.mean([e0.elapsed_time(e1) for e0, e1 in ev]))
    link = iters.sum() * 4 * R / (ms / 1e3) / 1e9
    out = {"queries": nq, "k": "uniform over {1, 10, 100}",
           "L": "max(k, round(exp(U[ln 16, ln 256])))",
           "mean_L": round(float(Lq.mean()), 1),
           "qps": round(nq / (ms / 1e3), 1),
           "kernel_ms_mean": round(ms, 3),
           "mean_iterations": round(float(iters.mean()), 2),
           "adjacency_gbs": round(link, 2)}
    if gt is not None:
        sel = kq >= 10
        got = ids.cpu().numpy().view(np.uint32)[sel, :10]
        out["recall10_of_k_ge_10"] = round(recall_at_k(got, gt[sel], 10), 4)
    return out


def mixed_section(run, nq=100_000):
    """Configuration 3's query recipe on the 1M index: 100,000 queries
    (the 10,000 repeated) with k uniform over {1, 10, 100} and
    L = max(k, round(exp(U[ln 16, ln 256]))) in one persistent launch,
    with the autotuned take order and waves per CU against the batch's own
    order at full occupancy."""
    import synth
    from paper_2401_11324_amd import tuning
    torch = run.torch
    reps = -(-nq // run.q.shape[0])
    q = run.q.repeat(reps, 1)[:nq].contiguous()
    gt = np.tile(run.gt, (reps, 1))[:nq]
    kq, Lq = synth.mixed_batch(nq, salt=3)
    tiles, trials = tuning.launch_tiles(run.gi, q, kq, Lq)
    tuned = mixed_launch(run.gi, q, kq, Lq, tiles, run.a.steps, run.w.R, gt)
    plain = mixed_launch(run.gi, q, kq, Lq, None, run.a.steps, run.w.R, gt)
    del q
    torch.cuda.empty_cache()
    return {"tiles": {"chosen": tiles, "trials": trials}, "tuned": tuned,
            "untuned": plain,
            "speedup": round(tuned["qps"] / plain["qps"], 3)}


def copy_probe(mib: int) -> int:
    """A plain copy of `mib` MiB between two device buffers (reads and
    writes exactly that many bytes); its FETCH_SIZE / WRITE_SIZE readings
    turn the counters into bytes."""
    import torch
    n = mib * (1 << 20) // 4
    src = torch.arange(n, dtype=torch.int32, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(3):
        dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"copy_probe_mib": mib, "bytes_each_way": n * 4,
                      "dispatches": 3}), flush=True)
    return 0


def form_adc(T, codes, table):
    """The distance the search ranks by under a table form, as FP64 values
    comparable with the exact ADC, for rows `codes` [P][m] of one query's
    FP32 table T [m][256] (from bang_build_pq_tables).  The forms follow
    their definitions in include/bang.h: FP32, the sum in subspace order;
    F16, entries times 2^-k rounded to half, summed in FP32, times 2^k; U8,
    entries rint((T - lo_j) * 255 / max range) as integers, summed, then
    divided by the scale with the offsets added back."""
    m = T.shape[0]
    f32 = np.float32
    if table == "f32":
        acc = np.zeros(len(codes), dtype=f32)
        for j in range(m):
            acc = (acc + T[j, codes[:, j]]).astype(f32)
        return acc.astype(np.float64)
    if table == "f16":
        mx, mul = f32(T.max()), f32(1.0)
        while f32(mx * mul) > f32(65504.0):
            mul = f32(mul * f32(0.5))
        H = (T * mul).astype(f32).astype(np.float16).astype(f32)
        acc = np.zeros(len(codes), dtype=f32)
        for j in range(m):
            acc = (acc + H[j, codes[:, j]]).astype(f32)
        return acc.astype(np.float64) / float(mul)
    lo = T.min(1)
    rng = (T.max(1) - lo).astype(f32)
    mx = f32(rng.max())
    inv = f32(f32(255.0) / mx) if mx > 0 else f32(0.0)
    Q = np.minimum(np.rint(((T - lo[:, None]).astype(f32) * inv).astype(f32)),
                   255).astype(np.int64)
    isum = np.zeros(len(codes), dtype=np.int64)
    for j in range(m):
        isum += Q[j, codes[:, j]]
    return isum / float(inv) + float(lo.astype(np.float64).sum())


class Runner:
    """One workload's index on the GPU, its recall sweep over L and the
    timed measurement of one table form at one L."""

    def __init__(self, w, a, bang, torch, bf16_base=False):
        from synth import store
        self.w, self.a, self.torch = w, a, torch
        self.d = store.load(w)
        d = self.d
        self.gi = bang.Index(d["base"], d["adj"], d["medoid"],
                             d["codebooks"], d["codes"], bf16_base=bf16_base)
        self.dev = torch.device("cuda:0")
        self.q = torch.from_numpy(d["queries"]).to(self.dev)
        self.gt = d["gt_ids"]
        self.adj = d["adj"]
        self.adj_deg = (d["adj"] != 0xFFFFFFFF).sum(1)
        self.elem = 1 if w.dtype in ("u8", "i8") else 4
        self.rows = []

    def sweep(self, tables):
        """Recall and QPS of every (table, L): one untimed and one timed
        launch each."""
        torch, w, gi, q = self.torch, self.w, self.gi, self.q
        stream = torch.cuda.current_stream()
        nq, k = q.shape[0], w.k
        for table in tables:
            for L in w.Ls:
                ids, dist = gi.search(q, k, L, table=table)
                torch.cuda.synchronize()
                t0 = torch.cuda.Event(enable_timing=True)
                t1 = torch.cuda.Event(enable_timing=True)
                t0.record(stream)
                gi.search(q, k, L, out=(ids, dist), table=table)
                t1.record(stream)
                torch.cuda.synchronize()
                rec = recall_at_k(ids.cpu().numpy().view(np.uint32), self.gt,
                                  k)
                self.rows.append({"table": table, "L": L,
                                  "recall10": round(rec, 4),
                                  "qps": round(nq / (t0.elapsed_time(t1)
                                                     / 1e3))})
        return self.rows

    def pick_L(self, table):
        """The smallest swept L whose recall@10 reaches the target, else
        the L with the best recall (or --L when given)."""
        if self.a.L:
            return self.a.L
        rows = [s for s in self.rows if s["table"] == table]
        ok = [s for s in rows if s["recall10"] >= TARGET_RECALL]
        return ok[0]["L"] if ok else max(rows, key=lambda s: s["recall10"])["L"]

    def adc_error(self, table, cand, iters, nq=100, per_q=256,
                  bf16_tables=False):
        """Relative error of the distance the search ranks by under a table
        form, against the ADC in FP64 (the same codes, the codebooks and
        query in FP64), over the first nq queries and up to per_q of each
        one's expanded nodes (the nodes the search ranked); bf16_tables:
        the table built by BF16 MFMA."""
        torch = self.torch
        d, m = self.d, self.w.m
        ds = self.w.d // m
        T = self.gi.build_pq_tables(self.q[:nq], bf16=bf16_tables)
        torch.cuda.synchronize()
        T = T.cpu().numpy().reshape(nq, m, 256)
        cb = d["codebooks"].astype(np.float64)  # [m][256][ds]
        qn = d["queries"][:nq].astype(np.float64)
        errs = []
        for i in range(nq):
            ex = cand[i, :min(int(iters[i]), per_q)]
            codes = d["codes"][ex].astype(np.int64)
            qs = qn[i].reshape(m, 1, ds)
            T64 = ((qs - cb) ** 2).sum(-1)  # [m][256]
            ref = T64[np.arange(m)[None, :], codes].sum(1)
            got = form_adc(T[i], codes, table)
            errs.append(np.abs(got - ref) / np.maximum(ref, 1e-30))
        e = np.concatenate(errs)
        return {"pairs": int(e.size), "max": float(e.max()),
                "mean": float(e.mean()),
                "p99": float(np.percentile(e, 99))}

    def bf16_error(self, cand, iters, nq=100, per_q=128):
        """Relative error against FP64 of the distances the BF16 re-rank
        sums first (bfloat16 rows, FP32 sums in coordinate order) and of
        the canonical FP32 distances, over the first nq queries and up to
        per_q of each one's expanded nodes."""
        base, qs = self.d["base"], self.d["queries"]
        e16, e32 = [], []
        for i in range(nq):
            ex = cand[i, :min(int(iters[i]), per_q)]
            x = base[ex]
            b = x.view(np.uint32).astype(np.uint64)
            b = ((b + 0x7FFF + ((b >> 16) & 1)) >> 16) << 16
            xb = b.astype(np.uint32).view(np.float32)
            q = qs[i]
            ref = ((x.astype(np.float64) - q.astype(np.float64)) ** 2).sum(1)
            acc16 = np.zeros(len(ex), dtype=np.float32)
            acc32 = np.zeros(len(ex), dtype=np.float32)
            for t in range(x.shape[1]):
                acc16 = acc16 + (xb[:, t] - q[t]) * (xb[:, t] - q[t])
                acc32 = acc32 + (x[:, t] - q[t]) * (x[:, t] - q[t])
            den = np.maximum(ref, 1e-30)
            e16.append(np.abs(acc16 - ref) / den)
            e32.append(np.abs(acc32 - ref) / den)
        e16, e32 = np.concatenate(e16), np.concatenate(e32)
        return {"pairs": int(e16.size), "bf16_max": float(e16.max()),
                "bf16_mean": float(e16.mean()),
                "fp32_max": float(e32.max()), "fp32_mean": float(e32.mean())}

    def measure(self, table, L, index=None, filter="exact", rerank="exact",
                bf16_tables=False, seen_cache=True):
        """K timed steps of one form; returns its record.  bf16_tables: a
        step is the BF16-MFMA table build followed by the search ranking by
        those tables.  seen_cache=False: the exact-distance search without
        its seen-id cache."""
        torch, w, a = self.torch, self.w, self.a
        gi_ = index or self.gi
        q, dev, gt = self.q, self.dev, self.gt
        stream = torch.cuda.current_stream()
        nq, k = q.shape[0], w.k
        ids = torch.empty((nq, k), dtype=torch.int32, device=dev)
        dist = torch.empty((nq, k), dtype=torch.float32, device=dev)
        tabs = (gi_.build_pq_tables(q, bf16=True) if bf16_tables else None)

        def step():
            if bf16_tables:
                gi_.build_pq_tables(q, out=tabs, bf16=True)
            gi_.search(q, k, L, out=(ids, dist), table=table, filter=filter,
                       rerank=rerank, tables=tabs, seen_cache=seen_cache)

        for _ in range(a.warmup):
            step()
        torch.cuda.synchronize()
        ev = [(torch.cuda.Event(enable_timing=True),
               torch.cuda.Event(enable_timing=True)) for _ in range(a.steps)]
        wall0 = time.perf_counter()
        for e0, e1 in ev:
            e0.record(stream)
            step()
            e1.record(stream)
        torch.cuda.synchronize()
        wall = time.perf_counter() - wall0
        per = np.array([e0.elapsed_time(e1) for e0, e1 in ev])  # ms/launch
        got_ids = ids.cpu().numpy().view(np.uint32)
        rec = recall_at_k(got_ids, gt, k)
        # distance error against the FP64 ground truth, over the returned
        # ids that are true neighbours
        gd = self.d["gt_dists"][:, :k]
        hit = got_ids == self.d["gt_ids"][:, :k]
        dd = dist.cpu().numpy().astype(np.float64)
        rel = np.abs(dd[hit] - gd[hit]) / np.maximum(gd[hit], 1e-30)
        # one more (untimed) launch with counters, expanded nodes, stamps
        cap = max(4 * L, L + 64)
        _, _, cand, cnt, times = gi_.search(q, k, L, want_cand=cap,
                                           want_counters=True,
                                           want_times=True, table=table,
                                           filter=filter, rerank=rerank,
                                           tables=tabs, seen_cache=seen_cache)
        torch.cuda.synchronize()
        cand = cand.cpu().numpy().view(np.uint32)
        cnt = cnt.cpu().numpy()
        iters, status = cnt[:, 0], cnt[:, 1]
        t = times.cpu().numpy().astype(np.float64)
        # completion time of each query after the batch began, scaled so
        # that the span of the device clock equals the measured kernel time
        span = max(1.0, t[:, 1].max() - t[:, 0].min())
        kern_ms = float(per.mean())
        lat_ms = (t[:, 1] - t[:, 0].min()) / span * kern_ms
        exact = table == "exact"
        if filter == "exact":
            # |N'| counted on every NPRIME_EVERY-th query (a fixed sample),
            # scaled to the batch by expansions
            sel = np.arange(0, nq, NPRIME_EVERY)
            ns = unseen_neighbours(self.adj, int(self.d["medoid"]),
                                   iters[sel], cand[sel])
            per_exp = ns.sum() / max(1, iters[sel].astype(np.int64).sum())
            nprime = per_exp * iters.astype(np.float64)
        else:
            nprime = None  # a lossy filter: |N'| is not the exact set's
        design = packed_row_bytes(self.adj_deg, w.R, w.m, w.d, self.elem, k,
                                  iters, cand, 4 * L, exact=exact)
        ms_step = wall * 1e3 / a.steps
        recd = {"table": table, "L": L, "filter": filter, "rerank": rerank,
                "table_build": "bf16_mfma" if bf16_tables else "fp32",
                "recall10": round(rec, 4),
                "adjacency_bytes_per_launch": int(iters.astype(np.int64).sum()
                                                  * 4 * w.R),
                "qps": round(nq / (ms_step / 1e3), 1),
                "ms_per_step": round(ms_step, 4),
                "latency": "per-query completion time after the launch "
                           f"began, within one batch of {nq} queries",
                "p50_ms": round(float(np.percentile(lat_ms, 50)), 4),
                "p99_ms": round(float(np.percentile(lat_ms, 99)), 4),
                "mean_iterations": round(float(iters.mean()), 2),
                "iteration_capped_queries": int((status == 1).sum()),
                "lambda_pct": round(iteration_overhead(float(iters.mean()),
                                                       L), 2),
                "kernel_ms_mean": round(kern_ms, 4),
                "packed_row_bytes_per_launch": design,
                "packed_row_gbs": round(design / (kern_ms / 1e3) / 1e9, 2),
                "result_rel_dist_err_vs_fp64": float(rel.max()) if rel.size
                else 0.0}
        if not exact:
            recd["adc_rel_err_vs_fp64"] = self.adc_error(
                table, cand, iters, bf16_tables=bf16_tables)
        if rerank == "bf16":
            ncand = np.minimum(iters.astype(np.int64), 4 * L)
            recd["bf16_rerank"] = {
                "rechecked_fp32": int(cnt[:, 2].astype(np.int64).sum()),
                "candidates": int(ncand.sum()),
                "rechecked_frac": round(float(cnt[:, 2].astype(np.int64).sum()
                                              / max(1, ncand.sum())), 4),
                "bf16_dist_rel_err_vs_fp64": self.bf16_error(cand, iters)}
        if nprime is not None:
            B, parts = method_bytes(nprime, w.R, w.m, w.d, self.elem, k,
                                    iters, 4 * L, exact=exact)
            recd.update({
                "mean_unseen_per_expansion": round(float(per_exp), 3),
                "unseen_sample": f"every {NPRIME_EVERY}th query "
                                 f"({len(sel)} of {nq})",
                "expansions": int(iters.astype(np.int64).sum()),
                "method_bytes_per_launch": B,
                "method_bytes_parts": parts,
                "achieved_gbs": round(B / (kern_ms / 1e3) / 1e9, 2),
                "packed_row_over_method": round(design / B, 3)})
        return recd


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--L", type=int, default=0,
                    help="worklist size for every form (default: chosen by "
                         "the recall sweep)")
    ap.add_argument("--no-cpu", action="store_true",
                    help="skip the CPU oracle baseline")
    ap.add_argument("--no-sweep", action="store_true",
                    help="skip the recall sweep (needs --L)")
    ap.add_argument("--no-host", action="store_true",
                    help="skip the host-resident adjacency measurement")
    ap.add_argument("--no-serve", action="store_true",
                    help="skip the serving-loop measurement")
    ap.add_argument("--no-ablation", action="store_true",
                    help="skip the batch-size, PQ-subspace and Bloom-filter "
                         "studies")
    ap.add_argument("--no-deep", action="store_true",
                    help="skip the precision form on the d=96 float index")
    ap.add_argument("--scale-host", type=int, default=0, metavar="N",
                    help="only measure the host-resident adjacency on a "
                         "synthetic N-node int8 graph (throughput at scale, "
                         "no recall) and exit")
    ap.add_argument("--copy-probe", type=int, default=0, metavar="MIB",
                    help="only run a plain device copy of MIB mebibytes "
                         "(calibrates the HBM byte counters) and exit")
    a = ap.parse_args(argv)
    if a.copy_probe:
        return copy_probe(a.copy_probe)
    if a.scale_host:
        return scale_host(a)
    if a.no_sweep and not a.L:
        ap.error("--no-sweep needs --L")
    if a.gpus != 1:
        print(f"bench.py: this build runs on one GPU; --gpus {a.gpus} is not "
              "supported (queries are independent: see the sharding notes in "
              "the design document)", file=sys.stderr)
        return 2

    import torch
    import synth
    from synth import store
    import paper_2401_11324_amd as bang

    w = synth.WORKLOADS[WORKLOAD]
    if not store.exists(w):
        print(f"bench.py: index files for {w.name} are missing under "
              f"{store.DEFAULT_ROOT}; write them with "
              f"`python -m oracle.build_index {w.name}`", file=sys.stderr)
        return 3
    run = Runner(w, a, bang, torch)
    t0 = time.perf_counter()

    def progress(msg):
        # one line per finished section on stderr (the JSON line stays the
        # only output on stdout)
        print(f"[bench {time.perf_counter() - t0:6.1f}s] {msg}",
              file=sys.stderr, flush=True)
    d, gi, gt, k = run.d, run.gi, run.gt, w.k
    sweep = run.sweep(() if a.no_sweep else TABLES + ("exact",))
    pick_L = run.pick_L
    measure = run.measure

    progress("L sweep")
    plain = measure("f32", pick_L("f32"))
    progress("plain FP32")
    prec = {t: measure(t, pick_L(t)) for t in ("f16", "u8")}
    # the same forms ranking by tables built with BF16 MFMA (a step builds
    # them, then searches by them), at each form's point
    for t, rec0 in (("f32", plain), ("f16", prec["f16"]), ("u8", prec["u8"])):
        rec = measure(t, rec0["L"], bf16_tables=True)
        rec["recall_lost_vs_fp32_tables_same_L"] = round(
            rec0["recall10"] - rec["recall10"], 4)
        prec[t + "+bf16_mfma_tables"] = rec
    prec["table_build"] = table_build_section(run)
    progress("precision forms")
    # the paper's Exact-distance Version: no table, no re-rank
    exact = None if a.no_sweep and not a.L else measure("exact",
                                                         pick_L("exact"))
    if exact is not None:
        # the same point without the seen-id cache, which reads every
        # neighbour's base row (the packed-row figures above count that
        # design's reads)
        nc = measure("exact", exact["L"], seen_cache=False)
        exact["without_seen_cache"] = {
            "qps": nc["qps"], "kernel_ms_mean": nc["kernel_ms_mean"],
            "recall10": nc["recall10"]}
        exact["seen_cache_speedup"] = round(exact["qps"] / nc["qps"], 3)
        progress("exact distances")
    L = plain["L"]
    host = None
    if not a.no_host:
        # the same search with the adjacency in pinned host memory, read
        # across the host link (the paper's CPU-resident graph)
        hi = bang.Index(d["base"], d["adj"], d["medoid"], d["codebooks"],
                        d["codes"], host_adj=True)
        host = measure("f32", L, index=hi)
        hprobe = gather_probe(hi, torch, 1 << 20)
        hi.close()
        link = host["adjacency_bytes_per_launch"] / (
            host["kernel_ms_mean"] / 1e3) / 1e9
        host["host_link"] = {
            "bound": "host link", "achieved": round(link, 2),
            "peak": HOST_LINK_PEAK_GBS, "unit": "GB/s",
            "frac": round(link / HOST_LINK_PEAK_GBS, 4),
            "bytes": "adjacency rows, 4R bytes per expansion",
            "random_row_probe": hprobe,
            "frac_of_probe": round(link / hprobe["gbs"], 4)}
        progress("host-resident adjacency")
    # the rate at which random packed rows can be read at all (the search's
    # access pattern with no work between reads)
    probe = gather_probe(gi, torch, 1 << 22)
    traffic = None
    if os.path.exists(TRAFFIC_FILE):
        with open(TRAFFIC_FILE) as f:
            tr = json.load(f)
        if tr.get("kernel_hash") == kernel_hash() and tr.get("L") == L:
            traffic = tr.get("bytes_per_launch")

    out = {
        "metric": METRIC,
        "value": plain["qps"],
        "unit": "queries/s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": plain["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            "workload": "sift1m-like Gaussian mixture: n=1,000,000 d=128 "
                        "uint8, 1,000 centres U[0,255], sigma 20; 10,000 "
                        "queries; graph R=64 L_build=100 alpha=1.2; PQ m=32",
            "form": "plain FP32",
            "k": k, "L": L, "recall10": plain["recall10"],
            "target_recall10": TARGET_RECALL,
            "target_met": bool(plain["recall10"] >= TARGET_RECALL),
            "mean_iterations": plain["mean_iterations"],
            "lambda_pct": plain["lambda_pct"],
            "sweep": sweep,
        },
        "p50_ms": plain["p50_ms"],
        "p99_ms": plain["p99_ms"],
        "roofline": {
            "bound": "hbm",
            "kernel": "search_kernel<u8 data, m=32, d/m=4, FP32 table>",
            "achieved": plain["achieved_gbs"],
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": round(plain["achieved_gbs"] / HBM_PEAK_GBS, 5),
            "traffic": traffic,
            "bytes": "the method's bytes per launch: per expansion the "
                     "adjacency row (4R), visited-set probes (8R) and the "
                     "codes of the unseen neighbours (m each); re-ranked "
                     "base rows, queries and results",
            "method_bytes_per_launch": plain["method_bytes_per_launch"],
            "method_bytes_parts": plain["method_bytes_parts"],
            "mean_unseen_per_expansion":
                plain["mean_unseen_per_expansion"],
            "packed_row_bytes_per_launch":
                plain["packed_row_bytes_per_launch"],
            "packed_row_over_method": plain["packed_row_over_method"],
            "traffic_over_method": (round(traffic /
                                          plain["method_bytes_per_launch"], 3)
                                    if traffic else None),
            "kernel_ms_mean": plain["kernel_ms_mean"],
            "random_row_probe": probe,
        },
        "precision_form": prec,
    }
    if host is not None:
        out["host_resident"] = host
    if not a.no_ablation:
        out["batch_size"] = batch_section(run, L)
        progress("batch sizes")
        out["pq_subspaces"] = m_section(run, bang)
        progress("subspace counts")
        pts = [("f32", L, plain)]
        if exact is not None:
            pts.append(("exact", exact["L"], exact))
        out["bloom_filter"] = bloom_section(run, pts)
        progress("Bloom filter")
        out["mixed_batch"] = mixed_section(run)
        progress("mixed batch")
        # plus a small worklist, where the once-per-query table build and
        # re-rank weigh most
        out["phase_split"] = phase_section(
            run, [("f32", L), ("u8", prec["u8"]["L"])] +
            ([("exact", exact["L"])] if exact is not None else []) +
            ([("f32", 64)] if L != 64 else []))
        progress("phase split")
    if not a.no_serve:
        out["serving"] = serving_section(gi, d, w, gt)
        progress("serving")
    if not a.no_deep:
        out["precision_form_deep1m"] = deep_section(a, bang, torch)
        progress("deep1m")
    if exact is not None:
        out["exact_distance"] = exact
    if not a.no_cpu:
        out["cpu_baseline"] = cpu_baseline(d, d["queries"], k, L)
        progress("CPU baseline")
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
