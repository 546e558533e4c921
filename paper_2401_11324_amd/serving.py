"""Measurement and tuning of the serving loop (Server).

`run_load` replays an open-loop request stream through a Server and sums
it up (offered and sustained query rates, p50/p99 request latency);
`autotune` picks the server's batch size, slot count and whether slots
replay captured HIP graphs, for a load: it replays the same calibration
stream through each candidate configuration and keeps the one with the
highest sustained rate whose p99 latency stays within the target (else the
one with the lowest p99).
"""
from __future__ import annotations

import numpy as np

from . import Server


def run_load(index, queries, req, max_batch: int, slots: int, max_k: int,
             max_L: int, table: str = "f32", graphs: bool = False):
    """Replay `req` (synth.serving_requests output) through a new Server;
    returns (summary dict, ids, dists)."""
    sv = Server(index, max_batch=max_batch, slots=slots, max_k=max_k,
                max_L=max_L, table=table, graphs=graphs)
    try:
        ids, d, lat = sv.replay(queries[req["rows"]], req["nq"], req["k"],
                                req["L"], req["arrival_s"],
                                kstride=int(req["k"].max()))
        st = sv.stats()
    finally:
        sv.close()
    arr = req["arrival_s"]
    done = arr + lat
    nq = int(req["nq"].sum())
    span = float(done.max() - arr.min()) if len(arr) else 0.0
    offered = nq / float(max(arr.max(), 1e-9)) if len(arr) > 1 else 0.0
    out = {"max_batch": max_batch, "slots": slots, "graphs": bool(graphs),
           "requests": len(arr),
           "queries": nq, "offered_qps": round(offered, 1),
           "sustained_qps": round(nq / span, 1) if span > 0 else 0.0,
           "p50_ms": round(float(np.percentile(lat, 50)) * 1e3, 3),
           "p99_ms": round(float(np.percentile(lat, 99)) * 1e3, 3),
           "launches": st["launches"],
           "mean_batch": round(st["queries"] / max(1, st["launches"]), 1),
           "max_slots_busy": st["max_in_flight"]}
    return out, ids, d


def autotune(index, queries, req, candidates, max_k: int, max_L: int,
             p99_target_ms: float, table: str = "f32"):
    """Try each (max_batch, slots[, graphs]) on the calibration stream
    `req`; return (best (max_batch, slots, graphs), list of per-candidate
    summaries)."""
    trials = []
    for c in candidates:
        mb, sl = c[0], c[1]
        gr = bool(c[2]) if len(c) > 2 else False
        s, _, _ = run_load(index, queries, req, mb, sl, max_k, max_L, table,
                           graphs=gr)
        trials.append(s)
    best = choose(trials, p99_target_ms)
    return (best["max_batch"], best["slots"], best["graphs"]), trials


def choose(trials, p99_target_ms: float) -> dict:
    """The trial with the highest sustained rate among those within the
    p99 target, else the one with the lowest p99.  Sustained rates within
    1% of the best count as equal; the lower p99 then decides."""
    ok = [t for t in trials if t["p99_ms"] <= p99_target_ms]
    if not ok:
        return min(trials, key=lambda t: t["p99_ms"])
    top = max(t["sustained_qps"] for t in ok)
    near = [t for t in ok if t["sustained_qps"] >= 0.99 * top]
    return min(near, key=lambda t: t["p99_ms"])
