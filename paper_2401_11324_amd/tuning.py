"""Autotuner for one persistent search launch (a large mixed batch).

A launch's waves take the queries one at a time from a counter, so the only
choices left are the order in which they are taken and how many waves stay
resident per CU.  Neither changes any result.  `launch_tiles` times each
candidate on a calibration slice of the batch and keeps the fastest; the
"longest first" order gives the queries with the widest worklists (the
most expansions) to the first waves, so that no long query starts late and
holds the launch open after the others have drained.
"""
from __future__ import annotations

import numpy as np

ORDERS = ("given", "longest_first")
WAVES_PER_CU = (0, 3, 2)  # 0: as many as LDS and registers allow


def order_of(name: str, query_L: np.ndarray) -> np.ndarray | None:
    """The take order of a named policy (None: the batch's own order)."""
    if name == "given":
        return None
    if name == "longest_first":
        return np.argsort(-np.asarray(query_L, np.int64),
                          kind="stable").astype(np.int32)
    raise ValueError(name)


def time_launch(index, q, k, L, qL, qk, order, waves_per_cu, table, reps):
    import torch
    nq = q.shape[0]
    ids = torch.empty((nq, k), dtype=torch.int32, device=q.device)
    dist = torch.empty((nq, k), dtype=torch.float32, device=q.device)
    kw = dict(query_L=qL, query_k=qk, table=table, order=order,
              waves_per_cu=waves_per_cu, out=(ids, dist))
    index.search(q, k, L, **kw)
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    ts = []
    for _ in range(reps):
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        index.search(q, k, L, **kw)
        e1.record(stream)
        torch.cuda.synchronize()
        ts.append(e0.elapsed_time(e1))
    return float(np.mean(ts))


def launch_tiles(index, queries, k_q: np.ndarray, L_q: np.ndarray,
                 table: str = "f32", calib: int = 20000, reps: int = 3):
    """Choose (order, waves_per_cu) for one persistent launch of `queries`
    (a CUDA tensor [nq][d]) with per-query k_q and L_q (numpy), timing
    every candidate on the first `calib` queries.  Returns (choice dict,
    trials list)."""
    import torch
    dev = queries.device
    nc = min(calib, queries.shape[0])
    q = queries[:nc].contiguous()
    kc, Lc = np.asarray(k_q[:nc]), np.asarray(L_q[:nc])
    qk = torch.from_numpy(kc.astype(np.int32)).to(dev)
    qL = torch.from_numpy(Lc.astype(np.int32)).to(dev)
    k, L = int(kc.max()), int(Lc.max())
    trials = []
    for name in ORDERS:
        o = order_of(name, Lc)
        ot = None if o is None else torch.from_numpy(o).to(dev)
        for w in WAVES_PER_CU:
            ms = time_launch(index, q, k, L, qL, qk, ot, w, table, reps)
            trials.append({"order": name, "waves_per_cu": w,
                           "ms": round(ms, 4),
                           "qps": round(nc / (ms / 1e3), 1)})
    best = min(trials, key=lambda t: t["ms"])
    return {"order": best["order"], "waves_per_cu": best["waves_per_cu"],
            "calibration_queries": nc}, trials
