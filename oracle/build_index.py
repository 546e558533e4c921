"""Write the index files of a workload using only the oracle.

    python -m oracle.build_index tiny
    python -m oracle.build_index sift1m [--threads N]
    python -m oracle.build_index sift1m --extra-m 16 64

The second form adds, beside an existing index, the base encoded with other
numbers of subspaces (codebooks_m<m>, codes_m<m>): the same training sample,
the k-means init stream from its start.

Steps: generate base vectors and queries (synth), train PQ on a seeded
sample, encode every base vector, pick the medoid, build the graph (Vamana
plus the navigability devices of oracle/graph.py) over a seeded insertion
order, and compute exact ground truth.  Everything
but the generator is oracle code, so nothing stored here comes from the GPU
path.  Output goes to synth.store's directory (indexcache/<workload>/).
"""
from __future__ import annotations

import argparse
import sys
import time

import numpy as np

import synth
from synth import store

from . import bruteforce, medoid, default_threads
from .graph import build_graph
from .pq import train_pq, pq_encode

K_GT = 10


def build(w: synth.Workload, nthreads: int = 0, root: str | None = None,
          log=print) -> str:
    nthreads = nthreads or default_threads()
    t0 = time.time()
    rs = synth.streams(w)
    base, queries = synth.base_and_queries(w)
    log(f"[{w.name}] data {base.shape} {base.dtype} + queries {queries.shape} "
        f"({time.time() - t0:.1f}s)")
    ns = min(w.n, w.pq_sample)
    sample = base[np.sort(rs["pq_sample"].choice(w.n, ns, replace=False))]
    cb = train_pq(sample, w.m, w.kmeans_iters, rs["pq_init"], nthreads)
    log(f"[{w.name}] PQ trained m={w.m} ({time.time() - t0:.1f}s)")
    codes = pq_encode(base, cb, nthreads)
    log(f"[{w.name}] encoded ({time.time() - t0:.1f}s)")
    s = medoid(base)
    perm = rs["vamana_order"].permutation(w.n).astype(np.uint32)
    adj, ginfo = build_graph(base, w.R, w.L_build, w.alpha, perm, s,
                             nthreads=nthreads)
    reach = ginfo["reachable"]
    deg = (adj != 0xFFFFFFFF).sum(1)
    log(f"[{w.name}] graph R={w.R} L={w.L_build} alpha={w.alpha}: mean degree "
        f"{deg.mean():.1f}, {ginfo} ({time.time() - t0:.1f}s)")
    gt_ids, gt_d = bruteforce(base, queries, K_GT, nthreads)
    log(f"[{w.name}] ground truth ({time.time() - t0:.1f}s)")
    p = store.save(w, {"codebooks": cb, "codes": codes, "adj": adj,
                       "gt_ids": gt_ids, "gt_dists": gt_d}, s,
                   extra={"reachable": reach, "mean_degree": float(deg.mean()),
                          "graph": ginfo,
                          "build_seconds": time.time() - t0,
                          "threads": nthreads},
                   base=base, queries=queries, root=root)
    log(f"[{w.name}] wrote {p}")
    return p


def add_pq(w: synth.Workload, ms, nthreads: int = 0, root: str | None = None,
           log=print) -> str:
    nthreads = nthreads or default_threads()
    t0 = time.time()
    base, _ = synth.base_and_queries(w)
    ns = min(w.n, w.pq_sample)
    arrays = {}
    for m in ms:
        rs = synth.streams(w)
        sample = base[np.sort(rs["pq_sample"].choice(w.n, ns, replace=False))]
        cb = train_pq(sample, m, w.kmeans_iters, rs["pq_init"], nthreads)
        arrays[f"codebooks_m{m}"] = cb
        arrays[f"codes_m{m}"] = pq_encode(base, cb, nthreads)
        log(f"[{w.name}] PQ m={m} trained and encoded ({time.time() - t0:.1f}s)")
    p = store.save_extra(w, arrays, root=root)
    log(f"[{w.name}] added {sorted(arrays)} to {p}")
    return p


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("workload", choices=sorted(synth.WORKLOADS))
    ap.add_argument("--threads", type=int, default=0)
    ap.add_argument("--root", default=None)
    ap.add_argument("--extra-m", type=int, nargs="+", default=None)
    a = ap.parse_args(argv)
    if a.extra_m:
        add_pq(synth.WORKLOADS[a.workload], a.extra_m, a.threads, a.root)
    else:
        build(synth.WORKLOADS[a.workload], a.threads, a.root)


if __name__ == "__main__":
    sys.exit(main())
