"""Property tests of the oracle's search on random small graphs
(hypothesis): the facts below hold for any graph and query, so they pin the
search loop independently of how an index was built.

* Algorithm 1 (set union into the worklist) and the filtered form of
  Algorithm 2 (seen-set, sort, merge) expand the same nodes in the same
  order and answer the same (section "Greedy Search", Algorithms 1 and 2).
* With t >= n and every node reachable from s, every node is expanded and
  the exact-distance answer is the brute-force k nearest.
* Every answer is sorted by (distance, id) and holds distinct ids; every
  expanded node is distinct and at most iter_cap nodes are expanded.
"""
import numpy as np
import pytest
from hypothesis import HealthCheck, given, settings, strategies as st

import oracle

NONE = 0xFFFFFFFF


def random_index(seed, n, R, d, dtype):
    rng = np.random.default_rng(seed)
    if dtype == "u8":
        base = rng.integers(0, 256, size=(n, d), dtype=np.uint8)
    else:
        base = rng.standard_normal((n, d)).astype(np.float32)
    adj = np.full((n, R), NONE, dtype=np.uint32)
    for u in range(n):
        deg = int(rng.integers(0, R + 1))
        nb = rng.choice(n, size=min(deg, n), replace=False)
        adj[u, :len(nb)] = nb
    m = d // 2
    cb = rng.standard_normal((m, 256, 2)).astype(np.float32) * (
        60.0 if dtype == "u8" else 1.0) + (128.0 if dtype == "u8" else 0.0)
    codes = rng.integers(0, 256, size=(n, m), dtype=np.uint8)
    s = int(rng.integers(0, n))
    q = (rng.integers(0, 256, size=(3, d), dtype=np.uint8) if dtype == "u8"
         else rng.standard_normal((3, d)).astype(np.float32))
    return oracle.Index(base, adj, s, cb, codes), q


cases = st.tuples(st.integers(0, 2**31 - 1), st.integers(2, 40),
                  st.integers(1, 6), st.sampled_from(["u8", "f32"]),
                  st.integers(1, 12), st.sampled_from(["f32", "u8", "exact"]))


@settings(max_examples=60, deadline=None,
          suppress_health_check=[HealthCheck.too_slow])
@given(cases)
def test_algorithm1_equals_filtered_form(case):
    seed, n, R, dtype, L, table = case
    ix, q = random_index(seed, n, R, 4, dtype)
    k = min(L, 3)
    a = oracle.search(ix, q, k, L, mode=0, table=table, want_pq=True,
                      want_cand=True)
    b = oracle.search(ix, q, k, L, mode=1, table=table, want_pq=True,
                      want_cand=True)
    for key in ("ids", "dists", "pq_ids", "pq_dists", "cand", "iters",
                "status"):
        assert np.array_equal(a[key], b[key]), key
    cap = oracle.iter_cap_for(L)
    for qi in range(len(q)):
        I = a["iters"][qi]
        assert 1 <= I <= cap
        c = a["cand"][qi][:I]
        assert len(set(c.tolist())) == I
        ids, d = a["ids"][qi], a["dists"][qi]
        valid = ids != NONE
        keys = list(zip(d[valid].tolist(), ids[valid].tolist()))
        assert keys == sorted(keys) and len(set(ids[valid].tolist())) == len(
            keys)
        assert (~valid[:valid.sum()]).sum() == 0  # padding only at the end


@settings(max_examples=40, deadline=None,
          suppress_health_check=[HealthCheck.too_slow])
@given(st.tuples(st.integers(0, 2**31 - 1), st.integers(2, 40),
                 st.sampled_from(["u8", "f32"])))
def test_t_at_least_n_on_connected_graph_is_brute_force(case):
    seed, n, dtype = case
    ix, q = random_index(seed, n, 6, 4, dtype)
    # make every node reachable: a ring from s through all nodes
    order = np.random.default_rng(seed).permutation(n)
    order = np.concatenate([[ix.medoid], order[order != ix.medoid]])
    adj = ix.adj.copy()
    for a_, b_ in zip(order, np.roll(order, -1)):
        row = adj[a_]
        if b_ not in row:
            row[-1] = b_
    ix = oracle.Index(ix.base, adj, ix.medoid, ix.codebooks, ix.codes)
    assert oracle.reachable(adj, ix.medoid) == n
    k = min(n, 5)
    out = oracle.search(ix, q, k, n, iter_cap=n + 1, table="exact")
    assert (out["iters"] == n).all()
    for qi in range(len(q)):
        if dtype == "u8":
            ex = ((ix.base.astype(np.int64) - q[qi].astype(np.int64))
                  ** 2).sum(1)
        else:
            ex = ((ix.base.astype(np.float64) - q[qi].astype(np.float64))
                  ** 2).sum(1)
        order_ = np.lexsort((np.arange(n), ex))[:k]
        if dtype == "u8":
            assert out["ids"][qi].tolist() == order_.tolist()
        else:
            # FP32 sums may reorder near-ties against the FP64 reference
            np.testing.assert_allclose(np.sort(out["dists"][qi]),
                                       np.sort(ex[order_]), rtol=1e-5)
