"""GPU parity: the HIP path (through the C ABI) against the CPU oracle on the
same seeded inputs.  The bar is bit-exact: ids, distances, the order of
expanded nodes and the iteration counts must be identical, because both
sides compute FP32 sums in the same fixed order with no fused
multiply-add.  (The stated tolerance for distances is 1e-5 relative; the
design reaches exact equality, which the tests require.)"""
import numpy as np
import pytest

import oracle
import synth
from oracle.graph import build_graph
from oracle.pq import pq_encode, train_pq
from synth import store

pytestmark = pytest.mark.gpu
NONE = 0xFFFFFFFF

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a visible GPU")
    import paper_2401_11324_amd as bang  # raises if the library is missing
    bang.lib()


def bang_mod():
    import paper_2401_11324_amd as bang
    return bang


def make_index(w):
    rs = synth.streams(w)
    base, q = synth.base_and_queries(w)
    cb = train_pq(base, w.m, w.kmeans_iters, rs["pq_init"])
    codes = pq_encode(base, cb)
    s = oracle.medoid(base)
    perm = rs["vamana_order"].permutation(w.n).astype(np.uint32)
    adj, _ = build_graph(base, w.R, w.L_build, w.alpha, perm, s)
    return oracle.Index(base, adj, s, cb, codes), q


SMALL = {
    # (dtype, d, m): covers the three element types and d/m = 2, 4 and 8
    "f32-d32-m16": synth.small("f32", n=1500, d=32, nq=37, m=16, R=24,
                               seed_index=110),
    "u8-d64-m16": synth.small("u8", n=2000, d=64, nq=41, m=16, R=32,
                              seed_index=111),
    "i8-d96-m48": synth.small("i8", n=1200, d=96, nq=29, m=48, R=20,
                              seed_index=112),
    "u8-d128-m32": synth.small("u8", n=3000, d=128, nq=45, m=32, R=64,
                               ncent=12, seed_index=113),
    # d/m = 8 (the m = 16 encoding of d = 128 data)
    "f32-d128-m16": synth.small("f32", n=1600, d=128, nq=31, m=16, R=32,
                                seed_index=114),
}


@pytest.fixture(scope="module")
def small_indexes():
    out = {}
    for name, w in SMALL.items():
        ix, q = make_index(w)
        out[name] = (ix, q, bang_mod().Index(ix.base, ix.adj, ix.medoid,
                                             ix.codebooks, ix.codes))
    return out


def to_dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def u32(t):
    return t.cpu().numpy().view(np.uint32)


def f32bits(a):
    return np.ascontiguousarray(a, dtype=np.float32).view(np.uint32)


# the oracle's search mode for each GPU visited filter: the set union
# (Algorithm 1), the exact seen-set (Algorithm 2 without false positives)
# and the paper's Bloom filter
ORACLE_MODE = {"exact": "union", "seen": "exact", "bloom": "bloom"}


def run_and_compare(ix, gi, q, k, L, c_max=0, iter_cap=0, label="",
                    table="f32", rerank_global=False, filter="exact",
                    rerank="exact", seen_log_short=False):
    cap = iter_cap or oracle.iter_cap_for(L)
    qt = to_dev(q)
    ids, d, cand, cnt = gi.search(qt, k, L, c_max=c_max, iter_cap=iter_cap,
                                  want_cand=cap, want_counters=True,
                                  table=table, rerank_global=rerank_global,
                                  filter=filter, rerank=rerank,
                                  seen_log_short=seen_log_short)
    torch.cuda.synchronize()
    ref = oracle.search(ix, q, k, L, c_max=c_max or None,
                        iter_cap=iter_cap or None, want_cand=True,
                        table=table, mode=oracle.MODES[ORACLE_MODE[filter]])
    ids, d, cand, cnt = u32(ids), d.cpu().numpy(), u32(cand), u32(cnt)
    assert np.array_equal(cnt[:, 0], ref["iters"]), label
    assert np.array_equal(cnt[:, 1], ref["status"]), label
    assert np.array_equal(cand, ref["cand"]), label
    assert np.array_equal(ids, ref["ids"]), label
    assert np.array_equal(f32bits(d), f32bits(ref["dists"])), label
    return ref


# --------------------------------------------------------------------------
# stage 1
# --------------------------------------------------------------------------
@pytest.mark.parametrize("name", list(SMALL))
def test_tables_bit_exact(small_indexes, name):
    ix, q, gi = small_indexes[name]
    T = gi.build_pq_tables(to_dev(q))
    torch.cuda.synchronize()
    ref = oracle.pq_tables(q, ix.codebooks)
    assert np.array_equal(f32bits(T.cpu().numpy()), f32bits(ref))


# --------------------------------------------------------------------------
# stages 1-3
# --------------------------------------------------------------------------
@pytest.mark.parametrize("name", list(SMALL))
@pytest.mark.parametrize("k,L", [(1, 1), (10, 10), (10, 16), (5, 33),
                                 (10, 64), (10, 100), (32, 256), (10, 300),
                                 (100, 1024)])
def test_search_bit_exact(small_indexes, name, k, L):
    ix, q, gi = small_indexes[name]
    run_and_compare(ix, gi, q, k, L, label=f"{name} k={k} L={L}")


@pytest.mark.parametrize("L", [255, 256, 257, 511, 512, 513, 767, 768, 769])
def test_search_at_super_row_boundaries(small_indexes, L):
    """Worklist sizes on both sides of each super-row boundary (256 entries
    a super-row once L > 256): the merges of one live key and of several
    move entries across super-rows, and the first-level entries of the rank
    are clamped to the last entry; the search stays bit-exact with the
    oracle (3,000 points, so every worklist fills)."""
    ix, q, gi = small_indexes["u8-d128-m32"]
    run_and_compare(ix, gi, q, 10, L, label=f"u8-d128-m32 k=10 L={L}")


@pytest.mark.parametrize("table", ["f16", "u8"])
@pytest.mark.parametrize("name", list(SMALL))
@pytest.mark.parametrize("k,L", [(1, 1), (10, 16), (5, 33), (10, 100),
                                 (32, 256), (10, 600)])
def test_precision_form_bit_exact(small_indexes, name, k, L, table):
    """The precision form's half / u8 tables are derived from the canonical
    FP32 entries on both sides, so the search stays bit-exact."""
    ix, q, gi = small_indexes[name]
    run_and_compare(ix, gi, q, k, L, table=table,
                    label=f"{name} k={k} L={L} {table}")


@pytest.mark.parametrize("name", ["u8-d128-m32", "f32-d32-m16"])
def test_iteration_cap_and_candidate_cap(small_indexes, name):
    """A query stopped by the iteration cap reports status 1; with more
    expanded nodes than c_max only the c_max nearest by PQ key are
    re-ranked.  Both sides apply the same caps."""
    ix, q, gi = small_indexes[name]
    ref = run_and_compare(ix, gi, q, 10, 64, iter_cap=20)
    assert (ref["status"] == 1).all()
    ref = run_and_compare(ix, gi, q, 10, 64, c_max=12)
    assert (ref["iters"] > 12).all()


@pytest.mark.parametrize("name", ["u8-d64-m16", "f32-d32-m16"])
@pytest.mark.parametrize("k,L,c_max", [(10, 64, 0), (10, 64, 12),
                                       (100, 300, 0)])
def test_rerank_in_device_memory_bit_exact(small_indexes, name, k, L, c_max):
    """The re-rank's device-memory selection (taken when the expanded set
    does not fit on chip) returns the same results as the LDS sort."""
    ix, q, gi = small_indexes[name]
    run_and_compare(ix, gi, q, k, L, c_max=c_max, rerank_global=True,
                    label=f"{name} k={k} L={L} c_max={c_max} global")


def test_short_results_are_padded():
    w = synth.small("u8", n=400, d=32, nq=5, m=16, seed_index=114)
    base, q = synth.base_and_queries(w)
    cb = train_pq(base, 16, 3, synth.streams(w)["pq_init"])
    codes = pq_encode(base, cb)
    adj = np.full((w.n, 8), NONE, dtype=np.uint32)
    adj[3, :3] = [10, 20, 30]
    adj[20, 0] = 3
    ix = oracle.Index(base, adj, 3, cb, codes)
    gi = bang_mod().Index(base, adj, 3, cb, codes)
    ref = run_and_compare(ix, gi, q, 10, 16)
    assert (ref["ids"][:, 4:] == NONE).all()


def test_empty_batch_is_a_no_op(small_indexes):
    ix, q, gi = small_indexes["u8-d64-m16"]
    ids, d = gi.search(to_dev(q[:0]), 10, 32)
    torch.cuda.synchronize()
    assert ids.shape == (0, 10)


def test_invalid_arguments_raise(small_indexes):
    bang = bang_mod()
    ix, q, gi = small_indexes["u8-d64-m16"]
    qt = to_dev(q)
    for k, L in [(0, 10), (11, 10), (10, 1025)]:
        with pytest.raises(bang.BangError):
            gi.search(qt, k, L)
    with pytest.raises(TypeError):
        gi.search(qt.float(), 10, 32)
    small = torch.empty((len(q), 5), dtype=torch.int32, device=qt.device)
    d = torch.empty((len(q), 5), dtype=torch.float32, device=qt.device)
    with pytest.raises(ValueError):
        gi.search(qt, 10, 32, out=(small, d))


def test_deterministic_and_independent_of_batch_order(small_indexes):
    """Each query's result depends on that query alone: two runs agree bit
    for bit, and permuting the batch permutes the results."""
    ix, q, gi = small_indexes["u8-d128-m32"]
    qt = to_dev(q)
    a_ids, a_d = gi.search(qt, 10, 64)
    b_ids, b_d = gi.search(qt, 10, 64)
    a_ids, a_d = u32(a_ids), f32bits(a_d.cpu().numpy())
    assert np.array_equal(a_ids, u32(b_ids))
    assert np.array_equal(a_d, f32bits(b_d.cpu().numpy()))
    perm = np.random.default_rng(0).permutation(len(q))
    p_ids, p_d = gi.search(to_dev(q[perm]), 10, 64)
    assert np.array_equal(u32(p_ids), a_ids[perm])
    assert np.array_equal(f32bits(p_d.cpu().numpy()), a_d[perm])
    one_ids, _ = gi.search(to_dev(q[5:6]), 10, 64)
    assert np.array_equal(u32(one_ids)[0], a_ids[5])


# --------------------------------------------------------------------------
# stage 3 alone
# --------------------------------------------------------------------------
@pytest.mark.parametrize("name", list(SMALL))
def test_rerank_bit_exact(small_indexes, name):
    ix, q, gi = small_indexes[name]
    rng = np.random.default_rng(3)
    cm = 77
    cand = np.full((len(q), cm), NONE, dtype=np.uint32)
    for a in range(len(q)):
        c = rng.choice(ix.n, cm - 7, replace=False)
        cand[a, :cm - 7] = c
    cand[1, :] = NONE                      # nothing to rank
    cand[2, 3] = ix.n + 5                  # out of range: skipped
    for k in (1, 10, 80):
        ids, d = gi.rerank(to_dev(q), to_dev(cand.view(np.int32)), k)
        torch.cuda.synchronize()
        rid, rd = oracle.rerank(ix, q, cand, k)
        assert np.array_equal(u32(ids), rid)
        assert np.array_equal(f32bits(d.cpu().numpy()), f32bits(rd))


# --------------------------------------------------------------------------
# the benchmark's workloads
# --------------------------------------------------------------------------
def load_workload(name):
    w = synth.WORKLOADS[name]
    if not store.exists(w):
        from oracle.build_index import build
        build(w)
    d = store.load(w)
    ix = oracle.Index(d["base"], d["adj"], d["medoid"], d["codebooks"],
                      d["codes"])
    return w, ix, d


def test_tiny_workload_bit_exact():
    """10k float32 points, 100 queries, k=10, L=64: every query compared."""
    w, ix, d = load_workload("tiny")
    gi = bang_mod().Index(ix.base, ix.adj, ix.medoid, ix.codebooks, ix.codes)
    for L in w.Ls:
        for table in ("f32", "f16", "u8"):
            run_and_compare(ix, gi, d["queries"], w.k, L, table=table,
                            label=f"tiny L={L} {table}")


def test_sift1m_full_batch_sampled_bit_exact():
    """1M uint8 points: the full 10,000-query batch runs in the launch
    configuration the benchmark times; a seeded sample of queries is
    recomputed one by one by the oracle and compared bit for bit."""
    w, ix, d = load_workload("sift1m")
    gi = bang_mod().Index(ix.base, ix.adj, ix.medoid, ix.codebooks, ix.codes)
    q = d["queries"]
    qt = to_dev(q)
    sample = np.sort(np.random.default_rng(2024).choice(len(q), 160,
                                                        replace=False))
    for L, table in [(L, "f32") for L in w.Ls if L <= 256] + [
            (608, "f32"), (768, "f32"), (64, "f16"), (608, "f16"),
            (768, "f16"), (256, "u8"), (608, "u8"), (768, "u8")]:
        cap = oracle.iter_cap_for(L)
        ids, dist, cand, cnt = gi.search(qt, w.k, L, want_cand=cap,
                                         want_counters=True, table=table)
        torch.cuda.synchronize()
        ref = oracle.search(ix, q[sample], w.k, L, want_cand=True,
                            table=table)
        assert np.array_equal(u32(cnt)[sample, 0], ref["iters"]), L
        assert np.array_equal(u32(cand)[sample], ref["cand"]), L
        assert np.array_equal(u32(ids)[sample], ref["ids"]), L
        assert np.array_equal(f32bits(dist.cpu().numpy()[sample]),
                              f32bits(ref["dists"])), L
        # every query, not only the sample: results sorted, distinct
        allids = u32(ids)
        dd = dist.cpu().numpy()
        assert (np.diff(dd, axis=1) >= 0).all()
        assert all(len(set(r)) == len(r) for r in allids[:500])


@pytest.mark.parametrize("m", [16, 64])
def test_sift1m_other_subspace_counts_sampled_bit_exact(m):
    """The compression-ratio study's encodings (the same base with m = 16 or
    64 subspaces): the full batch on the GPU, a seeded sample of queries
    recomputed by the oracle."""
    w, ix, d = load_workload("sift1m")
    names = store.extra_names(w)
    if f"codes_m{m}" not in names:
        pytest.skip(f"no m={m} encoding beside the index (python -m "
                    f"oracle.build_index sift1m --extra-m {m})")
    ex = store.load_extra(w, [f"codebooks_m{m}", f"codes_m{m}"])
    cb, codes = ex[f"codebooks_m{m}"], ex[f"codes_m{m}"]
    ixm = oracle.Index(d["base"], d["adj"], d["medoid"], cb, codes)
    gi = bang_mod().Index(d["base"], d["adj"], d["medoid"], cb, codes)
    q = d["queries"]
    qt = to_dev(q)
    sample = np.sort(np.random.default_rng(2025 + m).choice(len(q), 96,
                                                            replace=False))
    for L, table in [(64, "f32"), (768, "f32"), (256, "u8")]:
        cap = oracle.iter_cap_for(L)
        ids, dist, cand, cnt = gi.search(qt, w.k, L, want_cand=cap,
                                         want_counters=True, table=table)
        torch.cuda.synchronize()
        ref = oracle.search(ixm, q[sample], w.k, L, want_cand=True,
                            table=table)
        assert np.array_equal(u32(cnt)[sample, 0], ref["iters"]), (m, L)
        assert np.array_equal(u32(cand)[sample], ref["cand"]), (m, L)
        assert np.array_equal(u32(ids)[sample], ref["ids"]), (m, L)
        assert np.array_equal(f32bits(dist.cpu().numpy()[sample]),
                              f32bits(ref["dists"])), (m, L)
    gi.close()


# --------------------------------------------------------------------------
# host-resident adjacency (BANG_INDEX_HOST_ADJ): the same search, adjacency
# rows read across the host link, codes gathered from device memory
# --------------------------------------------------------------------------
@pytest.fixture(scope="module")
def small_host_indexes(small_indexes):
    return {name: bang_mod().Index(ix.base, ix.adj, ix.medoid, ix.codebooks,
                                   ix.codes, host_adj=True)
            for name, (ix, q, _) in small_indexes.items()}


@pytest.mark.parametrize("name", list(SMALL))
@pytest.mark.parametrize("k,L,table", [(1, 1, "f32"), (10, 16, "f32"),
                                       (5, 33, "u8"), (10, 100, "f32"),
                                       (10, 300, "f16"), (100, 1024, "f32")])
def test_host_adjacency_bit_exact(small_indexes, small_host_indexes, name, k,
                                  L, table):
    ix, q, _ = small_indexes[name]
    run_and_compare(ix, small_host_indexes[name], q, k, L, table=table,
                    label=f"host {name} k={k} L={L} {table}")


def test_sift1m_host_adjacency_bit_exact():
    """1M uint8 points with the adjacency in pinned host memory: the full
    batch equals the device-resident run bit for bit, and a seeded sample
    equals the oracle."""
    w, ix, d = load_workload("sift1m")
    bang = bang_mod()
    dev = bang.Index(ix.base, ix.adj, ix.medoid, ix.codebooks, ix.codes)
    host = bang.Index(ix.base, ix.adj, ix.medoid, ix.codebooks, ix.codes,
                      host_adj=True)
    q = d["queries"]
    qt = to_dev(q)
    sample = np.sort(np.random.default_rng(2025).choice(len(q), 96,
                                                        replace=False))
    for L, table in [(64, "f32"), (768, "f32"), (768, "u8")]:
        a_ids, a_d, a_cnt = host.search(qt, w.k, L, want_counters=True,
                                        table=table)
        b_ids, b_d, b_cnt = dev.search(qt, w.k, L, want_counters=True,
                                       table=table)
        torch.cuda.synchronize()
        assert np.array_equal(u32(a_ids), u32(b_ids)), (L, table)
        assert np.array_equal(f32bits(a_d.cpu().numpy()),
                              f32bits(b_d.cpu().numpy())), (L, table)
        assert np.array_equal(u32(a_cnt), u32(b_cnt)), (L, table)
        ref = oracle.search(ix, q[sample], w.k, L, table=table)
        assert np.array_equal(u32(a_ids)[sample], ref["ids"]), (L, table)
        assert np.array_equal(f32bits(a_d.cpu().numpy()[sample]),
                              f32bits(ref["dists"])), (L, table)
    host.close()
    dev.close()


# --------------------------------------------------------------------------
# exact-distance search (BANG_TABLE_EXACT): no table, no re-rank
# --------------------------------------------------------------------------
@pytest.mark.parametrize("name", list(SMALL))
@pytest.mark.parametrize("k,L", [(1, 1), (10, 10), (5, 33), (10, 100),
                                 (32, 256), (100, 1024)])
def test_exact_distance_bit_exact(small_indexes, name, k, L):
    ix, q, gi = small_indexes[name]
    run_and_compare(ix, gi, q, k, L, table="exact",
                    label=f"exact {name} k={k} L={L}")


@pytest.mark.parametrize("name", ["u8-d128-m32", "i8-d96-m48"])
def test_exact_distance_host_adjacency_bit_exact(small_indexes,
                                                 small_host_indexes, name):
    ix, q, _ = small_indexes[name]
    run_and_compare(ix, small_host_indexes[name], q, 10, 64, table="exact",
                    label=f"exact host {name}")


def test_sift1m_exact_distance_sampled_bit_exact():
    """1M uint8 points, exact distances in the search: full batch on the
    GPU, a seeded sample recomputed by the oracle."""
    w, ix, d = load_workload("sift1m")
    gi = bang_mod().Index(ix.base, ix.adj, ix.medoid, ix.codebooks, ix.codes)
    q = d["queries"]
    qt = to_dev(q)
    sample = np.sort(np.random.default_rng(2026).choice(len(q), 128,
                                                        replace=False))
    for L in (16, 64, 256):
        cap = oracle.iter_cap_for(L)
        ids, dist, cand, cnt = gi.search(qt, w.k, L, want_cand=cap,
                                         want_counters=True, table="exact")
        torch.cuda.synchronize()
        ref = oracle.search(ix, q[sample], w.k, L, want_cand=True,
                            table="exact")
        assert np.array_equal(u32(cnt)[sample, 0], ref["iters"]), L
        assert np.array_equal(u32(cand)[sample], ref["cand"]), L
        assert np.array_equal(u32(ids)[sample], ref["ids"]), L
        assert np.array_equal(f32bits(dist.cpu().numpy()[sample]),
                              f32bits(ref["dists"])), L
    gi.close()


def test_seen_cache_changes_no_result():
    """The exact-distance search's seen-id cache (on by default) only skips
    base rows of neighbours the set union would drop: ids, distances,
    expansion order and iteration counts equal those of the search without
    it, on the 1M index at the bench's worklist sizes, and with one wave
    per CU (the largest cache, 4,096 ids)."""
    w, ix, d = load_workload("sift1m")
    gi = bang_mod().Index(ix.base, ix.adj, ix.medoid, ix.codebooks, ix.codes)
    qt = to_dev(d["queries"][:2000])
    for L, wpc in ((64, 0), (256, 0), (608, 0), (1024, 0), (256, 1)):
        cap = oracle.iter_cap_for(L)
        got = []
        for cache in (True, False):
            ids, dist, cand, cnt = gi.search(
                qt, w.k, L, want_cand=cap, want_counters=True, table="exact",
                seen_cache=cache, waves_per_cu=wpc)
            torch.cuda.synchronize()
            got.append((u32(ids), f32bits(dist.cpu().numpy()), u32(cand),
                        u32(cnt)))
        for a, b in zip(*got):
            assert np.array_equal(a, b), (L, wpc)
    gi.close()


# --------------------------------------------------------------------------
# mixed batches (per-query k and L) and the serving loop: every result is
# the one the query gets alone
# --------------------------------------------------------------------------
def _alone(gi, q, k, L, table):
    ids, d = gi.search(to_dev(q), k, L, table=table)
    torch.cuda.synchronize()
    return u32(ids), d.cpu().numpy()


@pytest.mark.parametrize("name", ["u8-d128-m32", "f32-d32-m16", "i8-d96-m48"])
@pytest.mark.parametrize("table", ["f32", "u8", "exact"])
def test_mixed_batch_equals_each_query_alone(small_indexes, name, table):
    ix, q, gi = small_indexes[name]
    rng = np.random.default_rng(7)
    nq = len(q)
    Ls = rng.choice([1, 10, 33, 100, 256], nq).astype(np.int32)
    ks = np.array([rng.integers(1, min(32, L) + 1) for L in Ls], np.int32)
    kmax, Lmax = int(ks.max()), int(Ls.max())
    ids, d = gi.search(to_dev(q), kmax, Lmax, table=table,
                       query_L=to_dev(Ls), query_k=to_dev(ks))
    torch.cuda.synchronize()
    ids, d = u32(ids), d.cpu().numpy()
    for (k, L) in sorted(set(zip(ks.tolist(), Ls.tolist()))):
        sel = np.where((ks == k) & (Ls == L))[0]
        a_ids, a_d = _alone(gi, q[sel], k, L, table)
        assert np.array_equal(ids[sel, :k], a_ids), (k, L)
        assert np.array_equal(f32bits(d[sel, :k]), f32bits(a_d)), (k, L)
        assert (ids[sel, k:] == NONE).all() and np.isinf(d[sel, k:]).all()
        ref = oracle.search(ix, q[sel], k, L, table=table)
        assert np.array_equal(a_ids, ref["ids"]), (k, L)


@pytest.mark.parametrize("graphs", [False, True])
def test_server_replay_results_equal_alone(small_indexes, graphs):
    """Requests with mixed sizes, k and L arrive open-loop (Poisson) and
    overlap on the device in two slots; each result equals a search of its
    queries alone, also when the slots replay captured HIP graphs (batches
    rounded up to a power of two, several (k, L) combinations, each graph
    replayed many times)."""
    ix, q, gi = small_indexes["u8-d128-m32"]
    bang = bang_mod()
    rng = np.random.default_rng(11)
    nreq = 60
    nq = rng.integers(1, 9, nreq).astype(np.uint32)
    k = rng.choice([1, 5, 10, 32], nreq).astype(np.uint32)
    L = np.maximum(k, rng.choice([16, 33, 64, 128], nreq)).astype(np.uint32)
    rows = rng.integers(0, len(q), int(nq.sum()))
    Q = q[rows]
    arr = np.cumsum(rng.exponential(2e-4, nreq))
    sv = bang.Server(gi, max_batch=24, slots=2, max_k=32, max_L=128,
                     graphs=graphs)
    ids, d, lat = sv.replay(Q, nq, k, L, arr, kstride=32)
    st = sv.stats()
    sv.close()
    assert st["requests"] == nreq and st["queries"] == int(nq.sum())
    assert (lat >= 0).all()
    off = 0
    for j in range(nreq):
        sl = slice(off, off + int(nq[j]))
        a_ids, a_d = _alone(gi, Q[sl], int(k[j]), int(L[j]), "f32")
        assert np.array_equal(ids[sl, :k[j]], a_ids), j
        assert np.array_equal(f32bits(d[sl, :k[j]]), f32bits(a_d)), j
        assert (ids[sl, k[j]:] == NONE).all()
        off += int(nq[j])


def test_server_threads_submit_and_wait(small_indexes):
    """Several host threads submit and wait at once; every ticket returns
    its own request's results."""
    import threading
    ix, q, gi = small_indexes["f32-d32-m16"]
    bang = bang_mod()
    sv = bang.Server(gi, max_batch=16, slots=3, max_k=10, max_L=64,
                     table="exact")
    errors = []

    def worker(seed):
        r = np.random.default_rng(seed)
        try:
            for _ in range(15):
                n = int(r.integers(1, 6))
                sel = r.integers(0, len(q), n)
                kk, LL = int(r.choice([1, 10])), int(r.choice([10, 33, 64]))
                t = sv.submit(q[sel], kk, LL)
                got_ids, got_d = sv.wait(t)
                a_ids, a_d = _alone(gi, q[sel], kk, LL, "exact")
                if not (np.array_equal(got_ids, a_ids)
                        and np.array_equal(f32bits(got_d), f32bits(a_d))):
                    errors.append((seed, n, kk, LL))
        except Exception as ex:  # surfaced below
            errors.append(repr(ex))

    th = [threading.Thread(target=worker, args=(s,)) for s in range(4)]
    for t in th:
        t.start()
    for t in th:
        t.join()
    sv.close()
    assert not errors, errors


def test_deep1m_sampled_bit_exact():
    """1M float32 points, d=96, m=48 (a 48 KB FP32 table): every table form
    and the exact-distance search on the full batch; a seeded sample is
    recomputed by the oracle and compared bit for bit."""
    w, ix, d = load_workload("deep1m")
    gi = bang_mod().Index(ix.base, ix.adj, ix.medoid, ix.codebooks, ix.codes,
                          bf16_base=True)
    q = d["queries"]
    qt = to_dev(q)
    sample = np.sort(np.random.default_rng(2027).choice(len(q), 96,
                                                        replace=False))
    for L, table, rr in [(128, "f32", "exact"), (256, "f32", "exact"),
                         (256, "f16", "exact"), (256, "u8", "exact"),
                         (128, "exact", "exact"), (512, "f32", "exact"),
                         (128, "f32", "bf16"), (256, "u8", "bf16")]:
        cap = oracle.iter_cap_for(L)
        ids, dist, cand, cnt = gi.search(qt, w.k, L, want_cand=cap,
                                         want_counters=True, table=table,
                                         rerank=rr)
        torch.cuda.synchronize()
        ref = oracle.search(ix, q[sample], w.k, L, want_cand=True,
                            table=table)
        assert np.array_equal(u32(cnt)[sample, 0], ref["iters"]), (L, table)
        assert np.array_equal(u32(cand)[sample], ref["cand"]), (L, table)
        assert np.array_equal(u32(ids)[sample], ref["ids"]), (L, table, rr)
        assert np.array_equal(f32bits(dist.cpu().numpy()[sample]),
                              f32bits(ref["dists"])), (L, table, rr)
    gi.close()


def test_server_rejects_bad_requests_and_times_out_cleanly(small_indexes):
    """Validation happens at submit; an unknown ticket and a wait that
    times out are errors that leave the server usable."""
    ix, q, gi = small_indexes["u8-d128-m32"]
    bang = bang_mod()
    with pytest.raises(bang.BangError):
        bang.Server(gi, max_batch=0)
    with pytest.raises(bang.BangError):
        bang.Server(gi, max_k=64, max_L=32)
    sv = bang.Server(gi, max_batch=8, slots=1, max_k=10, max_L=64)
    for args in ((q[:9], 10, 64),      # more queries than max_batch
                 (q[:2], 11, 64),      # k above max_k
                 (q[:2], 10, 65),      # L above max_L
                 (q[:2], 20, 16)):     # k above L
        with pytest.raises(bang.BangError) as e:
            sv.submit(*args)
        assert e.value.code == -1
    with pytest.raises(bang.BangError):
        sv.wait(12345)                 # unknown ticket (binding)
    with pytest.raises(bang.BangError):
        sv._shapes[12345] = (1, 1)
        sv.wait(12345)                 # unknown ticket (library)
    sv._shapes.pop(12345)
    t = sv.submit(q[:3], 5, 32)
    ids, d = sv.wait(t)
    a_ids, a_d = _alone(gi, q[:3], 5, 32, "f32")
    assert np.array_equal(ids, a_ids)
    assert np.array_equal(f32bits(d), f32bits(a_d))
    sv.close()


def test_mixed_batch_rejects_explicit_caps(small_indexes):
    ix, q, gi = small_indexes["u8-d64-m16"]
    bang = bang_mod()
    Ls = to_dev(np.full(len(q), 16, np.int32))
    with pytest.raises(bang.BangError):
        gi.search(to_dev(q), 10, 16, c_max=8, query_L=Ls)
    with pytest.raises(ValueError):
        gi.search(to_dev(q), 10, 16, query_L=Ls[:3])


@pytest.mark.parametrize("dtype,d,m", [("u8", 32, 16), ("i8", 32, 16),
                                       ("u8", 64, 32), ("i8", 128, 64)])
def test_exact_distance_integer_row_widths_bit_exact(dtype, d, m):
    """The integer exact distances read each base row with 2, 4 or 8 lanes
    (d = 32, 64, 128 bytes); every width against the oracle."""
    w = synth.small(dtype, n=1500, d=d, nq=40, m=m, R=32,
                    seed_index=130 + d + (dtype == "i8"))
    ix, q = make_index(w)
    gi = bang_mod().Index(ix.base, ix.adj, ix.medoid, ix.codebooks, ix.codes)
    for k, L in ((1, 1), (10, 33), (10, 200)):
        run_and_compare(ix, gi, q, k, L, table="exact",
                        label=f"exact {dtype} d={d} k={k} L={L}")
    gi.close()


@pytest.mark.parametrize("table", ["f32", "u8", "exact"])
def test_ties_are_broken_by_id(table):
    """Every base vector appears four times (ids 4i..4i+3), so PQ and exact
    distances tie in groups: orders (worklist, re-rank, results) must fall
    back to the node id exactly as the oracle's do."""
    w = synth.small("u8", n=1200, d=64, nq=30, m=16, R=24, seed_index=140)
    base0, q = synth.base_and_queries(w)
    base = np.repeat(base0[:300], 4, axis=0)
    rs = synth.streams(w)
    cb = train_pq(base, w.m, 4, rs["pq_init"])
    codes = pq_encode(base, cb)
    s = oracle.medoid(base)
    perm = rs["vamana_order"].permutation(len(base)).astype(np.uint32)
    adj, _ = build_graph(base, w.R, w.L_build, w.alpha, perm, s)
    ix = oracle.Index(base, adj, s, cb, codes)
    gi = bang_mod().Index(base, adj, s, cb, codes)
    ref = run_and_compare(ix, gi, q, 10, 48, table=table,
                          label=f"ties {table}")
    # tied neighbours come out in id order
    for ids, d in zip(ref["ids"], ref["dists"]):
        for a, b, da, db in zip(ids[:-1], ids[1:], d[:-1], d[1:]):
            if da == db:
                assert a < b
    gi.close()


def test_single_node_and_isolated_start():
    """n = 1, and a start node without edges: one expansion, the start
    node alone in the result, the rest padded."""
    w = synth.small("f32", n=300, d=32, nq=4, m=16, seed_index=141)
    base, q = synth.base_and_queries(w)
    cb = train_pq(base, 16, 3, synth.streams(w)["pq_init"])
    codes = pq_encode(base, cb)
    for n in (1, 64):
        adj = np.full((n, 8), NONE, dtype=np.uint32)
        ix = oracle.Index(base[:n], adj, 0, cb, codes[:n])
        gi = bang_mod().Index(base[:n], adj, 0, cb, codes[:n])
        for table in ("f32", "exact"):
            ref = run_and_compare(ix, gi, q, 1 if n == 1 else 5, 8,
                                  table=table, label=f"n={n} {table}")
            assert (ref["iters"] == 1).all()
            assert (ref["ids"][:, 0] == 0).all()
        gi.close()


def test_search_replays_from_a_hip_graph(small_indexes):
    """bang_search is stream-ordered with no allocation (once the workspace
    has grown) and no memset (the kernel returns its counters to zero), so
    a captured search replays: every replay, with new queries copied into
    the captured input and eager searches in between, equals the eager
    result of those queries."""
    ix, q, gi = small_indexes["u8-d128-m32"]
    k, L = 10, 64
    n = len(q) // 2
    qa, qb = to_dev(q[:n]), to_dev(q[n:2 * n])
    qbuf = qa.clone()
    ids = torch.empty((n, k), dtype=torch.int32, device=qa.device)
    dist = torch.empty((n, k), dtype=torch.float32, device=qa.device)
    gi.search(qbuf, k, L, out=(ids, dist))          # grows the workspace
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        with torch.cuda.graph(g, stream=s, capture_error_mode="relaxed"):
            gi.search(qbuf, k, L, out=(ids, dist), stream=s)
    torch.cuda.synchronize()
    for rep, src in enumerate((qa, qb, qa, qb)):
        qbuf.copy_(src)
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        got_ids, got_d = u32(ids).copy(), dist.cpu().numpy().copy()
        e_ids, e_d = gi.search(src, k, L)           # eager, between replays
        torch.cuda.synchronize()
        assert np.array_equal(got_ids, u32(e_ids)), rep
        assert np.array_equal(f32bits(got_d), f32bits(e_d.cpu().numpy())), rep


def test_server_admission_by_memory_budget(small_indexes):
    """hbm_budget_bytes caps the slots: a budget for one slot gives one
    slot (and correct results), a budget below one slot is refused."""
    ix, q, gi = small_indexes["u8-d64-m16"]
    bang = bang_mod()
    with pytest.raises(bang.BangError) as e:
        bang.Server(gi, max_batch=64, slots=4, max_k=10, max_L=64,
                    hbm_budget_bytes=1024)
    assert e.value.code == -2
    big = bang.Server(gi, max_batch=64, slots=4, max_k=10, max_L=64)
    assert big.stats()["slots"] == 4
    big.close()
    # grow the budget until two slots fit: the first budget that allows
    # more than one slot lies between one and two slots' footprint
    one = None
    for mb in (1, 2, 4, 8, 16, 32, 64, 128, 256):
        try:
            sv = bang.Server(gi, max_batch=64, slots=4, max_k=10, max_L=64,
                             hbm_budget_bytes=mb << 20)
        except bang.BangError:
            continue
        n = sv.stats()["slots"]
        if one is None:
            one = (mb, n)
            t = sv.submit(q[:5], 10, 64)
            ids, d = sv.wait(t)
            a_ids, _ = _alone(gi, q[:5], 10, 64, "f32")
            assert np.array_equal(ids, a_ids)
        sv.close()
        if n == 4:
            break
    assert one is not None and 1 <= one[1] <= 4


# --------------------------------------------------------------------------
# the paper's Bloom filter (BANG_FILTER_BLOOM) against the oracle's
# Algorithm 2 with the same filter (search mode 2)
# --------------------------------------------------------------------------
@pytest.mark.parametrize("name", list(SMALL))
@pytest.mark.parametrize("k,L,table", [(1, 1, "f32"), (10, 16, "f32"),
                                       (5, 33, "u8"), (10, 100, "f16"),
                                       (10, 64, "exact"),
                                       (100, 1024, "f32")])
def test_bloom_filter_bit_exact(small_indexes, name, k, L, table):
    ix, q, gi = small_indexes[name]
    run_and_compare(ix, gi, q, k, L, table=table, filter="bloom",
                    label=f"bloom {name} k={k} L={L} {table}")


@pytest.mark.parametrize("name", ["u8-d64-m16", "f32-d128-m16"])
def test_bloom_filter_host_adjacency_bit_exact(small_indexes,
                                               small_host_indexes, name):
    ix, q, _ = small_indexes[name]
    for k, L, table in [(10, 33, "f32"), (10, 64, "exact")]:
        run_and_compare(ix, small_host_indexes[name], q, k, L, table=table,
                        filter="bloom",
                        label=f"bloom host {name} k={k} L={L} {table}")


def test_bloom_filter_repeated_launches_stay_exact(small_indexes):
    """Every wave keeps its filter entries across queries and launches
    (tags carry a per-wave query epoch; the entries are cleared when the
    epochs run out, after 4,095 queries per wave): 260 launches of 20,000
    queries take every wave past that point, and results stay equal to
    the oracle's."""
    ix, q, gi = small_indexes["u8-d128-m32"]
    reps = -(-20000 // len(q))
    qq = np.ascontiguousarray(np.tile(q, (reps, 1))[:20000])
    qt = to_dev(qq)
    ref = oracle.search(ix, q, 10, 24, mode=oracle.MODES["bloom"])
    for it in range(260):
        ids, dist = gi.search(qt, 10, 24, filter="bloom")
        if it % 65 == 64 or it == 0:
            torch.cuda.synchronize()
            got = u32(ids)
            for r in range(0, 20000, len(q)):
                n = min(len(q), 20000 - r)
                assert np.array_equal(got[r:r + n], ref["ids"][:n]), (it, r)
                assert np.array_equal(f32bits(dist.cpu().numpy()[r:r + n]),
                                      f32bits(ref["dists"][:n])), (it, r)


def _collision_index(row):
    """Medoid s = 12446 whose only neighbours are `row`; node 11616's first
    filter entry is one of s's and its second one of node 12330's."""
    s = 12446
    n, d = s + 1, 32
    rng = np.random.default_rng(5)
    base = rng.random((n, d), dtype=np.float32)
    adj = np.full((n, 2), 0xFFFFFFFF, dtype=np.uint32)
    adj[s, :len(row)] = row
    cb = rng.random((16, 256, 2), dtype=np.float32)
    codes = rng.integers(0, 256, (n, 16), dtype=np.uint8)
    return (oracle.Index(base, adj, s, cb, codes),
            bang_mod().Index(base, adj, s, cb, codes), base[:3].copy())


@pytest.mark.parametrize("row,dropped", [([12330, 11616], True),
                                         ([11616, 12330], False)])
def test_bloom_filter_false_positive_follows_row_order(row, dropped):
    """Row [a, y] under s: y's entries were set by s and then by a, so y
    counts as visited and is never expanded (a false positive); row
    [y, a]: y is tested before a sets its entry and is kept.  The exact
    filter keeps y either way."""
    ix, gi, q = _collision_index(row)
    for flt in ("bloom", "exact"):
        ids, dist, cand, cnt = gi.search(to_dev(q), 1, 8, want_cand=8,
                                         want_counters=True, filter=flt)
        torch.cuda.synchronize()
        c, it = u32(cand), u32(cnt)[:, 0]
        for i in range(len(q)):
            got = set(c[i, :it[i]].tolist())
            if flt == "bloom" and dropped:
                assert got == {12446, 12330}
            else:
                assert got == {12446, 12330, 11616}
        run_and_compare(ix, gi, q, 1, 8, filter=flt,
                        label=f"collision {row} {flt}")
    gi.close()


def test_sift1m_bloom_filter_sampled_bit_exact():
    """The full 10,000-query batch with the Bloom filter at the benchmark
    point; a seeded sample recomputed by the oracle's Algorithm 2 with the
    same filter."""
    w, ix, d = load_workload("sift1m")
    gi = bang_mod().Index(ix.base, ix.adj, ix.medoid, ix.codebooks, ix.codes)
    q = d["queries"]
    qt = to_dev(q)
    sample = np.sort(np.random.default_rng(2026).choice(len(q), 64,
                                                        replace=False))
    for L, table in [(64, "f32"), (768, "f32"), (256, "exact")]:
        cap = oracle.iter_cap_for(L)
        ids, dist, cand, cnt = gi.search(qt, w.k, L, want_cand=cap,
                                         want_counters=True, table=table,
                                         filter="bloom")
        torch.cuda.synchronize()
        ref = oracle.search(ix, q[sample], w.k, L, want_cand=True,
                            table=table, mode=oracle.MODES["bloom"])
        assert np.array_equal(u32(cnt)[sample, 0], ref["iters"]), L
        assert np.array_equal(u32(cand)[sample], ref["cand"]), L
        assert np.array_equal(u32(ids)[sample], ref["ids"]), L
        assert np.array_equal(f32bits(dist.cpu().numpy()[sample]),
                              f32bits(ref["dists"])), L
    gi.close()


# --------------------------------------------------------------------------
# roofline probe (bang_index_probe)
# --------------------------------------------------------------------------
def test_index_probe_reads_rows(small_indexes, small_host_indexes):
    """The probe runs on both adjacency placements, reports the bytes the
    search reads per row, accepts nreads = 0 and rejects a null sink."""
    import ctypes
    bang = bang_mod()
    ix, q, gi = small_indexes["u8-d128-m32"]
    hi = small_host_indexes["u8-d64-m16"]
    assert gi.probe(0) == (ix.R * 4 + 15) // 16 * 16 + ix.R * ix.m
    assert gi.probe(100_000, seed=3) == (ix.R * 4 + 15) // 16 * 16 + \
        ix.R * ix.m
    assert hi.probe(50_000) == 4 * small_indexes["u8-d64-m16"][0].R
    torch.cuda.synchronize()
    rb = ctypes.c_uint32(0)
    rc = bang.lib().bang_index_probe(gi._h, 10, 0, None, ctypes.byref(rb),
                                     None)
    assert rc == -1


@pytest.mark.parametrize("name", ["u8-d128-m32", "f32-d128-m16"])
def test_bloom_filter_mixed_batch_equals_oracle(small_indexes, name):
    """A mixed batch (per-query k and L) with the Bloom filter: every query
    equals the oracle's Algorithm 2 with the same filter at its own (k, L),
    whatever wave and filter epoch it ran in."""
    ix, q, gi = small_indexes[name]
    rng = np.random.default_rng(8)
    nq = len(q)
    Ls = rng.choice([1, 12, 40, 128], nq).astype(np.int32)
    ks = np.array([rng.integers(1, min(16, L) + 1) for L in Ls], np.int32)
    kmax, Lmax = int(ks.max()), int(Ls.max())
    ids, d = gi.search(to_dev(q), kmax, Lmax, filter="bloom",
                       query_L=to_dev(Ls), query_k=to_dev(ks))
    torch.cuda.synchronize()
    ids, d = u32(ids), d.cpu().numpy()
    for (k, L) in sorted(set(zip(ks.tolist(), Ls.tolist()))):
        sel = np.where((ks == k) & (Ls == L))[0]
        ref = oracle.search(ix, q[sel], k, L, mode=oracle.MODES["bloom"])
        assert np.array_equal(ids[sel, :k], ref["ids"]), (k, L)
        assert np.array_equal(f32bits(d[sel, :k]), f32bits(ref["dists"])), \
            (k, L)


# --------------------------------------------------------------------------
# the timed copy of the search (bang_search_opts.out_phases)
# --------------------------------------------------------------------------
@pytest.mark.parametrize("table", ["f32", "u8", "exact"])
def test_timed_search_same_results_and_phases(small_indexes, table):
    """The timed search returns the same results bit for bit; every query
    has positive table, scoring and re-rank times (no re-rank for exact
    distances), and the loop phases are zero exactly when nothing was
    expanded."""
    ix, q, gi = small_indexes["u8-d128-m32"]
    qt = to_dev(q)
    ids0, d0 = gi.search(qt, 10, 64, table=table)
    ids1, d1, cnt, ph = gi.search(qt, 10, 64, table=table,
                                  want_counters=True, want_phases=True)
    torch.cuda.synchronize()
    assert np.array_equal(u32(ids0), u32(ids1))
    assert np.array_equal(f32bits(d0.cpu().numpy()), f32bits(d1.cpu().numpy()))
    p = u32(ph).astype(np.int64)
    it = u32(cnt)[:, 0]
    assert (it > 0).all()
    assert (p[:, 0] > 0).all() and (p[:, 2] > 0).all() and (p[:, 3] > 0).all()
    assert (p[:, 6] > 0).all()
    # the loop's phases sum to most of a query's cycles at this L
    assert (p[:, 1:6].sum(1) > p[:, 0]).all()


def test_timed_search_refused_with_host_rows_or_bloom(small_indexes,
                                                     small_host_indexes):
    ix, q, gi = small_indexes["u8-d64-m16"]
    hi = small_host_indexes["u8-d64-m16"]
    bang = bang_mod()
    with pytest.raises(bang.BangError):
        hi.search(to_dev(q), 10, 32, want_phases=True)
    with pytest.raises(bang.BangError):
        gi.search(to_dev(q), 10, 32, want_phases=True, filter="bloom")


@pytest.mark.parametrize("name", ["u8-d64-m16", "f32-d128-m16"])
def test_bloom_filter_equals_exact_filter_without_collisions(small_indexes,
                                                            name):
    """Where no node's two filter entries are both shared with other nodes
    no neighbour can be a false positive, so the Bloom-filter search equals
    the default set-union search bit for bit (no false negatives either)."""
    from collections import Counter
    ix, q, gi = small_indexes[name]
    sl = [oracle.bloom_slots(x) for x in range(ix.n)]
    cnt = Counter(h for s in sl for h in set(s))
    assert not [x for x, s in enumerate(sl) if all(cnt[h] > 1 for h in set(s))]
    qt = to_dev(q)
    for k, L, table in [(10, 33, "f32"), (10, 100, "u8"), (5, 64, "exact")]:
        a = gi.search(qt, k, L, table=table, want_cand=oracle.iter_cap_for(L))
        b = gi.search(qt, k, L, table=table, filter="bloom",
                      want_cand=oracle.iter_cap_for(L))
        torch.cuda.synchronize()
        for x, y in zip(a, b):
            assert np.array_equal(x.cpu().numpy(), y.cpu().numpy()), (k, L)


# --------------------------------------------------------------------------
# stop requests and bounded waits
# --------------------------------------------------------------------------
def test_stop_request_set_before_the_launch_pads_every_query(small_indexes):
    """A search carrying a stop request that is already set searches
    nothing: every row is padding with status 2, the request reports that
    it stopped the search, and once cleared the same index searches
    normally (the persistent launch left its counters at zero)."""
    ix, q, gi = small_indexes["u8-d128-m32"]
    bang = bang_mod()
    ab = bang.StopRequest()
    assert not ab.stopped()
    ab.set()
    ids, d, cand, cnt = gi.search(to_dev(q), 10, 64, want_cand=8,
                                  want_counters=True, abort=ab)
    torch.cuda.synchronize()
    assert (u32(ids) == NONE).all() and np.isinf(d.cpu().numpy()).all()
    assert (u32(cand) == NONE).all()
    c = u32(cnt)
    assert (c[:, 0] == 0).all() and (c[:, 1] == 2).all()
    assert ab.stopped()
    ab.clear()
    assert not ab.stopped()
    run_and_compare(ix, gi, q, 10, 64, label="after a stopped launch")
    ab.close()


def test_stop_request_ends_a_long_launch_early(small_indexes):
    """Set from the host while a long persistent launch runs: the launch
    ends early, every query is either finished (status 0, the result of a
    search without the request) or stopped (status 2, padding), and the
    index searches normally afterwards."""
    import time
    ix, q, gi = small_indexes["u8-d128-m32"]
    bang = bang_mod()
    k, L, reps = 10, 1024, 1500
    qrep = to_dev(np.tile(q, (reps, 1)))
    nq = qrep.shape[0]
    ref_ids, ref_d = _alone(gi, q, k, L, "f32")
    ab = bang.StopRequest()
    ids, d, cnt = gi.search(qrep, k, L, want_counters=True, abort=ab)
    torch.cuda.synchronize()          # warm: the workspace has grown
    t0 = time.perf_counter()
    gi.search(qrep, k, L, want_counters=True, abort=ab, out=(ids, d))
    torch.cuda.synchronize()
    full = time.perf_counter() - t0
    assert not ab.stopped()
    assert (u32(cnt)[:, 1] == 0).all()
    print(f"full launch: {nq} queries in {full * 1e3:.1f} ms", flush=True)
    t0 = time.perf_counter()
    _, _, cnt = gi.search(qrep, k, L, want_counters=True, abort=ab,
                          out=(ids, d))
    time.sleep(full * 0.2)
    ab.set()
    torch.cuda.synchronize()
    cut = time.perf_counter() - t0
    st = u32(cnt)[:, 1]
    got_ids, got_d = u32(ids), d.cpu().numpy()
    print(f"stopped launch: {cut * 1e3:.1f} ms, {int((st == 0).sum())} "
          f"finished, {int((st == 2).sum())} stopped", flush=True)
    assert set(np.unique(st).tolist()) <= {0, 2}
    assert (st == 2).any() and ab.stopped()
    assert cut < 0.8 * full
    fin = np.where(st == 0)[0]
    assert np.array_equal(got_ids[fin], ref_ids[fin % len(q)])
    assert np.array_equal(f32bits(got_d[fin]), f32bits(ref_d[fin % len(q)]))
    stop = np.where(st == 2)[0]
    assert (got_ids[stop] == NONE).all() and np.isinf(got_d[stop]).all()
    ab.clear()
    run_and_compare(ix, gi, q, 10, 64, label="after an interrupted launch")
    ab.close()


def test_server_wait_with_zero_timeout_keeps_the_ticket(small_indexes):
    """A wait that times out (timeout_ms = 0 on a request still queued
    behind a long one on the only slot) returns EABORTED and leaves the
    ticket valid: a later wait collects the request's results."""
    ix, q, gi = small_indexes["u8-d128-m32"]
    bang = bang_mod()
    big = np.tile(q, (200, 1))
    sv = bang.Server(gi, max_batch=len(big), slots=1, max_k=10, max_L=1024)
    t1 = sv.submit(big, 10, 1024)
    t2 = sv.submit(q[:5], 10, 64)
    with pytest.raises(bang.BangError) as e:
        sv.wait(t2, timeout_ms=0)
    assert e.value.code == -5
    ids2, d2 = sv.wait(t2)
    a_ids, a_d = _alone(gi, q[:5], 10, 64, "f32")
    assert np.array_equal(ids2, a_ids)
    assert np.array_equal(f32bits(d2), f32bits(a_d))
    ids1, _ = sv.wait(t1, timeout_ms=60000)
    b_ids, _ = _alone(gi, q, 10, 1024, "f32")
    assert np.array_equal(ids1, np.tile(b_ids, (200, 1)))
    sv.close()


def test_server_many_tickets_and_concurrent_waits(small_indexes):
    """Threads hold many tickets at once (the server's ticket table grows
    while others wait on it), and two threads waiting on one ticket: one
    collects it, the other is told it was already collected."""
    import threading
    ix, q, gi = small_indexes["u8-d64-m16"]
    bang = bang_mod()
    sv = bang.Server(gi, max_batch=32, slots=2, max_k=10, max_L=64)
    ref_ids, _ = _alone(gi, q, 10, 64, "f32")
    errors = []

    def worker(seed):
        r = np.random.default_rng(seed)
        try:
            pend = []
            for _ in range(40):
                sel = r.integers(0, len(q), int(r.integers(1, 4)))
                pend.append((sv.submit(q[sel], 10, 64), sel))
            for t, sel in reversed(pend):
                got, _ = sv.wait(t)
                if not np.array_equal(got, ref_ids[sel]):
                    errors.append((seed, t))
        except Exception as ex:  # surfaced below
            errors.append(repr(ex))

    th = [threading.Thread(target=worker, args=(s,)) for s in range(6)]
    for t in th:
        t.start()
    for t in th:
        t.join()
    assert not errors, errors
    t = sv.submit(q[:3], 10, 64)
    outcome = []

    def waiter():
        try:
            outcome.append(("ok", sv.wait(t)[0]))
        except bang.BangError as ex:
            outcome.append(("err", ex.code))

    ws = [threading.Thread(target=waiter) for _ in range(2)]
    for w in ws:
        w.start()
    for w in ws:
        w.join()
    kinds = sorted(o[0] for o in outcome)
    assert kinds == ["err", "ok"], outcome
    assert [o[1] for o in outcome if o[0] == "err"] == [-1]
    got = [o[1] for o in outcome if o[0] == "ok"][0]
    assert np.array_equal(got, ref_ids[:3])
    sv.close()


# --------------------------------------------------------------------------
# the precision form's re-rank of float data: bfloat16 rows, FP32 recheck
# --------------------------------------------------------------------------
@pytest.fixture(scope="module")
def bf16_indexes(small_indexes):
    out = {}
    for name in ("f32-d32-m16", "f32-d128-m16"):
        ix, q, _ = small_indexes[name]
        out[name] = (ix, q, bang_mod().Index(ix.base, ix.adj, ix.medoid,
                                             ix.codebooks, ix.codes,
                                             bf16_base=True))
    return out


@pytest.mark.parametrize("name", ["f32-d32-m16", "f32-d128-m16"])
@pytest.mark.parametrize("k,L,c_max,table", [(10, 64, 0, "f32"),
                                             (1, 16, 0, "u8"),
                                             (10, 128, 20, "f16"),
                                             (100, 256, 0, "f32")])
def test_bf16_rerank_equals_the_fp32_rerank(bf16_indexes, name, k, L, c_max,
                                            table):
    """The search with the BF16 re-rank returns the oracle's FP32 answer bit
    for bit (ids, distances, expanded nodes, iterations), including the
    c_max cut and k above 64 (the sorted path); fewer candidates than were
    expanded get an FP32 distance."""
    ix, q, gi = bf16_indexes[name]
    run_and_compare(ix, gi, q, k, L, c_max=c_max, table=table, rerank="bf16",
                    label=f"{name} k={k} L={L} bf16")
    _, _, cnt = gi.search(to_dev(q), k, L, c_max=c_max, table=table,
                          want_counters=True, rerank="bf16")
    torch.cuda.synchronize()
    c = u32(cnt)
    nc = np.minimum(c[:, 0], c_max or 4 * L)
    assert (c[:, 2] <= nc).all()
    assert (c[:, 2] >= np.minimum(nc, k)).all()
    if k == 10 and L >= 64:
        assert c[:, 2].sum() < nc.sum()


def test_bf16_rerank_global_fallback_equals_fp32(bf16_indexes):
    ix, q, gi = bf16_indexes["f32-d32-m16"]
    run_and_compare(ix, gi, q, 10, 64, rerank="bf16", rerank_global=True,
                    label="bf16 global fallback")


def test_bf16_rerank_near_ties():
    """Rows that differ from each other by less than a bfloat16 step, so
    that the BF16 sums alone misorder them: on a graph where every node is
    expanded (L >= n), the answer still equals the oracle's FP32 re-rank."""
    rng = np.random.default_rng(31)
    n, d, m, R = 300, 32, 16, 24
    base = rng.standard_normal((n, d)).astype(np.float32)
    q = rng.standard_normal((8, d)).astype(np.float32)
    anchor = q[0] + np.float32(0.2) * rng.standard_normal(d).astype(np.float32)
    base[:60] = anchor + (rng.standard_normal((60, d)) * 1e-4).astype(
        np.float32)
    w = synth.small("f32", n=n, d=d, nq=8, m=m, R=R, seed_index=131)
    rs = synth.streams(w)
    cb = train_pq(base, m, 4, rs["pq_init"])
    codes = pq_encode(base, cb)
    s = oracle.medoid(base)
    perm = rs["vamana_order"].permutation(n).astype(np.uint32)
    adj, _ = build_graph(base, R, 32, 1.2, perm, s)
    ix = oracle.Index(base, adj, s, cb, codes)
    gi = bang_mod().Index(base, adj, s, cb, codes, bf16_base=True)
    run_and_compare(ix, gi, q, 10, 512, rerank="bf16", label="near ties")
    gi.close()


def test_bf16_rerank_is_refused_where_it_does_not_apply(small_indexes,
                                                       bf16_indexes):
    bang = bang_mod()
    _, q, gi = small_indexes["f32-d32-m16"]
    with pytest.raises(bang.BangError) as e:
        gi.search(to_dev(q), 10, 64, rerank="bf16")   # no bfloat16 base
    assert e.value.code == -1
    _, q, gb = bf16_indexes["f32-d32-m16"]
    with pytest.raises(bang.BangError) as e:
        gb.search(to_dev(q), 10, 64, rerank="bf16", table="exact")
    assert e.value.code == -1
    ix, _, _ = small_indexes["u8-d64-m16"]
    with pytest.raises(bang.BangError) as e:
        bang.Index(ix.base, ix.adj, ix.medoid, ix.codebooks, ix.codes,
                   bf16_base=True)
    assert e.value.code == -4


# --------------------------------------------------------------------------
# the exact seen bitmap (BANG_FILTER_SEEN)
# --------------------------------------------------------------------------
@pytest.mark.parametrize("name", list(SMALL))
@pytest.mark.parametrize("k,L,table", [(1, 1, "f32"), (10, 16, "f32"),
                                       (5, 33, "f32"), (10, 100, "f32"),
                                       (10, 300, "f32"), (10, 1024, "f32"),
                                       (10, 64, "f16"), (10, 200, "u8"),
                                       (10, 64, "exact"),
                                       (10, 300, "exact")])
def test_seen_filter_bit_exact(small_indexes, name, k, L, table):
    """The seen bitmap drops neighbours seen before the worklist rank: ids,
    distances, expanded nodes and iteration counts equal the oracle's
    Algorithm 2 with an exact seen-set, for every table form."""
    ix, q, gi = small_indexes[name]
    run_and_compare(ix, gi, q, k, L, table=table, filter="seen",
                    label=f"{name} k={k} L={L} {table} seen")


@pytest.mark.parametrize("name", ["u8-d64-m16", "f32-d128-m16",
                                  "i8-d96-m48"])
@pytest.mark.parametrize("k,L,table", [(10, 64, "f32"), (10, 256, "u8"),
                                       (10, 100, "exact")])
def test_seen_filter_host_adjacency_bit_exact(small_indexes,
                                              small_host_indexes, name, k, L,
                                              table):
    """Host-resident rows with the seen bitmap: equal to the oracle."""
    ix, q, _ = small_indexes[name]
    run_and_compare(ix, small_host_indexes[name], q, k, L, table=table,
                    filter="seen", label=f"{name} host seen")


@pytest.mark.parametrize("k,L,table", [(10, 64, "f32"), (10, 512, "f32"),
                                       (10, 100, "exact")])
def test_seen_filter_saturated_log_bit_exact(small_indexes, k, L, table):
    """A query whose log is full only tests its bitmap from then on (new
    neighbours are ranked and the set union drops repeats): results are
    still the oracle's, and the next search, with the log in full use, is
    exact as well (the bits the short-logged queries set were cleared)."""
    for name in ("u8-d128-m32", "f32-d32-m16"):
        ix, q, gi = small_indexes[name]
        run_and_compare(ix, gi, q, k, L, table=table, filter="seen",
                        seen_log_short=True, label=f"{name} short log")
        run_and_compare(ix, gi, q, k, L, table=table, filter="seen",
                        label=f"{name} after short log")


def test_seen_filter_repeated_launches_leave_the_bitmap_clear(small_indexes):
    """Each query clears the bits it set: many launches with different
    query sets, worklist sizes and table forms through one workspace each
    equal the set-union search (whose results depend on no state)."""
    ix, q, gi = small_indexes["u8-d128-m32"]
    rng = np.random.default_rng(31)
    qt = to_dev(q)
    for rep in range(12):
        L = int(rng.choice([16, 64, 200, 700]))
        table = ["f32", "u8", "exact"][rep % 3]
        sel = np.sort(rng.choice(len(q), int(rng.integers(1, len(q) + 1)),
                                 replace=False))
        qs = qt[torch.from_numpy(sel).cuda()].contiguous()
        a = gi.search(qs, 10, L, table=table, filter="seen", want_cand=4 * L)
        b = gi.search(qs, 10, L, table=table, filter="exact",
                      want_cand=4 * L)
        torch.cuda.synchronize()
        for x, y in zip(a, b):
            assert np.array_equal(x.cpu().numpy(), y.cpu().numpy()), (rep, L)


@pytest.mark.parametrize("name", ["u8-d128-m32", "f32-d32-m16"])
@pytest.mark.parametrize("table", ["f32", "u8", "exact"])
def test_seen_filter_mixed_batch_equals_each_query_alone(small_indexes, name,
                                                         table):
    """A mixed batch (per-query k and L) with the seen bitmap: each row
    equals that query searched alone with the set union."""
    ix, q, gi = small_indexes[name]
    nq = len(q)
    rng = np.random.default_rng(77)
    Ls = rng.choice([8, 16, 64, 150], nq).astype(np.int32)
    ks = np.minimum(rng.choice([1, 5, 10], nq), Ls).astype(np.int32)
    ids, d = gi.search(to_dev(q), 10, 150, table=table, filter="seen",
                       query_L=to_dev(Ls), query_k=to_dev(ks))
    torch.cuda.synchronize()
    ids, d = u32(ids), d.cpu().numpy()
    for i in range(nq):
        r = oracle.search(ix, q[i:i + 1], int(ks[i]), int(Ls[i]),
                          table=table)
        assert np.array_equal(ids[i, :ks[i]], r["ids"][0]), i
        assert np.array_equal(f32bits(d[i, :ks[i]]),
                              f32bits(r["dists"][0])), i
        assert (ids[i, ks[i]:] == NONE).all()


def test_seen_filter_stopped_launch_leaves_the_bitmap_clear(small_indexes):
    """Queries cut short by a stop request clear the bits they set: a
    search after a stopped launch equals the oracle."""
    import time
    ix, q, gi = small_indexes["u8-d128-m32"]
    bang = bang_mod()
    qrep = to_dev(np.tile(q, (400, 1)))
    ab = bang.StopRequest()
    ids, d, cnt = gi.search(qrep, 10, 1024, want_counters=True, abort=ab,
                            filter="seen")
    torch.cuda.synchronize()
    gi.search(qrep, 10, 1024, want_counters=True, abort=ab, filter="seen",
              out=(ids, d))
    time.sleep(0.002)
    ab.set()
    torch.cuda.synchronize()
    ab.clear()
    run_and_compare(ix, gi, q, 10, 1024, filter="seen",
                    label="after a stopped seen-filter launch")
    run_and_compare(ix, gi, q, 10, 64, table="exact", filter="seen",
                    label="after a stopped seen-filter launch (exact)")
    ab.close()


@pytest.mark.parametrize("table", ["f32", "exact"])
def test_seen_filter_timed_search_same_results(small_indexes, table):
    """The timed copy of the seen-filter search returns the same results
    and reports its phases."""
    ix, q, gi = small_indexes["u8-d128-m32"]
    qt = to_dev(q)
    a = gi.search(qt, 10, 256, table=table, filter="seen", want_cand=1024,
                  want_counters=True)
    b = gi.search(qt, 10, 256, table=table, filter="seen", want_cand=1024,
                  want_counters=True, want_phases=True)
    torch.cuda.synchronize()
    for x, y in zip(a, b[:4]):
        assert np.array_equal(x.cpu().numpy(), y.cpu().numpy())
    ph = b[4].cpu().numpy().astype(np.int64)
    assert ph.shape == (len(q), 7) and (ph[:, 2] > 0).all()


def test_sift1m_seen_filter_sampled_bit_exact():
    """1M uint8 points with the seen bitmap, in the benchmark's launch
    configuration: a seeded sample of queries equals the oracle bit for
    bit at the bench points."""
    w, ix, d = load_workload("sift1m")
    gi = bang_mod().Index(ix.base, ix.adj, ix.medoid, ix.codebooks, ix.codes)
    q = d["queries"]
    qt = to_dev(q)
    sample = np.sort(np.random.default_rng(2031).choice(len(q), 96,
                                                        replace=False))
    for L, table in [(64, "f32"), (768, "f32"), (768, "u8"), (256, "exact"),
                     (1024, "f16")]:
        cap = oracle.iter_cap_for(L)
        ids, dist, cand, cnt = gi.search(qt, w.k, L, want_cand=cap,
                                         want_counters=True, table=table,
                                         filter="seen")
        torch.cuda.synchronize()
        ref = oracle.search(ix, q[sample], w.k, L, want_cand=True,
                            table=table, mode=oracle.MODES["exact"])
        assert np.array_equal(u32(cnt)[sample, 0], ref["iters"]), L
        assert np.array_equal(u32(cand)[sample], ref["cand"]), L
        assert np.array_equal(u32(ids)[sample], ref["ids"]), L
        assert np.array_equal(f32bits(dist.cpu().numpy()[sample]),
                              f32bits(ref["dists"])), L


# --------------------------------------------------------------------------
# tables built beforehand: the BF16-MFMA build and bang_search_opts.tables
# --------------------------------------------------------------------------
@pytest.mark.parametrize("name", list(SMALL))
def test_bf16_mfma_tables_within_the_bound(small_indexes, name):
    """Every entry of the BF16-MFMA table lies within the oracle's error
    bound of the exact (FP64) table, for each data type and d/m = 2, 4, 8;
    rows past a multiple of 32 queries are written too."""
    ix, q, gi = small_indexes[name]
    T = gi.build_pq_tables(to_dev(q), bf16=True)
    torch.cuda.synchronize()
    T = T.cpu().numpy().astype(np.float64)
    T64, E = oracle.bf16_table_bound(q, ix.codebooks)
    err = np.abs(T - T64)
    assert (err <= E).all(), (name, float((err / E).max()))
    # the rounding is visible (the build is not the FP32 one) unless every
    # input is exactly representable
    T32 = oracle.pq_tables(q, ix.codebooks).astype(np.float64)
    assert not np.array_equal(T, T32)


@pytest.mark.parametrize("name", ["u8-d128-m32", "f32-d32-m16",
                                  "i8-d96-m48"])
@pytest.mark.parametrize("k,L,table", [(10, 64, "f32"), (10, 256, "f16"),
                                       (5, 100, "u8"), (10, 16, "f32")])
def test_search_by_given_tables_bit_exact(small_indexes, name, k, L, table):
    """A search ranking by tables given beforehand (the oracle's canonical
    FP32 tables, moved to the device) equals the oracle's search, which
    builds the same tables itself: ids, distances and expanded nodes."""
    ix, q, gi = small_indexes[name]
    T = to_dev(oracle.pq_tables(q, ix.codebooks))
    cap = oracle.iter_cap_for(L)
    ids, d, cand, cnt = gi.search(to_dev(q), k, L, want_cand=cap,
                                  want_counters=True, table=table, tables=T)
    torch.cuda.synchronize()
    ref = oracle.search(ix, q, k, L, want_cand=True, table=table)
    assert np.array_equal(u32(cnt)[:, 0], ref["iters"])
    assert np.array_equal(u32(cand), ref["cand"])
    assert np.array_equal(u32(ids), ref["ids"])
    assert np.array_equal(f32bits(d.cpu().numpy()), f32bits(ref["dists"]))


@pytest.mark.parametrize("table", ["f32", "f16", "u8"])
def test_search_by_bf16_mfma_tables_returns_exact_distances(small_indexes,
                                                            table):
    """Searching by the BF16-MFMA tables: the answer is re-ranked exactly,
    so each returned distance is the canonical FP32 distance of its id (the
    oracle's re-rank of the returned ids), rows are sorted and distinct."""
    ix, q, gi = small_indexes["u8-d128-m32"]
    qt = to_dev(q)
    T = gi.build_pq_tables(qt, bf16=True)
    ids, d = gi.search(qt, 10, 128, table=table, tables=T)
    torch.cuda.synchronize()
    ids, d = u32(ids), d.cpu().numpy()
    rid, rd = oracle.rerank(ix, q, ids, 10)
    assert np.array_equal(rid, ids)
    assert np.array_equal(f32bits(rd), f32bits(d))
    assert all(len(set(r)) == len(r) for r in ids)


def test_search_by_tables_rejected_for_exact_distances(small_indexes):
    ix, q, gi = small_indexes["u8-d64-m16"]
    bang = bang_mod()
    T = gi.build_pq_tables(to_dev(q))
    with pytest.raises(bang.BangError):
        gi.search(to_dev(q), 10, 32, table="exact", tables=T)


@pytest.mark.parametrize("wname,nq", [("sift1m", 96), ("deep1m", 64)])
def test_bf16_mfma_tables_within_the_bound_1m(wname, nq):
    """The benchmark's indexes (d/m = 4 on the 1M uint8 index, d/m = 2 on
    the d=96 float index): a seeded sample of queries, every entry within
    the bound."""
    w, ix, d = load_workload(wname)
    gi = bang_mod().Index(ix.base, ix.adj, ix.medoid, ix.codebooks, ix.codes)
    sel = np.sort(np.random.default_rng(5).choice(len(d["queries"]), nq,
                                                  replace=False))
    q = d["queries"][sel]
    T = gi.build_pq_tables(to_dev(q), bf16=True)
    torch.cuda.synchronize()
    T64, E = oracle.bf16_table_bound(q, ix.codebooks)
    assert (np.abs(T.cpu().numpy().astype(np.float64) - T64) <= E).all()


@pytest.mark.parametrize("table", ["f32", "exact"])
def test_take_order_and_wave_cap_change_no_result(small_indexes, table):
    """A mixed batch taken in other orders (reversed, random, longest
    worklist first, with ids past the batch to skip) and with fewer
    resident waves returns the same rows, bit for bit."""
    ix, q, gi = small_indexes["u8-d128-m32"]
    nq = len(q)
    rng = np.random.default_rng(21)
    Ls = rng.choice([8, 16, 64, 150], nq).astype(np.int32)
    ks = np.minimum(rng.choice([1, 5, 10], nq), Ls).astype(np.int32)
    qt, qL, qk = to_dev(q), to_dev(Ls), to_dev(ks)
    base = gi.search(qt, 10, 150, table=table, query_L=qL, query_k=qk)
    torch.cuda.synchronize()
    orders = [np.arange(nq)[::-1], rng.permutation(nq),
              np.argsort(-Ls, kind="stable")]
    for o in orders:
        for w in (0, 1, 2):
            got = gi.search(qt, 10, 150, table=table, query_L=qL,
                            query_k=qk, order=to_dev(o.astype(np.int32)),
                            waves_per_cu=w)
            torch.cuda.synchronize()
            for x, y in zip(base, got):
                assert np.array_equal(x.cpu().numpy(), y.cpu().numpy()), w


def test_rows_past_4_gib_sampled_bit_exact():
    """A synthetic 17M-node int8 graph (synth.scale_graph_index: rows of
    random ids over the whole range): the packed rows in device memory (39
    GB) and the pinned host adjacency (4.4 GB) both reach past 2^32 bytes,
    so the search addresses rows with 64-bit offsets; 48 queries equal the
    oracle (ids, distances, expanded nodes and iteration counts) with both
    placements."""
    n = 17_000_000
    d = synth.scale_graph_index(n, nq=48)
    assert n * 2304 > 1 << 32 and n * 64 * 4 > 1 << 32
    ix = oracle.Index(d["base"], d["adj"], d["medoid"], d["codebooks"],
                      d["codes"])
    q = d["queries"]
    k, L = 10, 64
    cap = oracle.iter_cap_for(L)
    ref = oracle.search(ix, q, k, L, want_cand=True)
    # the search reaches rows above both 4 GiB marks
    expanded = ref["cand"][ref["cand"] != NONE].astype(np.int64)
    assert (expanded * 2304 >= 1 << 32).any()
    assert (expanded * 256 >= 1 << 32).any()
    for host in (False, True):
        gi = bang_mod().Index(d["base"], d["adj"], d["medoid"],
                              d["codebooks"], d["codes"], host_adj=host)
        ids, dist, cand, cnt = gi.search(to_dev(q), k, L, want_cand=cap,
                                         want_counters=True)
        torch.cuda.synchronize()
        assert np.array_equal(u32(cnt)[:, 0], ref["iters"]), host
        assert np.array_equal(u32(cand), ref["cand"]), host
        assert np.array_equal(u32(ids), ref["ids"]), host
        assert np.array_equal(f32bits(dist.cpu().numpy()),
                              f32bits(ref["dists"])), host
        gi.close()
