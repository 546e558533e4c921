"""Pins for the CPU oracle: checks against what the paper and the
mathematics fix, not against the oracle itself.

Each test names the passage or the mathematical fact it rests on.
"""
import numpy as np
import pytest

import oracle
import synth
from oracle.graph import build_graph
from oracle.pq import kmeans, kmeans_assign, pq_encode, train_pq

NONE = 0xFFFFFFFF


# --------------------------------------------------------------------------
# helpers: small indexes built with the oracle
# --------------------------------------------------------------------------
def make_index(w, graph=True):
    rs = synth.streams(w)
    base, q = synth.base_and_queries(w)
    cb = train_pq(base, w.m, w.kmeans_iters, rs["pq_init"])
    codes = pq_encode(base, cb)
    s = oracle.medoid(base)
    perm = rs["vamana_order"].permutation(w.n).astype(np.uint32)
    if graph:
        adj, info = build_graph(base, w.R, w.L_build, w.alpha, perm, s)
    else:
        adj = oracle.vamana_build(base, w.R, w.L_build, w.alpha, perm, s)
        info = {}
    return oracle.Index(base, adj, s, cb, codes), q, info


@pytest.fixture(scope="module")
def small_f32():
    return make_index(synth.small("f32", n=1500, d=32, nq=24))


@pytest.fixture(scope="module")
def small_u8():
    return make_index(synth.small("u8", n=1200, d=32, nq=24, seed_index=101))


@pytest.fixture(scope="module")
def small_i8():
    return make_index(synth.small("i8", n=900, d=16, nq=16, seed_index=102))


def exact_sq(base, q):
    """Squared L2 from q to every base row, exact (int64 or FP64)."""
    if base.dtype == np.float32:
        b = base.astype(np.float64)
        return ((b - q.astype(np.float64)) ** 2).sum(1)
    b = base.astype(np.int64)
    return ((b - q.astype(np.int64)) ** 2).sum(1)


# --------------------------------------------------------------------------
# Stage 1 + ADC: the worked example of Figure 2
# --------------------------------------------------------------------------
def toy_setup(golden):
    g = golden("toy_fig2.json")
    pts = np.array(g["points"], dtype=np.uint8)
    cid = np.array(g["fig2b_cluster_id"], dtype=np.uint8)
    cb = np.full((1, 256, 2), 255.0, dtype=np.float32)
    cb[0, cid] = pts.astype(np.float32)          # centroid = the point itself
    q = np.array([g["query"]], dtype=np.uint8)
    return g, pts, cid, cb, q


def test_toy_table_and_adc_match_fig2b(golden):
    """Figure 2b: with m=1 and every point its own centroid, the PQ distance
    of a node is the table entry of its cluster id."""
    g, pts, cid, cb, q = toy_setup(golden)
    T = oracle.pq_tables(q, cb)
    assert T.shape == (1, 1, 256)
    assert np.array_equal(T[0, 0, cid], np.array(g["fig2b_pq_distance"],
                                                 dtype=np.float32))
    codes = cid.reshape(-1, 1)
    d = oracle.adc(T[0], codes, np.arange(12, dtype=np.uint32))
    assert np.array_equal(d, np.array(g["fig2b_pq_distance"], np.float32))


def test_toy_rerank_matches_fig2d_and_final_order(golden):
    """Figure 2d lists the expanded candidates with exact distances; the
    text after the figure gives their sorted order and the top-2."""
    g, pts, cid, cb, q = toy_setup(golden)
    adj = np.full((12, 2), NONE, dtype=np.uint32)
    ix = oracle.Index(pts, adj, 6, cb, cid.reshape(-1, 1))
    cand = np.array([g["fig2d_expansion_order"]], dtype=np.uint32)
    ids, d = oracle.rerank(ix, q, cand, 8)
    assert ids[0].tolist() == g["final_sorted"]
    ids2, _ = oracle.rerank(ix, q, cand, 2)
    assert ids2[0].tolist() == g["top2"]
    exact = dict(zip(g["fig2d_expansion_order"], g["fig2d_exact_distance"]))
    assert d[0].tolist() == [float(exact[i]) for i in g["final_sorted"]]


# --------------------------------------------------------------------------
# Stage 1: table closed form
# --------------------------------------------------------------------------
@pytest.mark.parametrize("dtype", ["f32", "u8", "i8"])
def test_table_equals_subspace_distances(dtype):
    """T[j][c] is the squared distance between the j-th query subvector and
    centroid c of subspace j (section on the PQ distance table)."""
    rng = np.random.default_rng(7)
    m, ds = 8, 4
    d = m * ds
    cb = rng.normal(size=(m, 256, ds)).astype(np.float32) * 30
    if dtype == "f32":
        q = rng.normal(size=(5, d)).astype(np.float32) * 30
    elif dtype == "u8":
        q = rng.integers(0, 256, size=(5, d)).astype(np.uint8)
    else:
        q = rng.integers(-128, 128, size=(5, d)).astype(np.int8)
    T = oracle.pq_tables(q, cb)
    qs = q.astype(np.float64).reshape(5, m, 1, ds)
    ref = ((qs - cb.astype(np.float64)[None]) ** 2).sum(-1)
    np.testing.assert_allclose(T, ref, rtol=2e-6, atol=1e-3)


def test_table_integer_inputs_are_exact():
    """With integer queries and integer centroids every partial sum is an
    integer below 2^24, so the FP32 table is exact."""
    rng = np.random.default_rng(3)
    cb = rng.integers(0, 256, size=(4, 256, 4)).astype(np.float32)
    q = rng.integers(0, 256, size=(3, 16)).astype(np.uint8)
    T = oracle.pq_tables(q, cb)
    ref = ((q.astype(np.int64).reshape(3, 4, 1, 4)
            - cb.astype(np.int64)[None]) ** 2).sum(-1)
    assert np.array_equal(T.astype(np.int64), ref)


def test_adc_equals_distance_to_decoded_vector(small_f32):
    """ADC(x) = sum_j T[j][code_j] = ||q - x_hat||^2 where x_hat is x's
    decoded vector (concatenated centroids); exact in real arithmetic."""
    ix, q, _ = small_f32
    T = oracle.pq_tables(q[:3], ix.codebooks)
    ids = np.arange(0, ix.n, 7, dtype=np.uint32)
    ds = ix.d // ix.m
    for a in range(3):
        d = oracle.adc(T[a], ix.codes, ids).astype(np.float64)
        xhat = ix.codebooks[np.arange(ix.m)[None, :], ix.codes[ids]]
        xhat = xhat.reshape(len(ids), ix.m * ds).astype(np.float64)
        ref = ((xhat - q[a].astype(np.float64)) ** 2).sum(1)
        np.testing.assert_allclose(d, ref, rtol=1e-5)


# --------------------------------------------------------------------------
# Stage 2: greedy search
# --------------------------------------------------------------------------
@pytest.mark.parametrize("fx", ["small_f32", "small_u8", "small_i8"])
def test_search_with_L_at_least_n_is_brute_force(fx, request):
    """With t >= n nothing is ever evicted, so on a graph where every node
    is reachable from s (checked by breadth-first search) every node is
    expanded; the re-rank then returns the exact k nearest, and Algorithm
    1's own answer is the k nearest by PQ distance over all nodes."""
    ix, q, info = request.getfixturevalue(fx)
    assert oracle.reachable(ix.adj, ix.medoid) == ix.n
    L = 256 if ix.n <= 256 else ix.n
    k = 10
    # L above the GPU's 256 limit is fine for the oracle
    out = oracle.search(ix, q[:6], k, L, c_max=ix.n, iter_cap=ix.n + 1,
                        want_pq=True)
    assert (out["iters"] == ix.n).all()
    assert (out["status"] == 0).all()
    T = oracle.pq_tables(q[:6], ix.codebooks)
    allid = np.arange(ix.n, dtype=np.uint32)
    for a in range(6):
        ex = exact_sq(ix.base, q[a])
        order = np.lexsort((allid, ex))[:k]
        assert out["ids"][a].tolist() == order.tolist()
        if ix.base.dtype == np.float32:
            # FP32 left-to-right sum vs the FP64 value: a few ulp apart
            np.testing.assert_allclose(out["dists"][a], ex[order], rtol=2e-6)
        else:
            assert np.array_equal(out["dists"][a], ex[order].astype(np.float32))
        pqd = oracle.adc(T[a], ix.codes, allid)
        porder = np.lexsort((allid, pqd))[:k]
        assert out["pq_ids"][a].tolist() == porder.tolist()


@pytest.mark.parametrize("fx", ["small_f32", "small_u8"])
@pytest.mark.parametrize("L", [10, 16, 33, 64])
def test_algorithm1_and_filtered_form_agree(fx, L, request):
    """Algorithm 1 (set union into the worklist) and Algorithm 2's filtered
    form (distance only for never-seen nodes, sort, merge) expand the same
    nodes in the same order and return the same answer: a node evicted from
    a full worklist has a key at or above the worklist's last key, which
    never grows once the worklist is full, so it can never re-enter."""
    ix, q, _ = request.getfixturevalue(fx)
    a = oracle.search(ix, q, 10, L, mode=0, want_pq=True, want_cand=True)
    b = oracle.search(ix, q, 10, L, mode=1, want_pq=True, want_cand=True)
    for key in ("ids", "dists", "pq_ids", "pq_dists", "cand", "iters"):
        assert np.array_equal(a[key], b[key]), key
    # the filtered form computes fewer distances
    assert (b["added"] <= a["added"]).all()


def test_search_invariants(small_u8):
    """Invariants of Algorithm 1: every expansion is a distinct node; the
    number of iterations is at least min(t, reachable) (section on the
    worklist size: every worklist entry must be visited); results are
    sorted by (distance, id) and distinct."""
    ix, q, _ = small_u8
    for L in (10, 32):
        out = oracle.search(ix, q, 10, L, want_cand=True)
        for a in range(len(q)):
            I = out["iters"][a]
            c = out["cand"][a][:I]
            assert len(set(c.tolist())) == I
            assert I >= min(L, ix.n)
            assert (out["cand"][a][I:] == NONE).all()
            d, ids = out["dists"][a], out["ids"][a]
            keys = list(zip(d.tolist(), ids.tolist()))
            assert keys == sorted(keys)
            assert len(set(ids.tolist())) == len(ids)


def test_iteration_cap_sets_status(small_u8):
    ix, q, _ = small_u8
    out = oracle.search(ix, q[:4], 10, 32, iter_cap=5, want_cand=True)
    assert (out["iters"] == 5).all() and (out["status"] == 1).all()


def test_search_rejects_k_above_L(small_u8):
    ix, q, _ = small_u8
    with pytest.raises(ValueError):
        oracle.search(ix, q[:2], 20, 10)


def test_short_result_is_padded():
    """Fewer reachable nodes than k: the tail is (NONE, +inf)."""
    w = synth.small("u8", n=300, d=16, nq=4, seed_index=103)
    base, q = synth.base_and_queries(w)
    rs = synth.streams(w)
    cb = train_pq(base, w.m, 3, rs["pq_init"])
    codes = pq_encode(base, cb)
    adj = np.full((w.n, 4), NONE, dtype=np.uint32)
    adj[0, :3] = [1, 2, 3]                      # only 4 nodes reachable
    ix = oracle.Index(base, adj, 0, cb, codes)
    out = oracle.search(ix, q, 10, 16)
    assert (out["iters"] == 4).all()
    assert (out["ids"][:, 4:] == NONE).all()
    assert np.isinf(out["dists"][:, 4:]).all()
    assert set(out["ids"][0, :4].tolist()) == {0, 1, 2, 3}


# --------------------------------------------------------------------------
# Stage 3: re-rank
# --------------------------------------------------------------------------
@pytest.mark.parametrize("fx", ["small_f32", "small_u8", "small_i8"])
def test_rerank_is_sort_by_exact_distance(fx, request):
    """Re-rank definition (section "Re-ranking"): exact distances of the
    candidates, sorted by (distance, id), top-k.  Padding is skipped."""
    ix, q, _ = request.getfixturevalue(fx)
    rng = np.random.default_rng(11)
    cm = 40
    cand = rng.choice(ix.n, size=(len(q), cm)).astype(np.uint32)
    cand[:, -5:] = NONE
    cand[0, :] = NONE
    for a in range(len(q)):
        cand[a, :cm - 5] = rng.choice(ix.n, cm - 5, replace=False)
    cand[0, :] = NONE
    ids, d = oracle.rerank(ix, q, cand, 10)
    assert (ids[0] == NONE).all() and np.isinf(d[0]).all()
    for a in range(1, len(q)):
        c = cand[a][cand[a] != NONE]
        ex = exact_sq(ix.base[c], q[a])
        o = np.lexsort((c, ex))[:10]
        assert ids[a].tolist() == c[o].tolist()
        np.testing.assert_allclose(d[a], ex[o], rtol=1e-6)
        if ix.base.dtype != np.float32:
            assert np.array_equal(d[a], ex[o].astype(np.float32))


def test_cmax_keeps_smallest_pq_keys(small_u8):
    """With more expanded nodes than c_max, the c_max with the smallest
    (PQ distance, id) go to the re-rank: the result equals re-ranking that
    subset directly."""
    ix, q, _ = small_u8
    L, cm = 32, 20
    out = oracle.search(ix, q, 10, L, c_max=cm, want_cand=True)
    T = oracle.pq_tables(q, ix.codebooks)
    for a in range(len(q)):
        I = out["iters"][a]
        c = out["cand"][a][:I]
        assert I > cm
        pq = oracle.adc(T[a], ix.codes, c)
        keep = c[np.lexsort((c, pq))[:cm]]
        ids, d = oracle.rerank(ix, q[a:a + 1], keep[None, :], 10)
        assert ids[0].tolist() == out["ids"][a].tolist()


# --------------------------------------------------------------------------
# Ground truth
# --------------------------------------------------------------------------
@pytest.mark.parametrize("dtype", ["f32", "u8", "i8"])
def test_bruteforce_matches_sorted_exact_distances(dtype):
    w = synth.small(dtype, n=700, d=24, nq=9, seed_index=104)
    base, q = synth.base_and_queries(w)
    base[5] = base[6]          # an exact tie: ids break it
    ids, d = oracle.bruteforce(base, q, 12)
    allid = np.arange(w.n)
    for a in range(len(q)):
        ex = exact_sq(base, q[a])
        o = np.lexsort((allid, ex))[:12]
        assert ids[a].tolist() == o.tolist()
        if dtype == "f32":      # numpy sums pairwise, the oracle in order
            np.testing.assert_allclose(d[a], ex[o], rtol=1e-12)
        else:
            assert np.array_equal(d[a], ex[o].astype(np.float64))


# --------------------------------------------------------------------------
# PQ training and encoding
# --------------------------------------------------------------------------
def test_kmeans_objective_non_increasing_and_assignment_optimal():
    """Lloyd's iterations never increase the k-means objective; each point
    is assigned to its nearest centroid, ties to the lowest id."""
    rng = np.random.default_rng(5)
    X = rng.normal(size=(3000, 3)) * [1, 2, 3]
    hist = []
    C = kmeans(X, 256, 8, np.random.default_rng(6), history=hist)
    assert all(b <= a * (1 + 1e-12) for a, b in zip(hist, hist[1:]))
    a, obj = kmeans_assign(X, C)
    D = ((X[:, None, :] - C[None]) ** 2).sum(-1)
    assert np.array_equal(a, D.argmin(1))
    np.testing.assert_allclose(obj, D.min(1).sum(), rtol=1e-12)


def _lloyd_reference(X, init_idx, iters):
    """Lloyd's k-means written out plainly: nearest centroid by squared
    difference (ties to the lowest id), then each centroid becomes the mean
    of its points, summed in point order; an empty cluster keeps its
    centroid."""
    C = [list(map(float, X[i])) for i in init_idx]
    K = len(C)
    for _ in range(iters):
        assign = []
        for x in X:
            best, bi = None, 0
            for c in range(K):
                dd = sum((float(x[t]) - C[c][t]) ** 2 for t in range(len(x)))
                if best is None or dd < best:
                    best, bi = dd, c
            assign.append(bi)
        for c in range(K):
            pts = [X[i] for i in range(len(X)) if assign[i] == c]
            if pts:
                C[c] = [sum(float(p[t]) for p in pts) / len(pts)
                        for t in range(len(pts[0]))]
    return np.array(C)


def test_kmeans_and_train_pq_equal_plain_lloyd():
    """k-means (the PQ training reading: K = 256, init from distinct sample
    points, FP64 Lloyd, empty clusters keep their centroid) equals Lloyd's
    algorithm written out plainly, on 300 integer points (exact sums), and
    train_pq runs it per subspace in subspace order from one generator."""
    rng = np.random.default_rng(7)
    X = rng.integers(0, 12, size=(300, 4)).astype(np.float64)
    g1, g2 = np.random.default_rng(8), np.random.default_rng(8)
    C = kmeans(X[:, :2], 256, 3, g1)
    init = g2.choice(300, 256, replace=False)
    assert np.array_equal(C, _lloyd_reference(X[:, :2], init, 3))
    cb = train_pq(X, 2, 3, np.random.default_rng(8))
    assert np.array_equal(cb[0], C.astype(np.float32))
    init2 = g2.choice(300, 256, replace=False)
    assert np.array_equal(cb[1], _lloyd_reference(X[:, 2:], init2, 3)
                          .astype(np.float32))


def test_pq_encode_is_nearest_centroid_per_subspace(small_u8):
    ix, _, _ = small_u8
    ds = ix.d // ix.m
    X = ix.base[:200].astype(np.float64).reshape(200, ix.m, 1, ds)
    D = ((X - ix.codebooks.astype(np.float64)[None]) ** 2).sum(-1)
    assert np.array_equal(ix.codes[:200], D.argmin(-1).astype(np.uint8))


def test_medoid_is_point_nearest_the_mean(small_f32):
    ix, _, _ = small_f32
    b = ix.base.astype(np.float64)
    assert ix.medoid == int(((b - b.mean(0)) ** 2).sum(1).argmin())


# --------------------------------------------------------------------------
# Graph: structural invariants, RobustPrune and the whole build against
# plain re-statements on tiny inputs
# --------------------------------------------------------------------------
@pytest.mark.parametrize("fx", ["small_f32", "small_u8", "small_i8"])
def test_graph_invariants(fx, request):
    ix, _, info = request.getfixturevalue(fx)
    adj = ix.adj
    n, R = adj.shape
    valid = adj != NONE
    assert (adj[valid] < n).all()
    assert not (adj == np.arange(n, dtype=np.uint32)[:, None]).any()
    for row in adj:
        r = row[row != NONE]
        assert len(set(r.tolist())) == len(r)
    assert oracle.reachable(adj, ix.medoid) == n
    assert info["reachable"] == n


# RobustPrune (Vamana's pruning step; the paper names the Vamana graph in
# "Graph Index" and gives R and alpha in "Algorithm Parameters").  The
# candidates of the hand-worked case, 2-D integer points, p = point 0 at
# the origin (d = Euclidean distance to p):
#   id 1 a=( 2, 0) d=2      id 2 b=( 3, 1) d=3.162   id 3 c=( 0, 3) d=3
#   id 4 e=(-4, 0) d=4      id 5 f=( 1, 4) d=4.123   id 6 g=(-3,-3) d=4.243
#   id 7 h=( 5, 0) d=5      id 8 k=( 4,-6) d=7.211
_PRUNE_PTS = np.array([[0, 0], [2, 0], [3, 1], [0, 3], [-4, 0], [1, 4],
                       [-3, -3], [5, 0], [4, -6]], dtype=np.float32)


def test_robust_prune_hand_worked_alpha_1_2():
    """alpha = 1.2, order a, c, b, e, f, g, h, k.
    Keep a: b goes (1.2 d(a,b) = 1.2 sqrt 2 = 1.70 <= 3.16), h goes
    (1.2 * 3 = 3.6 <= 5); c stays (1.2 sqrt 13 = 4.33 > 3), e (7.2 > 4),
    f (1.2 sqrt 17 = 4.95 > 4.12), g (1.2 sqrt 34 = 7.0 > 4.24), k
    (1.2 sqrt 40 = 7.59 > sqrt 52 = 7.21).
    Keep c: f goes (1.2 sqrt 2 = 1.70 <= 4.12); e (6 > 4), g (8.05 > 4.24),
    k (1.2 sqrt 97 = 11.8 > 7.21) stay.
    Keep e: g goes (1.2 sqrt 10 = 3.79 <= 4.24); k stays (12 > 7.21).
    Keep k.  R = 4 -> [a, c, e, k]; R = 3 stops after e.
    Slips this separates: alpha on squared distances drops k at the first
    step (1.2 * 40 = 48 <= 52), giving [a, c, e] for R = 4."""
    cand = np.arange(1, 9, dtype=np.uint32)
    assert oracle.robust_prune(_PRUNE_PTS, 0, cand, 1.2, 4).tolist() == \
        [1, 3, 4, 8]
    assert oracle.robust_prune(_PRUNE_PTS, 0, cand, 1.2, 3).tolist() == \
        [1, 3, 4]
    # order of the candidate list does not matter; p itself and repeats
    # are not candidates
    shuf = np.array([8, 0, 5, 3, 3, 1, 7, 2, 6, 4, 1, 8], dtype=np.uint32)
    assert oracle.robust_prune(_PRUNE_PTS, 0, shuf, 1.2, 4).tolist() == \
        [1, 3, 4, 8]
    # alpha = 1 (the first Vamana pass) drops what a kept point is at least
    # as close to: keep a, which drops b (sqrt 2 <= 3.16), h (3 <= 5), k
    # (sqrt 40 <= sqrt 52) and f at equality (d(a,f) = d(p,f) = sqrt 17);
    # keep c, then e, which drops g (sqrt 10 <= 4.24)
    assert oracle.robust_prune(_PRUNE_PTS, 0, cand, 1.0, 8).tolist() == \
        [1, 3, 4]


def test_robust_prune_boundary_and_ties():
    """alpha * d(p*, p') == d(p, p') drops p' (the rule is <=): with
    alpha = 1.5 (exact in binary), p = (0,0), p* = (1,0), p' = (3,0):
    1.5 * 2 = 3.  With alpha = 1.2 and p' = (6,0): 1.2 * 5 = 6.  Equal
    distances to p are taken in id order."""
    pts = np.array([[0, 0], [1, 0], [3, 0]], dtype=np.float32)
    assert oracle.robust_prune(pts, 0, np.array([1, 2], np.uint32),
                               1.5, 4).tolist() == [1]
    # a slightly larger alpha keeps the far point (1.51 * 2 > 3)
    assert oracle.robust_prune(pts, 0, np.array([1, 2], np.uint32),
                               1.51, 4).tolist() == [1, 2]
    pts = np.array([[0, 0], [1, 0], [6, 0]], dtype=np.float32)
    assert oracle.robust_prune(pts, 0, np.array([2, 1], np.uint32),
                               1.2, 4).tolist() == [1]
    # ties: ids 3 and 5 both at distance 2; 3 first, then 5 stays
    # (1.2 * sqrt 8 = 3.39 > 2)
    pts = np.zeros((6, 2), np.float32)
    pts[3] = (2, 0)
    pts[5] = (0, 2)
    pts[[1, 2, 4]] = (50, 50)
    assert oracle.robust_prune(pts, 0, np.array([5, 3], np.uint32),
                               1.2, 2).tolist() == [3, 5]


def _prune_reference_ok(pts, p, cand, out, a2num, a2den, R):
    """Brute-force characterisation of RobustPrune's output in exact
    integer arithmetic (alpha^2 = a2num / a2den): in (distance, id) order,
    a candidate is kept iff fewer than R were kept before it and no
    earlier kept point p* has alpha^2 d2(p*, x) <= d2(p, x)."""
    X = pts.astype(np.int64)

    def d2(i, j):
        return int(((X[i] - X[j]) ** 2).sum())

    order = sorted({int(c) for c in cand if int(c) != p},
                   key=lambda c: (d2(p, c), c))
    kept = []
    for x in order:
        if len(kept) == R:
            break
        if all(a2num * d2(y, x) > a2den * d2(p, x) for y in kept):
            kept.append(x)
    return kept == [int(v) for v in out]


@pytest.mark.parametrize("seed", range(6))
def test_robust_prune_matches_brute_force_rule(seed):
    """Random integer points, alpha = 1.5 (alpha^2 = 9/4 exactly), random
    candidate lists with repeats and p itself: the kept list is exactly the
    greedy rule's, which also means every kept pair satisfies the alpha
    condition in selection order."""
    rng = np.random.default_rng(seed)
    pts = rng.integers(-20, 21, size=(60, 3)).astype(np.float32)
    for _ in range(40):
        p = int(rng.integers(0, 60))
        cand = rng.integers(0, 60, size=int(rng.integers(1, 50))).astype(
            np.uint32)
        R = int(rng.integers(1, 12))
        out = oracle.robust_prune(pts, p, cand, 1.5, R)
        assert _prune_reference_ok(pts, p, cand, out, 9, 4, R)


def test_connect_adds_the_in_edge_the_repair_rule_names():
    """Connectivity repair (NSG's device, a reading stated with the graph
    build): points on a line 0..3 and 10, s = 0, R = 2; node 4 has no
    in-edge.  The greedy search toward x4 = (10, 0) from 0 expands 0, 1, 2,
    3; by distance to x4 they are 3, 2, 1, 0.  Node 3 has a free slot, so
    the repair adds 3 -> 4.  With 3, 2 and 1 full, the nearest expanded
    node with a free slot is 0: 0 -> 4."""
    pts = np.array([[0, 0], [1, 0], [2, 0], [3, 0], [10, 0]], np.float32)
    N = NONE
    adj = np.array([[1, N], [0, 2], [1, 3], [2, N], [3, N]], np.uint32)
    assert oracle.reachable(adj, 0) == 4
    assert oracle.connect(pts, adj, 0, 8) == 1
    assert adj[3].tolist() == [2, 4]
    assert oracle.reachable(adj, 0) == 5
    adj = np.array([[1, N], [0, 2], [1, 3], [2, 1], [3, N]], np.uint32)
    assert oracle.connect(pts, adj, 0, 8) == 1
    assert adj[0].tolist() == [1, 4]
    assert adj[1:4].tolist() == [[0, 2], [1, 3], [2, 1]]
    assert oracle.reachable(adj, 0) == 5


def test_fold_levels_puts_coarse_neighbours_first():
    """Coarse levels folded into one graph (the navigability reading of the
    graph build): a point's coarse neighbours come first, the highest level
    first, then its base list; repeats and self ids are dropped and the row
    is cut to R."""
    from oracle.graph import fold_levels
    N = NONE
    adj0 = np.array([[1, 2, 3], [0, 2, N], [0, 1, N], [0, 2, N],
                     [3, N, N]], np.uint32)
    # level 1 over points {0, 3, 4}: local ids 0, 1, 2
    lvl1 = (np.array([0, 3, 4], np.uint32),
            np.array([[2, N], [2, 0], [0, 1]], np.uint32))
    # level 2 over points {0, 4}
    lvl2 = (np.array([0, 4], np.uint32), np.array([[1], [0]], np.uint32))
    adj = fold_levels(adj0, [lvl1, lvl2])
    assert adj[0].tolist() == [4, 1, 2]        # 4 (l2), 4 (l1, repeat), base
    assert adj[3].tolist() == [4, 0, 2]        # l1: 4, 0; base 0 (repeat), 2
    assert adj[4].tolist() == [0, 3, N]        # l2: 0; l1: 0, 3; base 3
    assert adj[1].tolist() == adj0[1].tolist()  # in no coarse level


def test_plain_vamana_degree_bound_and_prune_rule():
    """Vamana: out-degree at most R, no self loops, no duplicate ids; every
    list the build returns is one RobustPrune can produce: its entries
    satisfy the alpha condition pairwise in (distance, id) order, checked
    in exact arithmetic on integer points (alpha = 1.5)."""
    w = synth.small("f32", n=800, d=16, nq=2, seed_index=105)
    base, _ = synth.base_and_queries(w)
    s = oracle.medoid(base)
    perm = np.random.default_rng(1).permutation(w.n).astype(np.uint32)
    adj = oracle.vamana_build(base, 12, 24, 1.2, perm, s)
    deg = (adj != NONE).sum(1)
    assert deg.max() <= 12 and deg.mean() > 4
    assert not (adj == np.arange(w.n, dtype=np.uint32)[:, None]).any()
    # determinism across thread counts
    adj1 = oracle.vamana_build(base, 12, 24, 1.2, perm, s, nthreads=1)
    assert np.array_equal(adj, adj1)


def _vamana_reference(X, R, Lb, alphas, perm, s, cap):
    """The Vamana build as the graph reading states it, written plainly
    for tiny inputs, one insertion at a time: greedy search from s toward
    p (worklist of Lb, expanded nodes in order), RobustPrune of those plus
    p's current list, back-edges appended while a list holds at most cap
    ids (else that list is pruned), per pass; finally every list longer
    than R is pruned with the last alpha.  Exact integer arithmetic; alpha
    is given as alpha^2 = (num, den)."""
    X = X.astype(np.int64)
    n = len(X)

    def d2(a, b):
        return int(((X[a] - X[b]) ** 2).sum())

    def prune(p, cand, a2):
        order = sorted({c for c in cand if c != p}, key=lambda c: (d2(p, c), c))
        kept = []
        for x in order:
            if len(kept) == R:
                break
            if all(a2[0] * d2(y, x) > a2[1] * d2(p, x) for y in kept):
                kept.append(x)
        return kept

    def greedy(p, nbr):
        L = [(d2(s, p), s, False)]
        seen = {s}
        V = []
        while True:
            i = next((i for i, e in enumerate(L) if not e[2]), None)
            if i is None or len(V) == 4 * Lb + 64:
                return V
            dist, u, _ = L[i]
            L[i] = (dist, u, True)
            V.append(u)
            for x in nbr[u]:
                if x not in seen:
                    seen.add(x)
                    L.append((d2(x, p), x, False))
            L = sorted(L, key=lambda e: (e[0], e[1]))[:Lb]

    nbr = [[] for _ in range(n)]
    for a2 in alphas:
        for p in perm:
            p = int(p)
            new = prune(p, greedy(p, nbr) + nbr[p], a2)
            nbr[p] = new
            for j in new:
                lst = nbr[j] + ([p] if p not in nbr[j] and p != j else [])
                nbr[j] = lst if len(lst) <= cap else prune(j, lst, a2)
    for j in range(n):
        if len(nbr[j]) > R:
            nbr[j] = prune(j, nbr[j], alphas[-1])
    return nbr


def test_vamana_build_equals_plain_reference():
    """The oracle's Vamana build (one insertion per batch) equals a plain
    re-statement of the build on 40 integer points in the plane: two
    passes with alpha = 1 and alpha = 1.5, R = 4, L_build = 6, back-edge
    slack 1.3 (lists of up to 5 before a prune), so appends, overflow
    prunes and the final prune all occur."""
    rng = np.random.default_rng(11)
    X = rng.integers(-25, 26, size=(40, 2)).astype(np.float32)
    s = oracle.medoid(X)
    perm = rng.permutation(40).astype(np.uint32)
    adj = oracle.vamana_build(X, 4, 6, 1.5, perm, s, slack=1.3,
                              max_batch_frac=0.0)
    ref = _vamana_reference(X, 4, 6, [(1, 1), (9, 4)], perm, s, 5)
    got = [[int(x) for x in row if x != NONE] for row in adj]
    assert got == ref


# --------------------------------------------------------------------------
# Precision form: reduced-precision table storage
# --------------------------------------------------------------------------
def test_f16_conversion_matches_numpy_round_to_nearest_even():
    """The oracle's FP32 -> half conversion is IEEE round-to-nearest-even,
    as numpy's float16 cast is: checked on random values, exact ties, the
    subnormal range and the top of the finite range."""
    rng = np.random.default_rng(1)
    v = np.concatenate([
        rng.uniform(0, 65504, 20000), rng.uniform(0, 1, 5000),
        rng.uniform(0, 2 ** -14, 5000),                 # subnormal halves
        np.float32(1 + np.arange(64) * 2 ** -11 + 2 ** -12),  # exact ties
        [0.0, 65504.0, 65519.0, 2 ** -24, 2 ** -25, 3 * 2 ** -26]]
    ).astype(np.float32)
    L = oracle.lib()
    got = np.array([L.or_f32_to_f16(float(x)) for x in v], dtype=np.uint16)
    assert np.array_equal(got, v.astype(np.float16).view(np.uint16))
    back = np.array([L.or_f16_to_f32(int(h)) for h in got], dtype=np.float32)
    assert np.array_equal(back, got.view(np.float16).astype(np.float32))


def _u8_tables(w):
    ix, q, _ = w
    T = oracle.pq_tables(q, ix.codebooks)
    return ix, q, T


def test_f16_table_error_bound(small_u8):
    """Half storage with a power-of-two scale: each entry is the FP32 entry
    times 2^-k rounded to half, so its relative error is at most 2^-11
    (plus the FP32 entry's own rounding), and the largest entry fits."""
    ix, q, T = _u8_tables(small_u8)
    H = oracle.quantize_tables(T, "f16").view(np.float16).astype(np.float64)
    for a in range(len(q)):
        mx = T[a].max()
        k = 0
        while mx * 2.0 ** -k > 65504:
            k += 1
        assert np.isfinite(H[a]).all()
        np.testing.assert_allclose(H[a] * 2.0 ** k, T[a], rtol=2 ** -11,
                                   atol=2.0 ** (k - 24))


def test_u8_table_error_bound_and_range(small_u8):
    """u8 storage: each subspace's minimum maps to 0, the widest subspace
    spans 0..255, and lo_j + code / inv is within half a step (plus FP32
    rounding) of the FP32 entry."""
    ix, q, T = _u8_tables(small_u8)
    U = oracle.quantize_tables(T, "u8").astype(np.float64)
    for a in range(len(q)):
        t = T[a].astype(np.float64)
        lo = t.min(1, keepdims=True)
        R = (T[a].max(1) - T[a].min(1)).max()
        step = R / 255.0
        assert (U[a].min(1) == 0).all() and U[a].max() == 255
        err = np.abs(lo + U[a] * step - t)
        assert err.max() <= 0.5 * step * (1 + 1e-5) + 1e-6 * t.max()


@pytest.mark.parametrize("table", ["f16", "u8"])
@pytest.mark.parametrize("fx", ["small_f32", "small_u8"])
def test_precision_form_L_at_least_n_is_brute_force(fx, table, request):
    """Whatever the table storage, t >= n on a connected graph expands every
    node, so the exact re-rank returns the brute-force k nearest."""
    ix, q, _ = request.getfixturevalue(fx)
    out = oracle.search(ix, q[:4], 10, ix.n, c_max=ix.n, iter_cap=ix.n + 1,
                        table=table)
    assert (out["iters"] == ix.n).all()
    allid = np.arange(ix.n)
    for a in range(4):
        ex = exact_sq(ix.base, q[a])
        assert out["ids"][a].tolist() == np.lexsort((allid, ex))[:10].tolist()


@pytest.mark.parametrize("table", ["f16", "u8"])
def test_precision_form_algorithm1_equals_filtered_form(small_u8, table):
    ix, q, _ = small_u8
    a = oracle.search(ix, q, 10, 33, mode=0, table=table, want_cand=True)
    b = oracle.search(ix, q, 10, 33, mode=1, table=table, want_cand=True)
    for key in ("ids", "dists", "cand", "iters"):
        assert np.array_equal(a[key], b[key]), key


def test_precision_form_ranks_by_quantised_adc(small_u8):
    """The PQ answer of Algorithm 1 under u8 storage is ordered by the
    integer sum of the quantised entries (ties by id)."""
    ix, q, _ = small_u8
    T = oracle.pq_tables(q, ix.codebooks)
    U = oracle.quantize_tables(T, "u8").astype(np.int64)
    out = oracle.search(ix, q, 10, 32, table="u8", want_pq=True)
    for a in range(len(q)):
        ids = out["pq_ids"][a]
        s = U[a][np.arange(ix.m)[None, :], ix.codes[ids]].sum(1)
        assert np.array_equal(out["pq_dists"][a], s.astype(np.float32))
        keys = list(zip(s.tolist(), ids.tolist()))
        assert keys == sorted(keys)


# --------------------------------------------------------------------------
# Exact-distance Version (section "Implementation Variants"): no table, the
# search ranks by exact distances, no re-rank
# --------------------------------------------------------------------------
@pytest.mark.parametrize("fx", ["small_f32", "small_u8", "small_i8"])
def test_exact_distance_L_at_least_n_is_brute_force(fx, request):
    """t >= n on a connected graph expands every node and evicts none, so
    the worklist ends holding every node in exact-distance order: its k
    first entries are the brute-force k nearest."""
    ix, q, _ = request.getfixturevalue(fx)
    out = oracle.search(ix, q[:6], 10, ix.n, iter_cap=ix.n + 1,
                        table="exact")
    assert (out["iters"] == ix.n).all() and (out["status"] == 0).all()
    allid = np.arange(ix.n)
    for a in range(6):
        ex = exact_sq(ix.base, q[a])
        order = np.lexsort((allid, ex))[:10]
        assert out["ids"][a].tolist() == order.tolist()
        if ix.base.dtype == np.float32:
            np.testing.assert_allclose(out["dists"][a], ex[order], rtol=2e-6)
        else:
            assert np.array_equal(out["dists"][a],
                                  ex[order].astype(np.float32))


@pytest.mark.parametrize("fx", ["small_f32", "small_u8", "small_i8"])
@pytest.mark.parametrize("L", [10, 33, 64])
def test_exact_distance_answer_needs_no_rerank(fx, L, request):
    """Without a re-rank the answer is the worklist's k first entries; a
    node expanded but no longer in the worklist was evicted at or above its
    last key, so these are also the k nearest expanded nodes by exact
    distance, which is what a re-rank of the expanded nodes would return.
    The distances are the exact squared distances of the ids."""
    ix, q, _ = request.getfixturevalue(fx)
    out = oracle.search(ix, q, 10, L, table="exact", want_cand=True)
    rr_ids, rr_d = oracle.rerank(ix, q, out["cand"], 10)
    assert np.array_equal(out["ids"], rr_ids)
    assert np.array_equal(out["dists"], rr_d)
    for a in range(len(q)):
        ex = exact_sq(ix.base, q[a])[out["ids"][a].astype(np.int64)]
        if ix.base.dtype == np.float32:
            np.testing.assert_allclose(out["dists"][a], ex, rtol=2e-6)
        else:
            assert np.array_equal(out["dists"][a], ex.astype(np.float32))
        keys = list(zip(out["dists"][a].tolist(), out["ids"][a].tolist()))
        assert keys == sorted(keys)


@pytest.mark.parametrize("L", [10, 33])
def test_exact_distance_algorithm1_equals_filtered_form(small_u8, L):
    ix, q, _ = small_u8
    a = oracle.search(ix, q, 10, L, mode=0, table="exact", want_cand=True)
    b = oracle.search(ix, q, 10, L, mode=1, table="exact", want_cand=True)
    for key in ("ids", "dists", "cand", "iters"):
        assert np.array_equal(a[key], b[key]), key


def test_exact_distance_beats_pq_recall(small_u8):
    """Exact distances remove the PQ error the re-rank compensates for: at
    the same t the exact-distance search finds at least as many true
    neighbours on average."""
    ix, q, _ = small_u8
    gt = np.stack([np.lexsort((np.arange(ix.n), exact_sq(ix.base, x)))[:10]
                   for x in q])
    def recall(ids):
        return np.mean([len(set(a) & set(b)) for a, b in zip(ids, gt)]) / 10
    ex = oracle.search(ix, q, 10, 16, table="exact")
    pq = oracle.search(ix, q, 10, 16)
    assert recall(ex["ids"]) >= recall(pq["ids"])


# --------------------------------------------------------------------------
# The paper's Bloom filter (section "Parallel Filtering of Visited
# Neighbours"; z and the hash family in section "Algorithm Parameters")
# --------------------------------------------------------------------------
def test_fnv1a32_published_check_values():
    """FNV-1a-32 reference values of the FNV specification: the empty
    string is the offset basis, "a" and "foobar" are its test vectors."""
    assert oracle.fnv1a32(b"") == 0x811C9DC5
    assert oracle.fnv1a32(b"a") == 0xE40C292C
    assert oracle.fnv1a32(b"foobar") == 0xBF9CF968


def test_bloom_slots_are_the_hashes_of_the_id_bytes_mod_z():
    """The two entries of a node are FNV-1a-32 of its four little-endian
    bytes under the two offset bases, mod z (the reading in oracle.c)."""
    for x in (0, 1, 255, 256, 65537, 999_999, 0xFFFFFFFE):
        b = int(x).to_bytes(4, "little")
        h1, h2 = oracle.bloom_slots(x)
        assert h1 == oracle.fnv1a32(b, 0x811C9DC5) % oracle.BLOOM_Z
        assert h2 == oracle.fnv1a32(b, 0x811C9DC5 ^ 0xA5A5A5A5) % oracle.BLOOM_Z
        assert 0 <= h1 < oracle.BLOOM_Z and 0 <= h2 < oracle.BLOOM_Z


def test_bloom_false_positive_rate_matches_closed_form():
    """A two-hash Bloom filter of z entries holding n keys answers a fresh
    key positively with probability (1 - e^(-2n/z))^2 when the hashes
    spread evenly; at n = 9,600 that is 0.22%.  Checked within 5 sigma
    on 120,000 fresh ids."""
    rng = np.random.default_rng(11)
    ids = rng.choice(1 << 24, 9600 + 120_000, replace=False)
    ins, fresh = ids[:9600], ids[9600:]
    setb = set()
    for x in ins:
        setb.update(oracle.bloom_slots(int(x)))
    fp = sum(all(h in setb for h in oracle.bloom_slots(int(x))) for x in fresh)
    p = (1 - np.exp(-2 * 9600 / oracle.BLOOM_Z)) ** 2
    mu, sd = p * len(fresh), np.sqrt(p * (1 - p) * len(fresh))
    assert abs(fp - mu) < 5 * sd, (fp, mu, sd)


def _nodes_at_risk(n):
    """Nodes both of whose entries are also entries of other nodes: the
    only ones a Bloom filter over this graph can wrongly drop."""
    from collections import Counter
    sl = [oracle.bloom_slots(x) for x in range(n)]
    cnt = Counter(h for s in sl for h in set(s))
    return [x for x, s in enumerate(sl) if all(cnt[h] > 1 for h in set(s))]


@pytest.mark.parametrize("fx", ["small_f32", "small_u8"])
@pytest.mark.parametrize("L", [10, 33, 64])
def test_bloom_search_equals_exact_seen_set_without_collisions(fx, L,
                                                              request):
    """A Bloom filter has no false negatives, so where no node can be a
    false positive (no node's two entries are both shared with other
    nodes) Algorithm 2 with the Bloom filter is Algorithm 2 with an exact
    seen-set: same expansions, same answer."""
    ix, q, _ = request.getfixturevalue(fx)
    assert _nodes_at_risk(ix.n) == []
    a = oracle.search(ix, q, 10, L, mode=1, want_pq=True, want_cand=True)
    b = oracle.search(ix, q, 10, L, mode=2, want_pq=True, want_cand=True)
    for key in ("ids", "dists", "pq_ids", "pq_dists", "cand", "iters",
                "added"):
        assert np.array_equal(a[key], b[key]), key


def _collision_graph(row):
    """Medoid s = 12446 with the given adjacency row; every other row
    empty.  Node 11616's first entry is one of s's and its second one of
    node 12330's (found by search over the hash values)."""
    s, a, y = 12446, 12330, 11616
    hs, ha, hy = (oracle.bloom_slots(v) for v in (s, a, y))
    assert hy[0] in hs and hy[1] in ha
    assert hy[1] not in hs and hy[0] not in ha
    n, R = s + 1, 2
    rng = np.random.default_rng(5)
    base = rng.random((n, 4), dtype=np.float32)
    adj = np.full((n, R), NONE, dtype=np.uint32)
    adj[s, :len(row)] = row
    cb = rng.random((1, 256, 4), dtype=np.float32)
    codes = rng.integers(0, 256, (n, 1), dtype=np.uint8)
    return oracle.Index(base, adj, s, cb, codes), base[:1].copy(), s, a, y


def test_bloom_false_positive_depends_on_row_order():
    """Algorithm 2 tests and then sets each neighbour's entries; read with
    sequential in-row semantics, a neighbour sees the entries set by the
    ones before it.  Row [a, y] under s: y's entries were set by s (at the
    start) and by a (just before), so y counts as visited and is dropped,
    a false positive.  Row [y, a]: y is tested before a sets its entry, so
    it is kept.  The exact seen-set keeps y either way."""
    ix, q, s, a, y = _collision_graph([12330, 11616])
    exact = oracle.search(ix, q, 1, 8, mode=1, want_cand=True)
    bloom = oracle.search(ix, q, 1, 8, mode=2, want_cand=True)
    assert sorted(exact["cand"][0][:exact["iters"][0]].tolist()) == sorted(
        [s, a, y])
    assert bloom["cand"][0][:bloom["iters"][0]].tolist() == [s, a]
    ix2, q2, *_ = _collision_graph([11616, 12330])
    bloom2 = oracle.search(ix2, q2, 1, 8, mode=2, want_cand=True)
    assert sorted(bloom2["cand"][0][:bloom2["iters"][0]].tolist()) == sorted(
        [s, a, y])


# --------------------------------------------------------------------------
# the precision form's BF16 re-rank with an FP32 recheck (float data)
# --------------------------------------------------------------------------
def test_bf16_round_hand_worked_values():
    """bfloat16 keeps 8 significant bits: near 1 the step is 2^-7, and a
    value halfway between two neighbours goes to the one whose last
    significand bit is 0."""
    r = oracle.bf16_round
    assert r(1.0) == 1.0
    assert r(1 + 2 ** -8) == 1.0                    # tie, 1.0 is even
    assert r(1 + 3 * 2 ** -8) == 1 + 2 ** -6        # tie, 1+2^-6 is even
    assert r(1 + 2 ** -8 + 2 ** -20) == 1 + 2 ** -7  # just above the tie
    assert r(1 + 2 ** -8 - 2 ** -20) == 1.0          # just below
    assert r(-(1 + 2 ** -8 + 2 ** -20)) == -(1 + 2 ** -7)
    assert r(float(np.float32(np.pi))) == 3.140625
    assert r(0.0) == 0.0 and r(256.0) == 256.0 and r(257.0) == 256.0
    assert r(259.0) == 260.0                         # step 2 at 256..512
    assert r(1000.001) == 1000.0                      # step 4 at 512..1024


def _fp32_dists(ix, q, ids):
    """Canonical FP32 distances of ids, in the order given."""
    got_ids, got_d = oracle.rerank(ix, q[None, :],
                                   np.asarray(ids, np.uint32)[None, :],
                                   len(ids))
    order = {int(i): float(dv) for i, dv in zip(got_ids[0], got_d[0])}
    return np.array([order[int(i)] for i in ids], dtype=np.float64)


@pytest.mark.parametrize("scale,d", [(1.0, 96), (1e-3, 128), (1e3, 96),
                                     (1.0, 1024)])
def test_bf16_band_contains_fp32_and_exact_distances(scale, d):
    """For random rows and queries at several magnitudes, and rows that
    nearly equal the query (where the BF16 rounding of a large coordinate
    is larger than the whole distance), both the canonical FP32 distance
    and the exact FP64 one lie inside [lower, upper]; for ordinary rows
    the band is a small fraction of the distance."""
    rng = np.random.default_rng(int(d + scale * 7))
    n = 400
    base = (rng.standard_normal((n, d)) * scale).astype(np.float32)
    q = (rng.standard_normal(d) * scale).astype(np.float32)
    base[:40] = (q + rng.standard_normal((40, d)).astype(np.float32)
                 * np.float32(scale * 1e-4))
    base[40:60] = q + np.float32(1000.0 * scale)
    base[60:70] = q
    adj = np.full((n, 4), 0xFFFFFFFF, dtype=np.uint32)
    ix = oracle.Index(base, adj, 0, np.zeros((1, 256, d), np.float32),
                      np.zeros((n, 1), np.uint8))
    ids = np.arange(n, dtype=np.uint32)
    dt, lo, hi = oracle.bf16_band(ix, q, ids)
    f32 = _fp32_dists(ix, q, ids)
    exact = ((base.astype(np.float64) - q.astype(np.float64)) ** 2).sum(1)
    assert np.all(lo <= f32) and np.all(f32 <= hi)
    assert np.all(lo <= exact) and np.all(exact <= hi)
    assert np.all(lo >= 0)
    ordinary = slice(70, n)
    width = (hi[ordinary] - lo[ordinary]) / dt[ordinary]
    assert width.max() < 0.05


def test_bf16_rerank_equals_fp32_rerank_on_near_ties():
    """Candidates whose FP32 distances differ in the last bits, so that the
    BF16 sums alone order them differently: the recheck restores the FP32
    answer exactly (ids and distances), recomputing fewer candidates than
    it was given."""
    rng = np.random.default_rng(21)
    d, n, k = 96, 600, 10
    q = rng.standard_normal(d).astype(np.float32)
    base = rng.standard_normal((n, d)).astype(np.float32)
    # 30 near-copies of one row that differ by less than a BF16 step
    anchor = rng.standard_normal(d).astype(np.float32) * np.float32(0.3) + q
    base[:30] = anchor + (rng.standard_normal((30, d)) *
                          1e-4).astype(np.float32)
    adj = np.full((n, 4), 0xFFFFFFFF, dtype=np.uint32)
    ix = oracle.Index(base, adj, 0, np.zeros((1, 256, d), np.float32),
                      np.zeros((n, 1), np.uint8))
    cand = np.stack([rng.permutation(n).astype(np.uint32) for _ in range(6)])
    qs = np.tile(q, (6, 1))
    want_ids, want_d = oracle.rerank(ix, qs, cand, k)
    got_ids, got_d, rechecked = oracle.rerank_bf16(ix, qs, cand, k)
    assert np.array_equal(got_ids, want_ids)
    assert np.array_equal(got_d.view(np.uint32), want_d.view(np.uint32))
    assert (rechecked >= k).all() and (rechecked < n).all()
    # the BF16 sums alone order the near-copies differently from FP32: the
    # recheck is what makes the answers equal
    dt, _, _ = oracle.bf16_band(ix, q, np.arange(30, dtype=np.uint32))
    f32 = _fp32_dists(ix, q, np.arange(30, dtype=np.uint32))
    assert not np.array_equal(np.lexsort((np.arange(30), dt)),
                              np.lexsort((np.arange(30), f32)))


def test_bf16_rerank_with_k_candidates_or_fewer_rechecks_all():
    rng = np.random.default_rng(4)
    d, n = 32, 50
    base = rng.standard_normal((n, d)).astype(np.float32)
    q = rng.standard_normal((1, d)).astype(np.float32)
    adj = np.full((n, 4), 0xFFFFFFFF, dtype=np.uint32)
    ix = oracle.Index(base, adj, 0, np.zeros((1, 256, d), np.float32),
                      np.zeros((n, 1), np.uint8))
    cand = np.array([[3, 0xFFFFFFFF, 7, 11, 0xFFFFFFFF]], dtype=np.uint32)
    ids, dists, rc = oracle.rerank_bf16(ix, q, cand, 5)
    want_ids, want_d = oracle.rerank(ix, q, cand, 5)
    assert rc[0] == 3
    assert np.array_equal(ids, want_ids)
    assert np.array_equal(dists.view(np.uint32), want_d.view(np.uint32))


# --------------------------------------------------------------------------
# the precision form's BF16-MFMA table: FP64 terms and the error bound
# --------------------------------------------------------------------------
def test_bf16_round_array_hand_worked_and_equal_to_the_scalar_rounding():
    """Hand-worked bfloat16 roundings (8-bit significand, ties to even),
    and agreement with the oracle's scalar rounding on random floats and on
    exact midpoints."""
    x = np.array([1.0, 1 + 2 ** -8, 1 + 3 * 2 ** -8, 1 + 2 ** -8 + 2 ** -20,
                  255.0, 257.0, -3.0, 0.0])
    want = np.array([1.0, 1.0, 1 + 2 ** -6, 1 + 2 ** -7, 255.0, 256.0, -3.0,
                     0.0])
    assert np.array_equal(oracle.bf16_round_array(x), want)
    rng = np.random.default_rng(11)
    r = (rng.standard_normal(300) * 10.0 ** rng.integers(-3, 4, 300))
    r = r.astype(np.float32).astype(np.float64)
    mids = (1.0 + (2 * rng.integers(0, 128, 50) + 1) * 2.0 ** -8) * \
        2.0 ** rng.integers(-5, 6, 50)
    for v in np.concatenate([r, mids, -mids]):
        assert oracle.bf16_round_array(np.array([v]))[0] == \
            oracle.bf16_round(v), v


def test_pq_table_terms_closed_forms():
    """T is the table of the FP32 oracle up to FP32 rounding; with inputs
    that bfloat16 holds exactly (integers up to 256) the rounded inner
    product is exact, so T_b equals T."""
    rng = np.random.default_rng(12)
    q = rng.integers(0, 256, (5, 16)).astype(np.float32)
    cb = rng.integers(-256, 257, (4, 256, 4)).astype(np.float32)
    T, S_qc, S_qq, S_cc, Tb = oracle.pq_table_terms(q, cb)
    assert np.array_equal(Tb, T)
    T32 = oracle.pq_tables(q, cb).astype(np.float64)
    assert np.allclose(T32, T, rtol=0, atol=1e-6 * T.max())
    assert np.allclose(S_qq[:, :, 0], (q.reshape(5, 4, 4) ** 2).sum(-1))
    assert (S_qc <= np.sqrt(S_qq * S_cc) * (1 + 1e-12)).all()


@pytest.mark.parametrize("ds", [2, 4, 8])
def test_bf16_table_bound_contains_the_rounded_and_fp32_forms(ds):
    """The bound contains the error of the table with bf16-rounded inner
    products (exact arithmetic otherwise) and of FP32 evaluations of the
    formula in two summation orders, on float data of several magnitudes
    and on integer data; and it is not vacuous: on coordinates that round
    by nearly the most, the rounded table's error reaches a quarter of it."""
    rng = np.random.default_rng(13 + ds)
    m = 8
    for scale in (1e-2, 1.0, 300.0):
        q = (rng.standard_normal((6, m * ds)) * scale).astype(np.float32)
        cb = (rng.standard_normal((m, 256, ds)) * scale).astype(np.float32)
        T, E = oracle.bf16_table_bound(q, cb)
        _, _, S_qq, S_cc, Tb = oracle.pq_table_terms(q, cb)
        assert (np.abs(Tb - T) <= E).all()
        # FP32 evaluations: norms in order, inner product in order and in
        # reverse, then (|q|^2 + |c|^2) - 2X
        qb = oracle.bf16_round_array(q).astype(np.float32)
        cbb = oracle.bf16_round_array(cb).astype(np.float32)
        qs = q.reshape(6, m, 1, ds)
        qbs = qb.reshape(6, m, 1, ds)
        for order in (range(ds), reversed(range(ds))):
            X = np.zeros((6, m, 256), np.float32)
            for t in order:
                X = X + qbs[..., t] * cbb[None, :, :, t]
            nq_ = np.zeros((6, m, 1), np.float32)
            nc_ = np.zeros((1, m, 256), np.float32)
            for t in range(ds):
                nq_ = nq_ + qs[..., t] * qs[..., t]
                nc_ = nc_ + cb[None, :, :, t] * cb[None, :, :, t]
            T32 = (nq_ + nc_) - np.float32(2.0) * X
            assert (np.abs(T32.astype(np.float64) - T) <= E).all()
    # coordinates just below a bfloat16 midpoint, all of one sign: each
    # factor rounds down by almost u/2 relative, so the inner product errs
    # by close to u times S_qc
    q = np.full((1, m * ds), 1 + 2 ** -8 - 2 ** -20, np.float32)
    cb = np.full((m, 256, ds), 1 + 2 ** -8 - 2 ** -20, np.float32)
    T, E = oracle.bf16_table_bound(q, cb)
    _, _, _, _, Tb = oracle.pq_table_terms(q, cb)
    assert (np.abs(Tb - T) <= E).all()
    assert (np.abs(Tb - T) >= 0.25 * E).all()
