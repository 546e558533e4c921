"""The benchmark's measurement formulas, pinned to the paper where it
prints values (CPU only)."""
import numpy as np

import bench


def test_iteration_overhead_matches_table5(golden):
    """Table 5 prints t, I and lambda = (I - t) / t * 100 to one decimal."""
    for row in golden("table5.json")["rows"]:
        lam = bench.iteration_overhead(row["I"], row["t"])
        assert round(lam, 1) == row["lambda"]


def test_recall_at_k_definition():
    """k-recall@k = |S ∩ S~| / k ("Algorithm Parameters")."""
    gt = np.array([[1, 2, 3, 4], [5, 6, 7, 8]])
    ids = np.array([[4, 3, 9, 9], [5, 6, 7, 8]])
    assert bench.recall_at_k(ids, gt, 4) == (2 / 4 + 1) / 2
    assert bench.recall_at_k(ids, gt, 2) == (0 + 1) / 2


def test_packed_row_bytes_count_rows_codes_and_rerank():
    deg = np.array([3, 2, 1, 0])
    cand = np.array([[0, 1, 0xFFFFFFFF], [2, 0xFFFFFFFF, 0xFFFFFFFF]],
                    dtype=np.uint32)
    iters = np.array([2, 1])
    R, m, d, elem, k = 4, 8, 16, 1, 2
    got = bench.packed_row_bytes(deg, R, m, d, elem, k, iters, cand, c_max=1)
    want = (3 * 4 * R                 # three expansions, one row each
            + (3 + 2 + 1) * m         # codes of every neighbour
            + 2 * d * elem            # two queries
            + (1 + 1) * d * elem      # re-ranked rows, capped at c_max=1
            + 2 * 8 * k)              # results
    assert got == want


def test_packed_row_bytes_exact_distance_read_base_rows_and_no_rerank():
    deg = np.array([3, 2, 1, 0])
    cand = np.array([[0, 1, 0xFFFFFFFF], [2, 0xFFFFFFFF, 0xFFFFFFFF]],
                    dtype=np.uint32)
    iters = np.array([2, 1])
    R, m, d, elem, k = 4, 8, 16, 1, 2
    got = bench.packed_row_bytes(deg, R, m, d, elem, k, iters, cand, c_max=1,
                                  exact=True)
    want = (3 * 4 * R                 # three expansions, one row each
            + (3 + 2 + 1) * d * elem  # base row of every neighbour
            + 2 * d * elem            # two queries
            + 2 * 8 * k)              # results; no re-rank
    assert got == want


def test_more_than_one_gpu_is_refused_with_a_message(capsys):
    """This build runs on one GPU: --gpus N > 1 exits with status 2 and
    says so, before touching any device."""
    rc = bench.main(["--gpus", "2", "--no-sweep", "--L", "64"])
    assert rc == 2
    assert "one GPU" in capsys.readouterr().err


def test_no_sweep_needs_L():
    import pytest
    with pytest.raises(SystemExit):
        bench.main(["--no-sweep"])


def test_unseen_neighbours_equals_a_sequential_seen_set():
    """The sum of |N'| over a query's expansions, against Algorithm 2's
    exact filter run step by step (seen = {s}; each row's unseen ids are
    counted and added)."""
    rng = np.random.default_rng(5)
    n, R = 50, 6
    adj = np.full((n, R), 0xFFFFFFFF, dtype=np.uint32)
    for u in range(n):
        deg = rng.integers(0, R + 1)
        adj[u, :deg] = rng.choice(np.delete(np.arange(n), u), deg,
                                  replace=False)
    s = 7
    iters = np.array([12, 0, 30, 5])
    cand = np.full((4, 40), 0xFFFFFFFF, dtype=np.uint32)
    for q, it in enumerate(iters):
        cand[q, :it] = rng.integers(0, n, it)
    want = []
    for q, it in enumerate(iters):
        seen, tot = {s}, 0
        for u in cand[q, :it]:
            new = [x for x in adj[u] if x != 0xFFFFFFFF and x not in seen]
            tot += len(new)
            seen.update(new)
        want.append(tot)
    got = bench.unseen_neighbours(adj, s, iters, cand)
    assert got.tolist() == want


def test_method_bytes_follow_the_per_expansion_formula():
    nprime = np.array([5, 0, 7])
    iters = np.array([4, 1, 9])
    R, m, d, elem, k = 8, 16, 32, 1, 3
    tot, parts = bench.method_bytes(nprime, R, m, d, elem, k, iters, c_max=6)
    assert parts == {"adjacency": 14 * 4 * R, "visited_probes": 14 * 8 * R,
                     "codes_unseen": 12 * m,
                     "rerank_rows": (4 + 1 + 6) * d * elem,
                     "queries_and_results": 3 * (d * elem + 8 * k)}
    assert tot == sum(parts.values())
    tot, parts = bench.method_bytes(nprime, R, m, d, elem, k, iters, c_max=6,
                                    exact=True)
    assert parts["base_rows_unseen"] == 12 * d * elem
    assert parts["rerank_rows"] == 0


def test_form_adc_definitions():
    """FP32: the sequential FP32 sum; F16 and U8 dequantised values stay
    within their rounding bounds of the FP32 value (half: relative 2^-11
    per entry plus the FP32 sums; u8: half a step per subspace)."""
    rng = np.random.default_rng(3)
    m = 8
    T = (rng.random((m, 256)) * 1000).astype(np.float32)
    codes = rng.integers(0, 256, (40, m))
    f = bench.form_adc(T, codes, "f32")
    acc = np.zeros(40, dtype=np.float32)
    for j in range(m):
        acc = acc + T[j, codes[:, j]]
    assert np.array_equal(f, acc.astype(np.float64))
    exact = T.astype(np.float64)[np.arange(m)[None, :], codes].sum(1)
    h = bench.form_adc(T, codes, "f16")
    assert np.all(np.abs(h - exact) <= exact * (2.0 ** -11 + 1e-6))
    u = bench.form_adc(T, codes, "u8")
    step = (T.max(1) - T.min(1)).max() / 255.0
    assert np.all(np.abs(u - exact) <= m * 0.5 * step * (1 + 1e-5) + 1e-3)
    # large entries take a power-of-two scale before rounding to half
    T2 = T * np.float32(1000.0)
    h2 = bench.form_adc(T2, codes, "f16")
    ex2 = T2.astype(np.float64)[np.arange(m)[None, :], codes].sum(1)
    assert np.all(np.abs(h2 - ex2) <= ex2 * (2.0 ** -11 + 1e-6))
