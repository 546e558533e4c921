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


def test_algorithmic_bytes_counts_rows_codes_and_rerank():
    deg = np.array([3, 2, 1, 0])
    cand = np.array([[0, 1, 0xFFFFFFFF], [2, 0xFFFFFFFF, 0xFFFFFFFF]],
                    dtype=np.uint32)
    iters = np.array([2, 1])
    R, m, d, elem, k = 4, 8, 16, 1, 2
    got = bench.algorithmic_bytes(deg, R, m, d, elem, k, iters, cand, c_max=1)
    want = (3 * 4 * R                 # three expansions, one row each
            + (3 + 2 + 1) * m         # codes of every neighbour
            + 2 * d * elem            # two queries
            + (1 + 1) * d * elem      # re-ranked rows, capped at c_max=1
            + 2 * 8 * k)              # results
    assert got == want


def test_algorithmic_bytes_exact_distance_reads_base_rows_and_no_rerank():
    deg = np.array([3, 2, 1, 0])
    cand = np.array([[0, 1, 0xFFFFFFFF], [2, 0xFFFFFFFF, 0xFFFFFFFF]],
                    dtype=np.uint32)
    iters = np.array([2, 1])
    R, m, d, elem, k = 4, 8, 16, 1, 2
    got = bench.algorithmic_bytes(deg, R, m, d, elem, k, iters, cand, c_max=1,
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
