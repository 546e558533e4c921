"""Host-side pieces (no GPU): the seeded serving request stream, the
autotuner's choice rule, the launch autotuner's take orders, and the packed
adjacency storage of the index files."""
import numpy as np
import pytest

import synth
from paper_2401_11324_amd import serving


def test_request_stream_is_seeded_and_well_formed():
    w = synth.WORKLOADS["sift1m"]
    a = synth.serving_requests(w, 1e5, 0.5, salt=3)
    b = synth.serving_requests(w, 1e5, 0.5, salt=3)
    for key in a:
        assert np.array_equal(a[key], b[key])
    c = synth.serving_requests(w, 1e5, 0.5, salt=4)
    assert not np.array_equal(a["arrival_s"], c["arrival_s"])
    assert (np.diff(a["arrival_s"]) >= 0).all()
    assert a["arrival_s"].max() < 0.5
    assert ((a["nq"] >= 1) & (a["nq"] <= 256)).all()
    assert set(a["k"].tolist()) <= {10, 100}
    assert (a["L"] >= a["k"]).all()
    assert set(a["L"].tolist()) <= {32, 64, 100, 128}
    assert len(a["rows"]) == a["nq"].sum() and a["rows"].max() < w.nq
    # the mean query rate is the offered one, within sampling noise
    rate = a["nq"].sum() / 0.5
    assert 0.7e5 < rate < 1.3e5


def test_autotune_choice_rule():
    t = [{"max_batch": 1, "slots": 1, "sustained_qps": 5.0, "p99_ms": 10.0},
         {"max_batch": 2, "slots": 1, "sustained_qps": 9.0, "p99_ms": 60.0},
         {"max_batch": 3, "slots": 2, "sustained_qps": 7.0, "p99_ms": 40.0}]
    assert serving.choose(t, 50.0)["max_batch"] == 3   # fastest within target
    assert serving.choose(t, 5.0)["max_batch"] == 1    # none: lowest p99


def test_autotune_prefers_lower_p99_when_rates_tie():
    t = [{"max_batch": 1, "slots": 1, "sustained_qps": 100.0, "p99_ms": 9.0},
         {"max_batch": 2, "slots": 2, "sustained_qps": 99.5, "p99_ms": 3.0},
         {"max_batch": 3, "slots": 2, "sustained_qps": 90.0, "p99_ms": 1.0}]
    assert serving.choose(t, 50.0)["max_batch"] == 2


def test_packed_adjacency_roundtrip():
    from synth import store
    rng = np.random.default_rng(5)
    for n, R in ((1, 3), (1000, 7), (1_000_000, 64), (5, 64)):
        a = rng.integers(0, n, size=(min(n, 500), R)).astype(np.uint32)
        a[rng.random(a.shape) < 0.1] = 0xFFFFFFFF
        words, wbits = store.pack_ids(a, n)
        assert wbits == n.bit_length()
        assert words.nbytes <= (a.size * wbits + 63) // 64 * 8 + 64 * 8
        assert np.array_equal(store.unpack_ids(words, a.shape, n, wbits), a)


def test_extra_arrays_roundtrip_and_checks(tmp_path):
    """Arrays added beside an index (e.g. another PQ encoding) come back
    bit-identical, bad names are refused and a changed file is caught."""
    import pytest
    from synth import store
    w = synth.small("u8", n=300, d=16, nq=3, m=4, R=8, seed_index=150)
    rng = np.random.default_rng(7)
    arrays = {"codebooks": rng.random((4, 256, 4), dtype=np.float32),
              "codes": rng.integers(0, 256, (300, 4), dtype=np.uint8),
              "adj": rng.integers(0, 300, (300, 8)).astype(np.uint32),
              "gt_ids": np.zeros((3, 10), np.uint32),
              "gt_dists": np.zeros((3, 10), np.float64)}
    store.save(w, arrays, 0, root=str(tmp_path))
    extra = {"codes_m8": rng.integers(0, 256, (300, 8), dtype=np.uint8),
             "codebooks_m8": rng.random((8, 256, 2), dtype=np.float32)}
    store.save_extra(w, extra, root=str(tmp_path))
    assert store.extra_names(w, root=str(tmp_path)) == ["codebooks_m8",
                                                        "codes_m8"]
    got = store.load_extra(w, ["codes_m8", "codebooks_m8"],
                           root=str(tmp_path))
    for k, v in extra.items():
        assert got[k].dtype == v.dtype and np.array_equal(got[k], v)
    with pytest.raises(ValueError):
        store.save_extra(w, {"codes": extra["codes_m8"]}, root=str(tmp_path))
    with pytest.raises(KeyError):
        store.load_extra(w, ["codes_m99"], root=str(tmp_path))
    bad = extra["codes_m8"].copy()
    bad[0, 0] ^= 1
    np.save(tmp_path / w.name / "codes_m8.npy", bad, allow_pickle=False)
    with pytest.raises(ValueError):
        store.load_extra(w, ["codes_m8"], root=str(tmp_path))
    # the index itself is untouched by the extra arrays
    assert np.array_equal(store.load(w, root=str(tmp_path), with_base=False)
                          ["codes"], arrays["codes"])


def test_mixed_batch_recipe():
    """The 100M configuration's query mix: k uniform over {1, 10, 100},
    L = max(k, round(exp(U[ln 16, ln 256]))); seeded."""
    k, L = synth.mixed_batch(60_000, salt=3)
    k2, L2 = synth.mixed_batch(60_000, salt=3)
    assert np.array_equal(k, k2) and np.array_equal(L, L2)
    assert set(np.unique(k).tolist()) == {1, 10, 100}
    assert (L >= k).all() and L.min() >= 16 and L.max() <= 256
    # each k about a third; log L about uniform on [ln 16, ln 256]
    for v in (1, 10, 100):
        assert abs((k == v).mean() - 1 / 3) < 0.01
    lo = L[k < 16]  # not raised to k
    med = np.median(np.log(lo))
    assert abs(med - 0.5 * (np.log(16) + np.log(256))) < 0.05


def test_take_orders():
    """The launch autotuner's take orders: 'given' keeps the batch order,
    'longest_first' is a permutation with non-increasing L and the batch's
    order among equal L (stable); an unknown name is an error."""
    from paper_2401_11324_amd import tuning
    Lq = np.array([32, 256, 16, 256, 100, 32, 1024, 16])
    assert tuning.order_of("given", Lq) is None
    o = tuning.order_of("longest_first", Lq)
    assert o.dtype == np.int32
    assert sorted(o.tolist()) == list(range(len(Lq)))
    assert np.all(np.diff(Lq[o]) <= 0)
    assert o.tolist() == [6, 1, 3, 4, 0, 5, 2, 7]
    with pytest.raises(ValueError):
        tuning.order_of("shortest_first", Lq)
