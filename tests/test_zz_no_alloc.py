"""The search entry point that allocates nothing (bang_search_noalloc),
against bang_search on the same inputs, two calls in a row, the second with
a smaller batch: ids and distances bit for bit."""
import numpy as np
import pytest

import oracle
import synth
from oracle.graph import build_graph
from oracle.pq import pq_encode, train_pq

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _index(w):
    rs = synth.streams(w)
    base, q = synth.base_and_queries(w)
    cb = train_pq(base, w.m, w.kmeans_iters, rs["pq_init"])
    codes = pq_encode(base, cb)
    s = oracle.medoid(base)
    perm = rs["vamana_order"].permutation(w.n).astype(np.uint32)
    adj, _ = build_graph(base, w.R, w.L_build, w.alpha, perm, s)
    return base, adj, s, cb, codes, q


@pytest.fixture(scope="module")
def index():
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a visible GPU")
    import paper_2401_11324_amd as bang
    w = synth.small("u8", n=3000, d=128, nq=300, m=32, R=64, ncent=12,
                    seed_index=130)
    base, adj, s, cb, codes, q = _index(w)
    gi = bang.Index(base, adj, s, cb, codes)
    yield gi, q
    gi.close()


def _pair(gi, qt, k, L, table):
    nq = qt.shape[0]
    ids = torch.empty((nq, k), dtype=torch.int32, device="cuda")
    dist = torch.empty((nq, k), dtype=torch.float32, device="cuda")
    gi.search_noalloc(qt, k, L, out=(ids, dist), table=table)
    rid, rd = gi.search(qt, k, L, table=table)
    torch.cuda.synchronize()
    return (ids.cpu().numpy(), dist.cpu().numpy().view(np.uint32),
            rid.cpu().numpy(), rd.cpu().numpy().view(np.uint32))


@pytest.mark.parametrize("k,L,table", [(10, 64, "f32"), (10, 768, "f32"),
                                       (10, 256, "u8"), (10, 100, "exact"),
                                       (100, 1024, "f16")])
def test_noalloc_search_equals_search_twice(index, k, L, table):
    gi, q = index
    qt = torch.from_numpy(q).cuda()
    for nq in (len(q), 37):  # the second call with a smaller batch
        a, ad, b, bd = _pair(gi, qt[:nq].contiguous(), k, L, table)
        assert np.array_equal(a, b), (nq, k, L, table)
        assert np.array_equal(ad, bd), (nq, k, L, table)


def test_noalloc_search_rejects_filters_that_need_memory(index):
    import paper_2401_11324_amd as bang
    gi, q = index
    qt = torch.from_numpy(q[:4]).cuda()
    ids = torch.empty((4, 10), dtype=torch.int32, device="cuda")
    dist = torch.empty((4, 10), dtype=torch.float32, device="cuda")
    with pytest.raises(bang.BangError):
        gi.search(qt, 10, 64, out=(ids, dist), filter="bloom",
                  _entry="bang_search_noalloc")
