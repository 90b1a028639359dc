"""GPU composite-index build (dense tiles + landing-zone selection + reverse
pass) and GPU exact hybrid k-NN against the CPU oracle, through the C ABI.

The oracle ranks candidates by the float64 key delta^2 (m + chi)^2 in direct
form; the GPU re-scores its dense-tile candidates the same way, so graphs
agree edge for edge on integer-valued vectors (every quantity exact) and, on
float vectors, wherever no two keys tie to float64 rounding."""
import numpy as np
import pytest
import torch

import oracle
import synth

pytestmark = pytest.mark.gpu

nhq = pytest.importorskip("paper_2203_13601_amd")


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def _build(w, **kw):
    ix = nhq.nhq_build_index(_dev(w.x), _dev(w.attrs), **kw)
    torch.cuda.synchronize()
    return ix, nhq.nhq_index_get_graph(ix).cpu().numpy()


@pytest.mark.parametrize("d,integer,R,l", [(128, True, 32, 64), (37, True, 16, 40),
                                           (96, False, 24, 48), (128, False, 32, 64)])
def test_graph_matches_oracle(d, integer, R, l):
    w = synth.small(3000, d, 1, seed=61 + d, integer=integer, n_centres=6)
    ix, adj = _build(w, degree=R, cand=l, n_entry=64, seed=1)
    want = oracle.build_graph(w.x, w.attrs, l=l, R=R)
    same = (adj == want).all(axis=1)
    assert same.mean() == 1.0, (same.mean(), np.nonzero(~same)[0][:5])


def test_reverse_pass_matches_oracle():
    w = synth.small(2500, 64, 1, seed=62, integer=True, n_centres=5)
    ix, adj = _build(w, degree=16, cand=32, reverse_edges=True, n_entry=64)
    want = oracle.build_graph(w.x, w.attrs, l=32, R=16, reverse=True)
    assert (adj == want).all()


def test_graph_rows_at_scale_sampled():
    # 200k integer points: every sampled row equals the oracle's row, which
    # the oracle computes on its own from the object set
    w = synth.small(200_000, 128, 1, seed=63, integer=True, n_centres=64)
    ix, adj = _build(w, degree=32, cand=64, n_entry=64)
    rows = np.random.default_rng(0).choice(w.n, 48, replace=False)
    want = oracle.build_graph(w.x, w.attrs, l=64, R=32, rows=rows)
    assert (adj[rows] == want).all()
    # structural checks on every row: no self loops, no repeats, -1 only at the tail
    assert not (adj == np.arange(w.n)[:, None]).any()
    valid = adj >= 0
    assert (np.diff(valid.astype(np.int8), axis=1) <= 0).all()
    s = np.sort(np.where(valid, adj, -np.arange(1, 33)[None, :]), axis=1)
    assert not (s[:, 1:] == s[:, :-1]).any()


@pytest.mark.parametrize("integer,wild", [(True, False), (False, False), (True, True)])
def test_bruteforce_knn_matches_oracle(integer, wild):
    w = synth.small(20000, 128 if integer else 96, 300, seed=64, integer=integer,
                    wildcard_arity=wild)
    ix = nhq.nhq_index_create(_dev(w.x), _dev(w.attrs), n_entry=16)
    for k in (1, 10, 100):
        ids, dist = nhq.nhq_bruteforce_hybrid_knn(ix, _dev(w.q), _dev(w.qattrs), k)
        gi, gd, _ = oracle.bruteforce(w.x, w.attrs, w.q, w.qattrs, k)
        ids = ids.cpu().numpy()
        dist = dist.cpu().numpy()
        assert np.array_equal(ids, gi)
        fin = np.isfinite(gd)
        assert np.array_equal(np.isfinite(dist), fin)
        assert np.allclose(dist[fin], gd[fin], rtol=1e-6)


def test_build_then_search_recall():
    w = synth.config1(n=10_000, nq=100)
    ix, adj = _build(w, degree=32, cand=64, n_entry=512, seed=w.build_seed)
    gi, gd, _ = oracle.bruteforce(w.x, w.attrs, w.q, w.qattrs, 10)
    ids, dist = nhq.nhq_hybrid_search(ix, _dev(w.q), _dev(w.qattrs), 10, 128)
    rec = oracle.recall(ids.cpu().numpy(), w.x, w.attrs, w.q, w.qattrs, gi, gd, 10)
    assert rec.mean() > 0.8
