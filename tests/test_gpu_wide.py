"""Wide rows (the precision form's d = 960, d = 1000 padded to 1024, and
d = 500 padded to 512, the narrowest width whose searches read the query row
from LDS): the kernels' 16-lane row groups, the one-round-in-flight scoring,
the LDS query row and the wide matrix-core tiles, in the batch search and the
serving loop, against the CPU oracle.

Float vectors: orders can differ from the FP64 oracle only at near-ties, so
results must overlap and every returned distance must be Gamma of the
returned object to 1e-4 relative (FP64)."""
import numpy as np
import pytest
import torch

import oracle
from parity import assert_float_parity
import synth

pytestmark = pytest.mark.gpu

nhq = pytest.importorskip("paper_2203_13601_amd")


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def test_graph_matches_oracle_d960():
    w = synth.small(1500, 960, 1, seed=91, n_centres=6, cards=(2, 3, 5, 10))
    ix = nhq.nhq_build_index(_dev(w.x), _dev(w.attrs), degree=32, cand=48, n_entry=64, seed=1)
    adj = nhq.nhq_index_get_graph(ix).cpu().numpy()
    want = oracle.build_graph(w.x, w.attrs, l=48, R=32)
    same = (adj == want).all(axis=1)
    assert same.mean() >= 0.995, same.mean()


@pytest.mark.parametrize("d,cand", [(500, 64), (1000, 100)])
def test_graph_matches_oracle_wide_tiles(d, cand):
    # the LDS-staged tiles of 512+ element rows: 8 waves per workgroup with
    # 48 entries of survivor slack (cand 64, 80 kept), and 4 waves (cand 100,
    # 116 kept); 1,300 rows leave a ragged row block
    w = synth.small(1300, d, 1, seed=96, n_centres=6, cards=(2, 3, 5, 10))
    ix = nhq.nhq_build_index(_dev(w.x), _dev(w.attrs), degree=32, cand=cand, n_entry=64, seed=1)
    adj = nhq.nhq_index_get_graph(ix).cpu().numpy()
    want = oracle.build_graph(w.x, w.attrs, l=cand, R=32)
    same = (adj == want).all(axis=1)
    assert same.mean() >= 0.995, same.mean()
    ix.free()


@pytest.mark.parametrize("d", [500, 960, 1000])
@pytest.mark.parametrize("storage", ["fp32", "bf16", "fp8"])
def test_search_matches_oracle_wide(d, storage):
    w = synth.small(4000, d, 48, seed=92, n_centres=8, cards=(2, 3, 5))
    adj = synth.random_graph(w.n, 32, seed=5)
    if storage == "fp32":
        xs = w.x
    elif storage == "bf16":
        xs = oracle.from_bf16_bits(oracle.to_bf16_bits(w.x)).astype(np.float32)
    else:
        codes, s = oracle.fp8_rows(w.x)
        xs = oracle.fp8_decode_rows(codes, s).astype(np.float32)
    rr = 0 if storage == "fp32" else 4
    ix = nhq.nhq_index_create(_dev(w.x), _dev(w.attrs), storage=storage, n_entry=256, seed=w.build_seed,
                              degree=32)
    nhq.nhq_index_set_graph(ix, _dev(adj))
    entry = oracle.entry_points(w.build_seed, w.n, 256)
    ids, dist = nhq.nhq_hybrid_search(ix, _dev(w.q), _dev(w.qattrs), 10, 64, rerank=rr, expand=4)
    ids, dist = ids.cpu().numpy(), dist.cpu().numpy()
    oi, og, _, _, _ = oracle.search(adj, xs, w.attrs, w.q, w.qattrs, 10, 64, entry, rerank_n=10 * rr,
                                    xr=w.x if rr else None, expand=4)
    assert_float_parity(ids, oi, w.x, w.attrs, w.q, w.qattrs)
    for i in range(w.nq):
        mq = oracle.arity(w.qattrs[i])
        for v, g in zip(ids[i], dist[i]):
            if v < 0:
                assert np.isinf(g)
                continue
            c = oracle.chi(w.qattrs[i], w.attrs[v])
            assert c == 0
            want = oracle.gamma(oracle.delta(w.q[i], w.x[v]), c, mq)
            assert abs(g - want) <= 1e-4 * max(want, 1e-30), (i, v, g, want)


def test_bruteforce_knn_d960():
    w = synth.small(6000, 960, 40, seed=93, n_centres=8, cards=(2, 3, 5), wildcard_arity=True)
    ix = nhq.nhq_index_create(_dev(w.x), _dev(w.attrs), n_entry=64)
    gi, gd = nhq.nhq_bruteforce_hybrid_knn(ix, _dev(w.q), _dev(w.qattrs), 10)
    gi, gd = gi.cpu().numpy(), gd.cpu().numpy()
    oi, og, _ = oracle.bruteforce(w.x, w.attrs, w.q, w.qattrs, 10)
    # ids equal except where two exact distances tie in float32
    for i in range(w.nq):
        ok = (gi[i] == oi[i]) | np.isclose(gd[i], og[i], rtol=1e-6)
        assert ok.all(), i
        fin = np.isfinite(og[i])
        assert np.allclose(gd[i][fin], og[i][fin], rtol=1e-5)


@pytest.mark.parametrize("d,k,nq", [(500, 10, 150), (960, 100, 70), (1000, 40, 130)])
def test_bruteforce_knn_wide_tiles(d, k, nq):
    # exact kNN through the LDS-staged tiles: two row blocks of 8 waves (one
    # ragged), the 4-wave form (k = 100), and four column ranges of which
    # the last ends inside a 128-column tile
    w = synth.small(2900, d, nq, seed=95 + d, n_centres=8, cards=(2, 3, 5), wildcard_arity=True)
    ix = nhq.nhq_index_create(_dev(w.x), _dev(w.attrs), n_entry=64)
    gi, gd = nhq.nhq_bruteforce_hybrid_knn(ix, _dev(w.q), _dev(w.qattrs), k)
    gi, gd = gi.cpu().numpy(), gd.cpu().numpy()
    oi, og, _ = oracle.bruteforce(w.x, w.attrs, w.q, w.qattrs, k)
    for i in range(w.nq):
        ok = (gi[i] == oi[i]) | np.isclose(gd[i], og[i], rtol=1e-6)
        assert ok.all(), i
        fin = np.isfinite(og[i])
        assert np.array_equal(np.isfinite(gd[i]), fin), i
        assert np.allclose(gd[i][fin], og[i][fin], rtol=1e-5)
    ix.free()


@pytest.mark.parametrize("d,storage", [(500, "fp32"), (960, "bf16")])
def test_serve_matches_oracle_wide(d, storage):
    # the serving loop at widths that keep the query row in LDS: its own
    # entry ranking, then the shared per-query search, against the oracle's
    # search on the stored rows (FP32 re-score for bf16)
    w = synth.small(4000, d, 48, seed=94, n_centres=8, cards=(2, 3, 5), wildcard_arity=True)
    adj = synth.random_graph(w.n, 32, seed=6)
    rr = 0 if storage == "fp32" else 4
    xs = w.x if storage == "fp32" else oracle.from_bf16_bits(oracle.to_bf16_bits(w.x)).astype(np.float32)
    ix = nhq.nhq_index_create(_dev(w.x), _dev(w.attrs), storage=storage, n_entry=256, seed=w.build_seed,
                              degree=32)
    nhq.nhq_index_set_graph(ix, _dev(adj))
    n = w.nq
    k = np.full(n, 10, np.int32)
    beam = np.full(n, 64, np.int32)
    with nhq.Server(ix, n_init=16, expand=4, rerank=rr, lifetime_s=60.0, ring=128, slots_small=32,
                    beam_large=-1) as srv:
        r = srv.run(w.q, w.qattrs, k, beam, synth.poisson_arrivals(n, 50_000.0, 7), timeout_s=30.0)
    ids, dist = r["ids"][:, :10], r["dists"][:, :10]
    entry = oracle.entry_points(w.build_seed, w.n, 256)
    oi, og, _, _, _ = oracle.search(adj, xs, w.attrs, w.q, w.qattrs, 10, 64, entry, n_init=16,
                                    rerank_n=10 * rr, xr=w.x if rr else None, expand=4)
    assert_float_parity(ids, oi, w.x, w.attrs, w.q, w.qattrs)
    for i in range(n):
        mq = oracle.arity(w.qattrs[i])
        for v, g in zip(ids[i], dist[i]):
            if v < 0:
                assert np.isinf(g)
                continue
            assert oracle.chi(w.qattrs[i], w.attrs[v]) == 0
            want = oracle.gamma(oracle.delta(w.q[i], w.x[v]), 0, mq)
            assert abs(g - want) <= 1e-4 * max(want, 1e-30), (i, v, g, want)
    ix.free()
