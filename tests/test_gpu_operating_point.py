"""Parity at the plain workload's operating point, at a size where the
visited set is the LDS hash: 200,000 integer-valued 128-d vectors from 256
clusters (the 1M x 128 workload's recipe), 3 attributes of cardinality
3/4/5, full constraints, an entry sample of 4,096, 4 seeds, 6 expansions per
step, beam 32 -- the launch the benchmark times, through the same two calls
(seed ranking, then the seeded search).

The graph is the oracle's own (NN-descent candidate lists refined for three
rounds, then the landing-zone edge selection of Sec. 4.1), never the GPU's.
Integer data makes every distance exact in float32, so the kernel must agree
with the oracle's float32-key mode id for id, NDC for NDC and hop for hop."""
import numpy as np
import pytest
import torch

import oracle
import synth

pytestmark = pytest.mark.gpu
nhq = pytest.importorskip("paper_2203_13601_amd")

N, NQ, N_ENTRY, N_INIT, EXPAND, K = 200_000, 256, 4096, 4, 6, 10
SEED_MARGIN = 8


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


@pytest.fixture(scope="module")
def plain():
    w = synth.config2(n=N, nq=NQ)
    lists, _ = oracle.nndescent(w.x, w.attrs, l=64, s=8, rounds=3, seed=11)
    adj = oracle.select_lists(w.x, w.attrs, lists, 32)
    entry = oracle.entry_points(w.build_seed, w.n, N_ENTRY)
    return w, adj, entry


@pytest.mark.parametrize("storage", ["fp32", "bf16"])
@pytest.mark.parametrize("beam", [32, 64])
def test_bench_launch_matches_oracle(plain, storage, beam):
    w, adj, entry = plain
    ix = nhq.nhq_index_create(_dev(w.x), _dev(w.attrs), storage=storage, n_entry=N_ENTRY,
                              seed=w.build_seed, degree=32)
    nhq.nhq_index_set_graph(ix, _dev(adj))
    q, qa = _dev(w.q), _dev(w.qattrs)
    n_cand = N_INIT + SEED_MARGIN
    cand = nhq.nhq_seed_rank(ix, q, qa, n_cand)
    ids, dist, cnt = nhq.nhq_search_seeded(ix, q, qa, cand, K, beam, n_init=N_INIT, expand=EXPAND,
                                           counters=True)
    torch.cuda.synchronize()
    oi, og, ondc, ohops, oflag = oracle.search(adj, w.x, w.attrs, w.q, w.qattrs, K, beam, entry,
                                               n_init=N_INIT, key_mode=oracle.KEY32, expand=EXPAND)
    ids, dist, cnt = ids.cpu().numpy(), dist.cpu().numpy(), cnt.cpu().numpy()
    assert np.array_equal(ids, oi)
    assert np.array_equal(cnt[:, 0], ondc)
    assert np.array_equal(cnt[:, 1], ohops)
    fin = np.isfinite(og)
    assert np.array_equal(np.isfinite(dist), fin)
    assert np.allclose(dist[fin], og[fin], rtol=1e-4)
    assert not oflag.any() and nhq.nhq_index_device_error(ix) == 0
    ix.free()


# ---- the headline launch at full size: 1,000,000 x 960 Gaussian mixture,
# 4 attributes (2/3/5/10) all constrained, entry sample 1,024, 4 seeds, 2
# expansions per step, beam 20; float32 rows and bf16 rows with the float32
# re-score.  The graph is a seeded random degree-32 graph (the oracle cannot
# build the composite index at this size); float data, so the answers must
# overlap at >= 0.99 with Recall@10 within 0.005 and FP64-exact distances,
# on a sample of the batch the launch answers.
@pytest.fixture(scope="module")
def headline():
    w = synth.config3(n=1_000_000, nq=10_000)
    adj = synth.random_graph(w.n, 32, seed=21)
    return w, adj


@pytest.mark.parametrize("storage", ["fp32", "bf16"])
def test_headline_launch_full_size(headline, storage):
    from parity import assert_float_parity
    w, adj = headline
    ix = nhq.nhq_index_create(_dev(w.x), _dev(w.attrs), storage=storage, n_entry=1024, seed=w.build_seed,
                              degree=32)
    nhq.nhq_index_set_graph(ix, _dev(adj))
    rr = 4 if storage == "bf16" else 0
    q, qa = _dev(w.q), _dev(w.qattrs)
    cand = nhq.nhq_seed_rank(ix, q, qa, 4 + SEED_MARGIN)
    ids, dist = nhq.nhq_search_seeded(ix, q, qa, cand, K, 20, n_init=4, expand=2, rerank=rr)
    torch.cuda.synchronize()
    sel = np.arange(0, w.nq, 40)                       # 250 of the 10,000 answers
    ids, dist = ids.cpu().numpy()[sel], dist.cpu().numpy()[sel]
    xs = w.x if storage == "fp32" else oracle.from_bf16_bits(oracle.to_bf16_bits(w.x)).astype(np.float32)
    entry = oracle.entry_points(w.build_seed, w.n, 1024)
    oi, og, _, _, _ = oracle.search(adj, xs, w.attrs, w.q[sel], w.qattrs[sel], K, 20, entry, n_init=4,
                                    expand=2, rerank_n=min(4 * K, 20) if rr else 0, xr=w.x if rr else None)
    assert_float_parity(ids, oi, w.x, w.attrs, w.q[sel], w.qattrs[sel])
    # every returned distance is the FP64 Gamma of the returned object (all
    # four attributes constrained and matched: Gamma = delta)
    for i, qi in enumerate(sel):
        for v, g in zip(ids[i], dist[i]):
            if v < 0:
                assert np.isinf(g)
                continue
            assert oracle.chi(w.qattrs[qi], w.attrs[v]) == 0
            want = oracle.delta(w.q[qi], w.x[v])
            assert abs(g - want) <= 1e-4 * want, (qi, v, g, want)
    ix.free()
