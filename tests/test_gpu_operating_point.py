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
