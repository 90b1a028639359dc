"""Stratified entry sample on the GPU against the oracle: the blocks (one per
attribute pattern, members chosen by the published splitmix64 hash), and
the joint-pruning search seeded from the query's block (full constraints)
or from the global sample (partial constraints, or a pattern no object
holds) -- integer data, so id for id, NDC for NDC and hop for hop."""
import numpy as np
import pytest
import torch

import oracle
import synth

pytestmark = pytest.mark.gpu
nhq = pytest.importorskip("paper_2203_13601_amd")


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


@pytest.fixture(scope="module")
def zipf_set():
    w = synth.small(30000, 64, 300, seed=81, integer=True, n_centres=24, zipf=True)
    qa = w.qattrs.copy()
    rng = np.random.default_rng(3)
    part = rng.random(w.nq) < 0.25                  # a quarter with wildcards
    qa[part, rng.integers(0, 3, part.sum())] = 255
    qa[:3] = [4, 2, 1]                              # a pattern no object may hold is still answered
    w.qattrs[:] = qa
    adj = oracle.build_graph(w.x, w.attrs, l=48, R=24)
    return w, adj


@pytest.mark.parametrize("per,n_entry", [(64, 256), (300, 64), (7, 1)])
def test_blocks_match_oracle(zipf_set, per, n_entry):
    w, adj = zipf_set
    ix = nhq.nhq_index_create(_dev(w.x), _dev(w.attrs), n_entry=n_entry, seed=w.build_seed, degree=24,
                              entry_per_pattern=per)
    codes, offs, ids = nhq.nhq_index_entry_blocks(ix)
    ids = ids.cpu().numpy()
    want = oracle.entry_strata(w.build_seed, w.attrs, per)
    assert offs[0] == n_entry and len(codes) == len(want)
    for b, c in enumerate(codes):
        got = ids[offs[b] - n_entry: offs[b + 1] - n_entry]
        assert np.array_equal(got, want[tuple(int(v) for v in c)]), c
    assert np.array_equal(nhq.nhq_index_get_entry(ix).cpu().numpy(),
                          oracle.entry_points(w.build_seed, w.n, n_entry))
    ix.free()


@pytest.mark.parametrize("storage", ["fp32", "bf16"])
@pytest.mark.parametrize("expand,n_init,beam", [(1, 4, 32), (4, 8, 64), (2, 1, 16)])
def test_stratified_search_matches_oracle(zipf_set, storage, expand, n_init, beam):
    w, adj = zipf_set
    per, ne = 128, 256
    ix = nhq.nhq_index_create(_dev(w.x), _dev(w.attrs), storage=storage, n_entry=ne, seed=w.build_seed,
                              degree=24, entry_per_pattern=per)
    nhq.nhq_index_set_graph(ix, _dev(adj))
    ids, dist, cnt = nhq.nhq_hybrid_search(ix, _dev(w.q), _dev(w.qattrs), 10, beam, n_init=n_init,
                                           expand=expand, counters=True)
    torch.cuda.synchronize()
    strata = oracle.entry_strata(w.build_seed, w.attrs, per)
    glob = oracle.entry_points(w.build_seed, w.n, ne)
    oi, og, ondc, ohops, _ = oracle.search_strata(adj, w.x, w.attrs, w.q, w.qattrs, 10, beam, glob, strata,
                                                  n_init=n_init, expand=expand, key_mode=oracle.KEY32)
    ids, dist, cnt = ids.cpu().numpy(), dist.cpu().numpy(), cnt.cpu().numpy()
    assert np.array_equal(ids, oi)
    assert np.array_equal(cnt[:, 0], ondc) and np.array_equal(cnt[:, 1], ohops)
    fin = np.isfinite(og)
    assert np.allclose(dist[fin], og[fin], rtol=1e-4)
    # the allocation-free entry point takes the same path
    out = (torch.empty((w.nq, 10), dtype=torch.int32, device="cuda"),
           torch.empty((w.nq, 10), dtype=torch.float32, device="cuda"))
    nhq.nhq_hybrid_search_noalloc(ix, _dev(w.q), _dev(w.qattrs), 10, beam, out=out, n_init=n_init,
                                  expand=expand)
    assert np.array_equal(out[0].cpu().numpy(), ids)
    ix.free()


def test_stratified_search_in_seed_order(zipf_set):
    # 2,700 queries (the 300 nine times over): the one-call search launches
    # batches this large in the seed order, whose candidates here are
    # positions inside the pattern blocks; results equal the natural order's
    # bit for bit and the oracle's copy for copy
    w, adj = zipf_set
    per, ne, reps = 128, 256, 9
    ix = nhq.nhq_index_create(_dev(w.x), _dev(w.attrs), n_entry=ne, seed=w.build_seed, degree=24,
                              entry_per_pattern=per)
    nhq.nhq_index_set_graph(ix, _dev(adj))
    q, qa = _dev(np.tile(w.q, (reps, 1))), _dev(np.tile(w.qattrs, (reps, 1)))
    kw = dict(n_init=4, expand=2, counters=True)
    a = nhq.nhq_hybrid_search(ix, q, qa, 10, 32, **kw)
    nat = torch.arange(q.shape[0], dtype=torch.int32, device="cuda")
    b = nhq.nhq_hybrid_search(ix, q, qa, 10, 32, order=nat, **kw)
    torch.cuda.synchronize()
    assert torch.equal(a[0], b[0])
    assert torch.equal(a[1].view(torch.int32), b[1].view(torch.int32))
    assert torch.equal(a[2], b[2])
    strata = oracle.entry_strata(w.build_seed, w.attrs, per)
    glob = oracle.entry_points(w.build_seed, w.n, ne)
    oi, _, ondc, ohops, _ = oracle.search_strata(adj, w.x, w.attrs, w.q, w.qattrs, 10, 32, glob, strata,
                                                 n_init=4, expand=2, key_mode=oracle.KEY32)
    assert np.array_equal(a[0].cpu().numpy(), np.tile(oi, (reps, 1)))
    cnt = a[2].cpu().numpy()
    assert np.array_equal(cnt[:, 0], np.tile(ondc, reps)) and np.array_equal(cnt[:, 1], np.tile(ohops, reps))
    assert nhq.nhq_index_device_error(ix) == 0
    ix.free()


def test_stratified_index_file_round_trip(zipf_set, tmp_path):
    w, adj = zipf_set
    ix = nhq.nhq_index_create(_dev(w.x), _dev(w.attrs), n_entry=256, seed=w.build_seed, degree=24,
                              entry_per_pattern=96)
    nhq.nhq_index_set_graph(ix, _dev(adj))
    a = nhq.nhq_hybrid_search(ix, _dev(w.q), _dev(w.qattrs), 10, 48, n_init=4)[0].cpu().numpy()
    path = str(tmp_path / "strata.nhq")
    nhq.nhq_index_save(ix, path)
    jx = nhq.nhq_index_load(path)
    b = nhq.nhq_hybrid_search(jx, _dev(w.q), _dev(w.qattrs), 10, 48, n_init=4)[0].cpu().numpy()
    assert np.array_equal(a, b)
    ca, oa, ia = nhq.nhq_index_entry_blocks(ix)
    cb, ob, ib = nhq.nhq_index_entry_blocks(jx)
    assert np.array_equal(ca, cb) and np.array_equal(oa, ob) and torch.equal(ia, ib)
    ix.free()
    jx.free()


def test_stratified_argument_checks(zipf_set):
    w, _ = zipf_set
    for kw in (dict(entry_per_pattern=9000), dict(entry_per_pattern=8, n_entry=9000)):
        with pytest.raises(nhq.NHQError):
            nhq.nhq_index_create(_dev(w.x), _dev(w.attrs), degree=24, **kw)
