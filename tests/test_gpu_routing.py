"""GPU parity of two-stage routing (Sec. 4.2) against the CPU oracle, through
the C ABI.  On integer-valued vectors ids, NDC and hops must agree exactly;
on float vectors the answers overlap and every distance is Gamma of the
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


def _index(w, adj, n_entry=256, storage="fp32"):
    ix = nhq.nhq_index_create(_dev(w.x), _dev(w.attrs), storage=storage, n_entry=n_entry,
                              seed=w.build_seed, degree=adj.shape[1])
    nhq.nhq_index_set_graph(ix, _dev(adj))
    return ix


def _gpu(ix, w, k, L, **kw):
    ids, d, cnt = nhq.nhq_hybrid_search(ix, _dev(w.q), _dev(w.qattrs), k, L, counters=True, **kw)
    torch.cuda.synchronize()
    return ids.cpu().numpy(), d.cpu().numpy(), cnt.cpu().numpy()


@pytest.fixture(scope="module")
def int_set():
    w = synth.small(8000, 128, 96, seed=51, integer=True, n_centres=8)
    adj = oracle.build_graph(w.x, w.attrs, l=48, R=32)
    return w, adj


@pytest.mark.parametrize("h,E,L", [(2, 1, 64), (3, 1, 100), (5, 4, 64), (32, 1, 48), (4, 6, 128),
                                   (2, 8, 17), (7, 3, 256)])
def test_two_stage_integer_exact(int_set, h, E, L):
    w, adj = int_set
    ix = _index(w, adj)
    entry = oracle.entry_points(w.build_seed, w.n, 256)
    ids, dist, cnt = _gpu(ix, w, 10, L, expand=E, route_h=h)
    oi, og, ondc, ohops, _ = oracle.search(adj, w.x, w.attrs, w.q, w.qattrs, 10, L, entry,
                                           key_mode=oracle.KEY32, expand=E, route_h=h)
    assert np.array_equal(ids, oi)
    assert np.array_equal(cnt[:, 0], ondc)
    assert np.array_equal(cnt[:, 1], ohops)
    fin = np.isfinite(og)
    assert np.allclose(dist[fin], og[fin], rtol=1e-4)
    assert nhq.nhq_index_device_error(ix) == 0


def test_two_stage_random_graph_odd_degree_and_padding():
    # R = 24 (not a power of two) with -1 padded rows
    w = synth.small(6000, 32, 64, seed=57, integer=True, n_centres=4)
    adj = synth.random_graph(w.n, 24, seed=12, pad_frac=0.25)
    ix = _index(w, adj, n_entry=128)
    entry = oracle.entry_points(w.build_seed, w.n, 128)
    for h, E in ((3, 1), (5, 2)):
        ids, dist, cnt = _gpu(ix, w, 10, 80, expand=E, route_h=h)
        oi, og, ondc, ohops, _ = oracle.search(adj, w.x, w.attrs, w.q, w.qattrs, 10, 80, entry,
                                               key_mode=oracle.KEY32, expand=E, route_h=h)
        assert np.array_equal(ids, oi)
        assert np.array_equal(cnt[:, 0], ondc)
        assert np.array_equal(cnt[:, 1], ohops)


def test_two_stage_hop_cap_and_learned_kernel(int_set):
    # the hop cap can end the search inside S1; the checkpointing kernel
    # (traces on) runs the same routing
    w, adj = int_set
    ix = _index(w, adj)
    entry = oracle.entry_points(w.build_seed, w.n, 256)
    for mh in (3, 20):
        ids, dist, cnt = _gpu(ix, w, 10, 64, route_h=4, max_hops=mh)
        oi, og, ondc, ohops, _ = oracle.search(adj, w.x, w.attrs, w.q, w.qattrs, 10, 64, entry,
                                               key_mode=oracle.KEY32, route_h=4, max_hops=mh)
        assert np.array_equal(ids, oi)
        assert np.array_equal(cnt[:, 0], ondc)
        assert np.array_equal(cnt[:, 1], ohops)
    tr = nhq.TraceBuffers(w.nq, 16)
    ids, dist, cnt = _gpu(ix, w, 10, 64, route_h=3, expand=2, check_every=4, trace=tr)
    oi, og, ondc, ohops, _, otr = oracle.search(adj, w.x, w.attrs, w.q, w.qattrs, 10, 64, entry,
                                                key_mode=oracle.KEY32, route_h=3, expand=2,
                                                check_every=4, trace_cap=16)
    assert np.array_equal(ids, oi)
    assert np.array_equal(cnt[:, 0], ondc)
    assert np.array_equal(cnt[:, 1], ohops)
    torch.cuda.synchronize()
    assert np.array_equal(tr.count.cpu().numpy(), otr["count"])
    assert np.array_equal(tr.hop.cpu().numpy(), otr["hop"])


def test_two_stage_float_and_bf16():
    w = synth.config1(n=6000, nq=96)
    adj = oracle.build_graph(w.x, w.attrs, l=48, R=32)
    entry = oracle.entry_points(w.build_seed, w.n, 256)
    for storage in ("fp32", "bf16"):
        xs = w.x if storage == "fp32" else oracle.from_bf16_bits(
            oracle.to_bf16_bits(w.x)).astype(np.float32)
        ix = _index(w, adj, storage=storage)
        ids, dist, cnt = _gpu(ix, w, 10, 64, route_h=3, expand=4)
        oi, og, ondc, _, _ = oracle.search(adj, xs, w.attrs, w.q, w.qattrs, 10, 64, entry,
                                           route_h=3, expand=4)
        assert_float_parity(ids, oi, w.x, w.attrs, w.q, w.qattrs)
        for i in range(w.nq):
            mq = oracle.arity(w.qattrs[i])
            for v, g in zip(ids[i], dist[i]):
                if v < 0:
                    continue
                c = oracle.chi(w.qattrs[i], w.attrs[v])
                want = oracle.gamma(oracle.delta(w.q[i], w.x[v]), c, mq)
                assert abs(g - want) <= 1e-4 * max(want, 1e-30)


def test_route_h_argument_check(int_set):
    w, adj = int_set
    ix = _index(w, adj)
    for bad in (-1, 65):
        with pytest.raises(Exception):
            nhq.nhq_hybrid_search(ix, _dev(w.q[:2]), _dev(w.qattrs[:2]), 10, 64, route_h=bad)
