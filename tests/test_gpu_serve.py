"""Serving loop (continuous batching) through the C ABI.

- On integer-valued vectors every distance is exact in float32, so a request
  served by the persistent kernel must give exactly the batch search's ids,
  distances and counters (same seeds: the n_cand best of the entry sample).
- Any request gives bit-identical results alone and inside a mixed stream of
  requests with other k, beams, constraint arities and output modes, whose
  work overlaps on the device.
- Admission and failure handling: a full ring refuses a submit, an ended
  kernel (lifetime reached, forced from the host) fails submits, bad requests
  are refused.

No GPU call other than the server's is made while a server runs (a device
synchronisation would wait for its persistent kernels)."""
import time

import numpy as np
import pytest
import torch

import oracle
import synth

pytestmark = pytest.mark.gpu

nhq = pytest.importorskip("paper_2203_13601_amd")
from paper_2203_13601_amd.learned import init_params  # noqa: E402

LIFE = 60.0


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


@pytest.fixture(scope="module")
def int_index():
    w = synth.small(20000, 128, 192, seed=61, integer=True, n_centres=8, wildcard_arity=True)
    ix = nhq.nhq_build_index(_dev(w.x), _dev(w.attrs), degree=32, cand=64, n_entry=1024,
                             seed=w.build_seed)
    torch.cuda.synchronize()
    return w, ix


@pytest.fixture(scope="module")
def float_index():
    w = synth.small(12000, 96, 160, cards=(2, 3, 5, 10), seed=62, wildcard_arity=True, n_centres=16)
    ix = nhq.nhq_build_index(_dev(w.x), _dev(w.attrs), degree=32, cand=64, n_entry=512,
                             seed=w.build_seed)
    torch.cuda.synchronize()
    return w, ix


def _batch(ix, w, k, beam, **kw):
    ids, d, cnt = nhq.nhq_hybrid_search(ix, _dev(w.q), _dev(w.qattrs), k, beam, counters=True, **kw)
    torch.cuda.synchronize()
    return ids.cpu().numpy(), d.cpu().numpy(), cnt.cpu().numpy().astype(np.uint32)


def _alone(srv, q, qa, k, beam, flags):
    out = []
    for i in range(len(k)):
        t = srv.submit(q[i], qa[i], int(k[i]), int(beam[i]), int(flags[i]))
        assert t >= 0
        t_end = time.time() + 20.0
        r = None
        while r is None:
            assert time.time() < t_end, "request %d did not finish" % i
            r = srv.poll(t, int(k[i]))
        out.append(r)
    return out


@pytest.mark.parametrize("expand", [1, 4])
def test_serve_equals_batch_search_on_integer_data(int_index, expand):
    w, ix = int_index
    cases = [(10, 16), (10, 64), (50, 100), (10, 300)]  # the last uses the large class
    want = {c: _batch(ix, w, c[0], c[1], n_init=32, expand=expand) for c in cases}
    n = w.nq
    rng = np.random.default_rng(7)
    pick = rng.integers(0, len(cases), size=n)
    k = np.array([cases[p][0] for p in pick], np.int32)
    beam = np.array([cases[p][1] for p in pick], np.int32)
    with nhq.Server(ix, n_init=32, expand=expand, lifetime_s=LIFE, ring=256, slots_small=96,
                    slots_large=32) as srv:
        r = srv.run(w.q, w.qattrs, k, beam, np.zeros(n), timeout_s=30.0)
    for i in range(n):
        wi, wd, wc = want[cases[pick[i]]]
        kk = k[i]
        assert np.array_equal(r["ids"][i, :kk], wi[i]), i
        assert np.array_equal(r["dists"][i, :kk].view(np.uint32), wd[i].view(np.uint32)), i
        assert np.array_equal(r["counters"][i], wc[i]), i
        assert (r["ids"][i, kk:] == -1).all()


@pytest.mark.parametrize("storage", ["fp32", "bf16"])
def test_serve_alone_equals_mix(float_index, storage):
    w, ix0 = float_index
    ix = ix0
    if storage != "fp32":
        ix = nhq.nhq_index_create(_dev(w.x), _dev(w.attrs), storage=storage, n_entry=512,
                                  seed=w.build_seed, degree=32)
        nhq.nhq_index_set_graph(ix, nhq.nhq_index_get_graph(ix0))
    nhq.nhq_mlp_load(ix, init_params(5))
    torch.cuda.synchronize()
    n = w.nq
    rng = np.random.default_rng(11)
    k = rng.choice(np.array([1, 10, 50, 100], np.int32), size=n)
    beam = np.maximum(k, rng.choice(np.array([0, 32, 100, 128, 300, 512], np.int32), size=n)).astype(np.int32)
    beam[rng.random(n) < 0.15] = 0  # learned stop at the automatic beam
    flags = (rng.random(n) < 0.2).astype(np.int32) * nhq.SERVE_RAW
    arrival = synth.poisson_arrivals(n, 200_000.0, 12)
    with nhq.Server(ix, n_init=16, expand=2, rerank=2, lifetime_s=LIFE, ring=512, slots_small=64,
                    slots_large=16, auto_beam=128) as srv:
        mix = srv.run(w.q, w.qattrs, k, beam, arrival, flags=flags, timeout_s=30.0)
        alone = _alone(srv, w.q, w.qattrs, k, beam, flags)
        hz = srv.tick_hz
    for i in range(n):
        ids, d, cnt, _ = alone[i]
        assert np.array_equal(mix["ids"][i, :k[i]], ids), i
        assert np.array_equal(mix["dists"][i, :k[i]].view(np.uint32), d.view(np.uint32)), i
        assert np.array_equal(mix["counters"][i], cnt), i
    # the mix really overlapped: requests ran on the device at the same time
    tb = mix["ticks"][:, 0].astype(np.float64)
    te = mix["ticks"][:, 1].astype(np.float64)
    ev = sorted([(t, 1) for t in tb] + [(t, -1) for t in te], key=lambda x: (x[0], x[1]))
    cur = peak = 0
    for _, dlt in ev:
        cur += dlt
        peak = max(peak, cur)
    assert peak >= 4, peak
    assert (te >= tb).all() and hz > 0
    # results are the hybrid query's: matching attributes (filtered requests)
    for i in range(n):
        if flags[i]:
            continue
        for v in mix["ids"][i, :k[i]]:
            if v >= 0:
                assert oracle.chi(w.qattrs[i], w.attrs[v]) == 0
    if ix is not ix0:
        ix.free()


@pytest.mark.parametrize("mode,cf", [(1, 0.0), (3, 32.0)])
def test_serve_learned_requests_equal_batch_learned_search(int_index, mode, cf):
    # mode 1: the stop network at every checkpoint; mode 3: the beam-width
    # predictor (pool size cf * 2^(beam output) from the first checkpoint)
    w, ix = int_index
    nhq.nhq_mlp_load(ix, init_params(3))
    torch.cuda.synchronize()
    wi, wd, wc = _batch(ix, w, 10, 128, n_init=32, learned=mode, stop_threshold=0.7, check_every=4,
                        cap_factor=cf)
    n = w.nq
    with nhq.Server(ix, n_init=32, lifetime_s=LIFE, ring=256, slots_small=64, beam_large=-1,
                    auto_beam=128, stop_threshold=0.7, check_every=4, learned_mode=mode,
                    cap_factor=cf) as srv:
        r = srv.run(w.q, w.qattrs, np.full(n, 10, np.int32), np.zeros(n, np.int32), np.zeros(n),
                    timeout_s=30.0)
    nhq.nhq_mlp_load(ix, None)
    torch.cuda.synchronize()
    assert np.array_equal(r["ids"][:, :10], wi)
    assert np.array_equal(r["dists"][:, :10].view(np.uint32), wd.view(np.uint32))
    assert np.array_equal(r["counters"], wc)


def test_two_classes_run_side_by_side_after_many_streams(int_index):
    # Both memory classes live in one persistent launch.  Streams made busy
    # beforehand (the process's streams share a few hardware queues) must
    # not keep either class from running: every request of both classes
    # finishes and equals the batch search.
    w, ix = int_index
    streams = [torch.cuda.Stream() for _ in range(12)]
    for st in streams:
        with torch.cuda.stream(st):
            torch.ones(4096, device="cuda").cumsum(0)
    torch.cuda.synchronize()
    n = w.nq
    k = np.full(n, 10, np.int32)
    beam = np.where(np.arange(n) % 2 == 0, 64, 300).astype(np.int32)   # small class, large class
    want = {b: _batch(ix, w, 10, b, n_init=32) for b in (64, 300)}
    with nhq.Server(ix, n_init=32, lifetime_s=LIFE, ring=256, slots_small=64, slots_large=16) as srv:
        assert srv.slots[0] > 0 and srv.slots[1] > 0 and srv.beam_max[1] >= 300
        r = srv.run(w.q, w.qattrs, k, beam, np.zeros(n), timeout_s=30.0)
    for b in (64, 300):
        sel = beam == b
        assert np.array_equal(r["ids"][sel, :10], want[b][0][sel])
        assert np.array_equal(r["counters"][sel], want[b][2][sel])


def test_serve_full_ring_refuses_then_recovers(int_index):
    w, ix = int_index
    with nhq.Server(ix, lifetime_s=LIFE, ring=4, slots_small=8, beam_large=-1) as srv:
        tickets = [srv.submit(w.q[i], w.qattrs[i], 10, 64) for i in range(4)]
        assert min(tickets) >= 0
        assert srv.submit(w.q[4], w.qattrs[4], 10, 64) == -1  # NHQ_EBUSY: ring full
        for t in tickets:
            t_end = time.time() + 20.0
            while srv.poll(t, 10) is None:
                assert time.time() < t_end
        assert srv.submit(w.q[4], w.qattrs[4], 10, 64) >= 0
        with pytest.raises(nhq.NHQError):
            srv.poll(tickets[0], 10)  # already polled


def test_serve_kernel_lifetime_ends_the_server(int_index):
    w, ix = int_index
    srv = nhq.Server(ix, lifetime_s=0.3, ring=16, slots_small=4, beam_large=-1)
    time.sleep(1.5)
    with pytest.raises(nhq.NHQError) as e:
        srv.submit(w.q[0], w.qattrs[0], 10, 64)
    assert e.value.code == -4  # NHQ_EDEVICE
    srv.free()


def test_serve_rejects_bad_requests(int_index):
    w, ix = int_index
    with nhq.Server(ix, lifetime_s=LIFE, ring=16, slots_small=4, beam_large=256, slots_large=2,
                    max_k=20) as srv:
        for k, beam in ((21, 64), (0, 64), (10, 5), (10, 257), (10, 0)):
            with pytest.raises(nhq.NHQError):
                srv.submit(w.q[0], w.qattrs[0], k, beam)
        with pytest.raises(nhq.NHQError):
            srv.submit(w.q[0], w.qattrs[0], 10, 64, flags=8)
    with pytest.raises(nhq.NHQError):
        nhq.Server(ix, beam_small=128, beam_large=64)


# ---- served results against the CPU oracle (graph from the oracle's build)
@pytest.fixture(scope="module")
def oracle_int_index():
    w = synth.small(20000, 128, 240, seed=63, integer=True, n_centres=8, wildcard_arity=True)
    adj = oracle.build_graph(w.x, w.attrs, l=48, R=32)
    ix = nhq.nhq_index_create(_dev(w.x), _dev(w.attrs), n_entry=1024, seed=w.build_seed, degree=32)
    nhq.nhq_index_set_graph(ix, _dev(adj))
    torch.cuda.synchronize()
    return w, adj, ix, oracle.entry_points(w.build_seed, w.n, 1024)


@pytest.fixture(scope="module")
def oracle_float_index():
    w = synth.small(12000, 96, 200, cards=(2, 3, 5, 10), seed=64, wildcard_arity=True, n_centres=16)
    adj = oracle.build_graph(w.x, w.attrs, l=48, R=32)
    ix = nhq.nhq_index_create(_dev(w.x), _dev(w.attrs), n_entry=512, seed=w.build_seed, degree=32)
    nhq.nhq_index_set_graph(ix, _dev(adj))
    torch.cuda.synchronize()
    return w, adj, ix, oracle.entry_points(w.build_seed, w.n, 512)


def _mixed_stream(w, seed):
    rng = np.random.default_rng(seed)
    n = w.nq
    k = rng.choice(np.array([1, 10, 50, 100], np.int32), size=n)
    beam = np.maximum(k, rng.choice(np.array([16, 64, 128, 300], np.int32), size=n)).astype(np.int32)
    flags = (rng.random(n) < 0.2).astype(np.int32) * nhq.SERVE_RAW
    return k, beam, flags


@pytest.mark.parametrize("expand", [1, 4])
def test_serve_equals_oracle_on_integer_data(oracle_int_index, expand):
    # mixed k, beams (both memory classes), constraint arities (1..3 of 3
    # attributes constrained) and output modes in one overlapping stream;
    # every request must equal the oracle's search id for id and counter for
    # counter, with distances within 1e-4 of the FP64 Gamma
    w, adj, ix, entry = oracle_int_index
    k, beam, flags = _mixed_stream(w, 21 + expand)
    with nhq.Server(ix, n_init=32, expand=expand, lifetime_s=LIFE, ring=512, slots_small=96,
                    slots_large=32) as srv:
        r = srv.run(w.q, w.qattrs, k, beam, synth.poisson_arrivals(w.nq, 100_000.0, 5), flags=flags,
                    timeout_s=30.0)
    for kk in np.unique(k):
        for bb in np.unique(beam):
            for ff in (0, nhq.SERVE_RAW):
                sel = np.nonzero((k == kk) & (beam == bb) & (flags == ff))[0]
                if sel.size == 0:
                    continue
                oi, og, ondc, ohops, _ = oracle.search(
                    adj, w.x, w.attrs, w.q[sel], w.qattrs[sel], int(kk), int(bb), entry, n_init=32,
                    key_mode=oracle.KEY32, expand=expand, out_mode=1 if ff else 0)
                assert np.array_equal(r["ids"][sel, :kk], oi), (kk, bb, ff)
                assert np.array_equal(r["counters"][sel, 0], ondc), (kk, bb, ff)
                assert np.array_equal(r["counters"][sel, 1], ohops), (kk, bb, ff)
                got = r["dists"][sel, :kk].astype(np.float64)
                fin = np.isfinite(og)
                assert np.array_equal(np.isfinite(got), fin)
                assert np.allclose(got[fin], og[fin], rtol=1e-4)


def test_serve_float_data_against_oracle(oracle_float_index):
    # float data: orders can differ only at near-ties.  Results must overlap
    # the oracle's search (FP64 keys) at >= 0.99, carry FP64-exact Gamma, and
    # score the same Recall@k against the exact answers (oracle brute force)
    # within 0.005
    w, adj, ix, entry = oracle_float_index
    n = w.nq
    k = np.full(n, 10, np.int32)
    beam = np.full(n, 64, np.int32)
    with nhq.Server(ix, n_init=16, expand=2, lifetime_s=LIFE, ring=512, slots_small=64,
                    beam_large=-1) as srv:
        r = srv.run(w.q, w.qattrs, k, beam, synth.poisson_arrivals(n, 100_000.0, 6), timeout_s=30.0)
    ids, dist = r["ids"][:, :10], r["dists"][:, :10]
    oi, og, _, _, _ = oracle.search(adj, w.x, w.attrs, w.q, w.qattrs, 10, 64, entry, n_init=16,
                                    expand=2)
    # share of each result set found in the other (two empty answers agree)
    overlap = np.mean([len(set(a[a >= 0]) & set(b[b >= 0])) / max(1, (a >= 0).sum(), (b >= 0).sum())
                       if (a >= 0).any() or (b >= 0).any() else 1.0 for a, b in zip(ids, oi)])
    assert overlap >= 0.99, overlap
    for i in range(n):
        mq = oracle.arity(w.qattrs[i])
        for v, g in zip(ids[i], dist[i]):
            if v < 0:
                assert np.isinf(g)
                continue
            assert oracle.chi(w.qattrs[i], w.attrs[v]) == 0
            want = oracle.gamma(oracle.delta(w.q[i], w.x[v]), 0, mq)
            assert abs(g - want) <= 1e-4 * max(want, 1e-30)
    gi, gd, _ = oracle.bruteforce(w.x, w.attrs, w.q, w.qattrs, 10)
    rs = oracle.recall(ids, w.x, w.attrs, w.q, w.qattrs, gi, gd, 10).mean()
    ro = oracle.recall(oi, w.x, w.attrs, w.q, w.qattrs, gi, gd, 10).mean()
    assert abs(rs - ro) <= 0.005, (rs, ro)
