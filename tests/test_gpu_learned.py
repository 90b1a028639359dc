"""Learned stop network on the GPU against the CPU oracle: checkpoint traces,
training samples, gradients and Adam steps (FP64 reference), fp16 in-loop
inference, learned-stop searches, and what the trained network gains over
fixed-beam search at equal recall."""
import numpy as np
import pytest
import torch

import hand_walks
import oracle
import synth

pytestmark = pytest.mark.gpu
nhq = pytest.importorskip("paper_2203_13601_amd")


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def _flat(p):
    return np.concatenate([p[k].ravel() for k in ("W1", "b1", "W2", "b2", "W3", "b3")])


def _unflat(v):
    out, o = {}, 0
    for k in ("W1", "b1", "W2", "b2", "W3", "b3"):
        shp = oracle.MLPRef.SHAPES[k]
        sz = int(np.prod(shp))
        out[k] = np.asarray(v[o:o + sz], dtype=np.float64).reshape(shp)
        o += sz
    return out


@pytest.fixture(scope="module")
def setup():
    w = synth.small(8000, 64, 160, seed=91, integer=True, n_centres=6)
    adj = oracle.build_graph(w.x, w.attrs, l=48, R=24)
    ix = nhq.nhq_index_create(_dev(w.x), _dev(w.attrs), n_entry=256, seed=5, degree=24)
    nhq.nhq_index_set_graph(ix, _dev(adj))
    entry = oracle.entry_points(5, w.n, 256)
    return w, adj, ix, entry


def test_trace_matches_oracle(setup):
    w, adj, ix, entry = setup
    tr = nhq.TraceBuffers(w.nq, 48)
    ids, dist, cnt = nhq.nhq_hybrid_search(ix, _dev(w.q), _dev(w.qattrs), 10, 96, check_every=4,
                                           counters=True, trace=tr)
    torch.cuda.synchronize()
    o = oracle.search(adj, w.x, w.attrs, w.q, w.qattrs, 10, 96, entry, key_mode=oracle.KEY32,
                      check_every=4, trace_cap=48)
    otr = o[5]
    assert np.array_equal(ids.cpu().numpy(), o[0])
    assert np.array_equal(tr.count.cpu().numpy(), otr["count"])
    assert np.array_equal(tr.final_hash.cpu().numpy().view(np.uint32), otr["final_hash"])
    c = otr["count"]
    mask = np.arange(48)[None, :] < c[:, None]
    assert np.array_equal(tr.hop.cpu().numpy().view(np.uint32)[mask], otr["hop"][mask])
    assert np.array_equal(tr.hash.cpu().numpy().view(np.uint32)[mask], otr["hash"][mask])
    f = tr.feat.cpu().numpy()[mask]
    assert np.allclose(f, otr["feat"][mask], atol=2e-6, rtol=1e-5)
    # samples and labels
    X, ys, yb = nhq.nhq_trace_samples(tr, cnt)
    X, ys, yb = X.cpu().numpy(), ys.cpu().numpy(), yb.cpu().numpy()
    assert X.shape[0] == c.sum()
    wy, wb, r = [], [], 0
    for q in range(w.nq):
        lab = otr["hash"][q, :c[q]] == otr["final_hash"][q]
        first = o[3][q]
        for t in range(c[q] - 1, -1, -1):
            if not lab[t]:
                break
            first = otr["hop"][q, t]
        wy += list(lab.astype(np.float32))
        wb += [np.log2(max(1, first))] * c[q]
    assert np.array_equal(ys, np.array(wy, np.float32))
    assert np.allclose(yb, np.array(wb), atol=1e-6)


def test_gradient_matches_fp64_reference():
    rng = np.random.default_rng(0)
    p = oracle.MLPRef.init(1)
    for k in p:
        p[k] = p[k] + rng.standard_normal(p[k].shape) * 0.05
    n = 300
    X = rng.standard_normal((n, 8))
    ys = (rng.uniform(size=n) > 0.5).astype(np.float64)
    yb = rng.uniform(3, 8, size=n)
    g, loss, z = nhq.nhq_mlp_grad(_dev(_flat(p).astype(np.float32)), _dev(X.astype(np.float32)),
                                  _dev(ys.astype(np.float32)), _dev(yb.astype(np.float32)), 0.5,
                                  want_z=True)
    # the reference sees the same float32-rounded inputs
    p32 = {k: v.astype(np.float32).astype(np.float64) for k, v in p.items()}
    X32 = X.astype(np.float32).astype(np.float64)
    yb32 = yb.astype(np.float32).astype(np.float64)
    zr, cache = oracle.MLPRef.forward(p32, X32)
    gr = _flat(oracle.MLPRef.backward(p32, cache, zr, ys, yb32, lam=0.5))
    lr_ = oracle.MLPRef.loss(zr, ys, yb32, lam=0.5)
    assert np.allclose(z.cpu().numpy(), zr, rtol=1e-5, atol=1e-5)
    assert loss.item() == pytest.approx(lr_, rel=1e-5)
    gg = g.cpu().numpy().astype(np.float64)
    scale = np.abs(gr).max()
    assert np.abs(gg - gr).max() <= 1e-5 * scale


def test_adam_training_matches_reference():
    rng = np.random.default_rng(1)
    p = oracle.MLPRef.init(2)
    n = 256
    X = rng.standard_normal((n, 8)).astype(np.float32)
    ys = (X[:, 0] > 0).astype(np.float32)
    yb = (X[:, 1] * 2 + 5).astype(np.float32)
    params = _dev(_flat(p).astype(np.float32))
    state = torch.zeros(2 * nhq.MLP_PARAMS, dtype=torch.float32, device="cuda")
    step, losses = nhq.nhq_mlp_train(params, state, 0, _dev(X), _dev(ys), _dev(yb), epochs=5,
                                     batch=256, lr=1e-2, lam=1.0, seed=3)
    assert step == 5
    # one full batch per epoch: the order of samples does not matter
    pr = {k: v.astype(np.float32).astype(np.float64) for k, v in p.items()}
    st = {}
    X64, ys64, yb64 = X.astype(np.float64), ys.astype(np.float64), yb.astype(np.float64)
    ref_losses = []
    for _ in range(5):
        z, cache = oracle.MLPRef.forward(pr, X64)
        ref_losses.append(oracle.MLPRef.loss(z, ys64, yb64))
        pr = oracle.MLPRef.adam(pr, oracle.MLPRef.backward(pr, cache, z, ys64, yb64), st, lr=1e-2)
    got = params.cpu().numpy().astype(np.float64)
    want = _flat(pr)
    assert np.abs(got - want).max() <= 1e-4 * max(1.0, np.abs(want).max())
    assert np.allclose(losses.cpu().numpy(), ref_losses, rtol=1e-4)


def test_fp16_inference_matches_reference(setup):
    w, adj, ix, entry = setup
    p = oracle.MLPRef.init(4)
    flat = _flat(p).astype(np.float32)
    nhq.nhq_mlp_load(ix, _dev(flat))
    X = np.random.default_rng(5).standard_normal((500, 8)).astype(np.float32)
    Z = nhq.nhq_mlp_eval(ix, _dev(X)).cpu().numpy()
    ph = _unflat(flat.astype(np.float16).astype(np.float64))
    zr, _ = oracle.MLPRef.forward(ph, X.astype(np.float64))
    assert np.abs(Z - zr).max() <= 1e-2
    assert np.abs(Z - zr).max() <= 1e-4 * max(1.0, np.abs(zr).max())
    nhq.nhq_mlp_load(ix, None)


def _check_learned(ix, w, adj, entry, wh, mode, tau, cf, ce, beam=128):
    """The learned search against the oracle's.  Both evaluate the network on
    the same fp16 weights, the kernel in float32 with float32 features, the
    oracle in FP64, so a stop decision can differ only where the stop logit
    (or the budget exponent) lies within rounding of its threshold.  Every
    query must either equal the oracle's run, or stop at a hop count between
    the oracle's runs with the threshold and the budget moved by that rounding
    band -- and then return exactly the oracle's search state at that hop."""
    import math
    kw = dict(learned=mode, stop_threshold=tau, check_every=ce, counters=True)
    if cf:
        kw["cap_factor"] = cf
    ids, dist, cnt = nhq.nhq_hybrid_search(ix, _dev(w.q), _dev(w.qattrs), 10, beam, **kw)
    ids, hops = ids.cpu().numpy(), cnt.cpu().numpy()[:, 1].astype(np.int64)

    def orun(t, c):
        return oracle.search(adj, w.x, w.attrs, w.q, w.qattrs, 10, beam, entry, key_mode=oracle.KEY32,
                             check_every=ce, mlp=wh, stop_threshold=t, cap_factor=c, learned_mode=mode)
    o = orun(tau, cf)
    eps = 1e-3                                   # logit / log2-budget rounding band
    lg = math.log(tau / (1.0 - tau))
    sig = lambda z: 1.0 / (1.0 + math.exp(-z))  # noqa: E731
    early = orun(sig(lg - eps), cf * 2.0 ** -eps if cf else 0.0)
    late = orun(sig(lg + eps), cf * 2.0 ** eps if cf else 0.0)
    same = (ids == o[0]).all(axis=1) & (hops == o[3])
    for q in np.nonzero(~same)[0]:
        assert early[3][q] <= hops[q] <= late[3][q], (q, hops[q], early[3][q], o[3][q], late[3][q])
        ref = oracle.search(adj, w.x, w.attrs, w.q[q:q + 1], w.qattrs[q:q + 1], 10, beam, entry,
                            key_mode=oracle.KEY32, max_hops=int(hops[q]))
        assert np.array_equal(ref[0][0], ids[q]), q
    return float(same.mean())


def test_learned_search_matches_oracle(setup):
    w, adj, ix, entry = setup
    p = oracle.MLPRef.init(6)
    flat = _flat(p).astype(np.float32)
    flat[4864] = -1.0                 # a stop logit that crosses zero for some states
    nhq.nhq_mlp_load(ix, _dev(flat))
    wh = flat.astype(np.float16).astype(np.float64)
    for tau in (0.3, 0.6):
        _check_learned(ix, w, adj, entry, wh, 1, tau, 0.0, 4)
    # the hop budget (checked before every step) and the one-checkpoint mode
    for mode, tau, cf, ce in ((1, 0.6, 1.5, 4), (2, 0.6, 2.0, 8), (2, 0.99, 1.0, 4)):
        _check_learned(ix, w, adj, entry, wh, mode, tau, cf, ce)
    nhq.nhq_mlp_load(ix, None)
    with pytest.raises(nhq.NHQError):
        nhq.nhq_hybrid_search(ix, _dev(w.q), _dev(w.qattrs), 10, 64, learned=True)


def test_trained_network_gain_over_fixed_beam():
    # train on traces of training queries, evaluate on held-out queries:
    # the learned stop (from a large beam) against the fixed-beam sweep
    from paper_2203_13601_amd import learned
    from paper_2203_13601_amd.metrics import recall_at_k
    w = synth.small(30000, 64, 1200, seed=92, integer=True, n_centres=16, zipf=True)
    ix = nhq.nhq_build_index(_dev(w.x), _dev(w.attrs), degree=32, cand=64, n_entry=1024, seed=7)
    qtr, qatr = _dev(w.q[:800]), _dev(w.qattrs[:800])
    qte, qate = _dev(w.q[800:]), _dev(w.qattrs[800:])
    params, info = learned.train_stop_network(ix, qtr, qatr, k=10, beam=128, epochs=30, seed=1)
    nhq.nhq_mlp_load(ix, params)
    qa_np = w.qattrs[800:]
    gi, _, _ = oracle.bruteforce(w.x, w.attrs, w.q[800:], qa_np, 10)   # exact answers, FP64
    def run(**kw):
        ids, dist, cnt = nhq.nhq_hybrid_search(ix, qte, qate, 10, kw.pop("beam"), counters=True, **kw)
        r = recall_at_k(ids.cpu().numpy(), w.x, w.q[800:], w.attrs, qa_np, gi, 10).mean()
        return r, cnt.cpu().numpy()[:, 1].mean()
    fixed = {L: run(beam=L) for L in (12, 16, 24, 32, 48, 64, 96, 128)}
    learned_pts = {tau: run(beam=128, learned=True, stop_threshold=tau, check_every=4)
                   for tau in (0.5, 0.8, 0.9, 0.95, 0.99)}
    Ls = sorted(fixed)

    def fixed_hops_at(r):
        """hops the fixed beam needs for recall r (linear between swept beams)"""
        for a, b in zip(Ls, Ls[1:]):
            (ra, ha), (rb, hb) = fixed[a], fixed[b]
            if ra <= r <= rb:
                return ha + (hb - ha) * ((r - ra) / max(rb - ra, 1e-9))
        return None

    report = {tau: (round(r, 4), round(h, 1), fixed_hops_at(r)) for tau, (r, h) in learned_pts.items()}
    print("fixed beam (recall, hops):", {L: (round(r, 4), round(h, 1)) for L, (r, h) in fixed.items()})
    print("learned (recall, hops, fixed-beam hops at that recall):", report)
    # a higher threshold stops later and loses less recall
    taus = sorted(learned_pts)
    hops = [learned_pts[t][1] for t in taus]
    assert all(b >= a - 1e-9 for a, b in zip(hops, hops[1:]))
    # the most conservative threshold stays close to the largest beam's recall
    # while stopping well before that beam is exhausted
    r99, h99 = learned_pts[0.99]
    assert r99 >= fixed[128][0] - 0.02
    assert h99 < 0.8 * fixed[128][1]
    # the gain over the method without the network: at the recall a threshold
    # reaches, the fixed beam needs more expansions than the learned stop
    gains = [(tau, fixed_hops_at(r) - h) for tau, (r, h) in learned_pts.items()
             if fixed_hops_at(r) is not None]
    assert gains, report
    assert max(g for _, g in gains) > 0, report


def test_trace_with_multi_expansion_matches_oracle(setup):
    w, adj, ix, entry = setup
    tr = nhq.TraceBuffers(w.nq, 48)
    ids, dist, cnt = nhq.nhq_hybrid_search(ix, _dev(w.q), _dev(w.qattrs), 10, 96, check_every=4,
                                           counters=True, trace=tr, expand=3)
    o = oracle.search(adj, w.x, w.attrs, w.q, w.qattrs, 10, 96, entry, key_mode=oracle.KEY32,
                      check_every=4, trace_cap=48, expand=3)
    otr = o[5]
    assert np.array_equal(ids.cpu().numpy(), o[0])
    assert np.array_equal(tr.count.cpu().numpy(), otr["count"])
    c = otr["count"]
    mask = np.arange(48)[None, :] < c[:, None]
    assert np.array_equal(tr.hop.cpu().numpy().view(np.uint32)[mask], otr["hop"][mask])
    assert np.array_equal(tr.hash.cpu().numpy().view(np.uint32)[mask], otr["hash"][mask])
    assert np.allclose(tr.feat.cpu().numpy()[mask], otr["feat"][mask], atol=2e-6, rtol=1e-5)


# ---- hand-built walks: every checkpoint feature worked out by hand (tests/hand_walks.py)


@pytest.mark.parametrize("walk", [hand_walks.chain(), hand_walks.wide_step(1), hand_walks.wide_step(2)],
                         ids=["chain", "wide_step_S1", "wide_step_S2"])
def test_trace_features_on_hand_walks(walk):
    n = len(walk["x"])
    x = np.asarray(walk["x"], np.float32)[:, None]
    attrs = np.asarray(walk["attrs"], np.uint8)[:, None]
    adj = np.asarray(walk["adj"], np.int32)
    ix = nhq.nhq_index_create(_dev(x), _dev(attrs), n_entry=n, seed=1, degree=adj.shape[1])
    nhq.nhq_index_set_graph(ix, _dev(adj))
    entry = nhq.nhq_index_get_entry(ix).cpu().numpy()
    pos = [int(np.nonzero(entry == s)[0][0]) for s in walk["seeds"]]   # every vertex is in the sample
    cand = _dev(np.asarray([pos], np.int32))
    q = _dev(np.zeros((1, 1), np.float32))
    qa = _dev(np.zeros((1, 1), np.uint8))
    tr = nhq.TraceBuffers(1, 64)
    ids, dist, cnt = nhq.nhq_search_seeded(ix, q, qa, cand, walk["k"], walk["L"], n_init=len(pos),
                                           check_every=walk["check_every"], counters=True, trace=tr,
                                           expand=walk["expand"])
    torch.cuda.synchronize()
    assert ids.cpu().numpy()[0].tolist() == walk["ids"]
    assert np.allclose(dist.cpu().numpy()[0], walk["gamma"], rtol=1e-6)
    assert cnt.cpu().numpy()[0].tolist() == [walk["ndc"], walk["hops"]]
    nck = len(walk["feat"])
    assert tr.count.cpu().numpy()[0] >= nck
    assert tr.hop.cpu().numpy()[0, :nck].tolist() == walk["hop"]
    f = tr.feat.cpu().numpy()[0, :nck].astype(np.float64)
    assert np.allclose(f, np.asarray(walk["feat"]), rtol=0, atol=2e-6), f
    hs = tr.hash.cpu().numpy().view(np.uint32)[0, :nck]
    assert [int(h) for h in hs] == [hand_walks.fingerprint(t) for t in walk["topk"]]
    assert int(tr.final_hash.cpu().numpy().view(np.uint32)[0]) == hand_walks.fingerprint(walk["ids"])
    ix.free()


# ---- learned mode 3: the beam-width predictor

def _check_pool(ix, w, adj, entry, wh, cf, ce, beam=128):
    """Mode 3 against the oracle.  The pool size ceil(cf * 2^z1) is an integer
    taken from a float: the kernel's float32 network can land on the other
    side of an integer than the oracle's FP64 one only where cf * 2^z1 lies
    within rounding of it.  Every query must equal the oracle's run, or its
    run with cf moved by that rounding band either way."""
    ids, dist, cnt = nhq.nhq_hybrid_search(ix, _dev(w.q), _dev(w.qattrs), 10, beam, learned=3, check_every=ce,
                                           cap_factor=cf, counters=True)
    ids, cnt = ids.cpu().numpy(), cnt.cpu().numpy().astype(np.int64)

    def orun(c):
        return oracle.search(adj, w.x, w.attrs, w.q, w.qattrs, 10, beam, entry, key_mode=oracle.KEY32,
                             check_every=ce, mlp=wh, cap_factor=c, learned_mode=3)
    o = orun(cf)
    eps = 1e-3
    lo, hi = orun(cf * 2.0 ** -eps), orun(cf * 2.0 ** eps)

    def eq(r, q):
        return np.array_equal(ids[q], r[0][q]) and cnt[q, 0] == r[2][q] and cnt[q, 1] == r[3][q]
    same = np.array([eq(o, q) for q in range(w.nq)])
    for q in np.nonzero(~same)[0]:
        assert eq(lo, q) or eq(hi, q), q
    return float(same.mean()), o


def test_pool_size_predictor_matches_oracle(setup):
    w, adj, ix, entry = setup
    p = oracle.MLPRef.init(11)
    flat = _flat(p).astype(np.float32)
    flat[4865] = 5.0               # beam output about log2(32) plus the network's spread
    nhq.nhq_mlp_load(ix, _dev(flat))
    wh = flat.astype(np.float16).astype(np.float64)
    fixed = oracle.search(adj, w.x, w.attrs, w.q, w.qattrs, 10, 128, entry, key_mode=oracle.KEY32)
    for cf, ce in ((1.0, 2), (0.5, 4), (2.0, 1)):
        frac, o = _check_pool(ix, w, adj, entry, wh, cf, ce)
        assert frac >= 0.95, (cf, ce, frac)
        # the predictor did cut pools: some searches end earlier than at beam 128
        assert (o[3] < fixed[3]).mean() > 0.2, (cf, ce)
    with pytest.raises(nhq.NHQError):  # mode 3 needs its pool size factor
        nhq.nhq_hybrid_search(ix, _dev(w.q), _dev(w.qattrs), 10, 64, learned=3, check_every=2)
    nhq.nhq_mlp_load(ix, None)


def test_trained_pool_predictor_on_held_out_queries():
    # train the beam-width predictor on traces of training queries; on
    # held-out queries the predicted pool sizes follow the sizes the queries
    # need, and some factor reaches the fixed-beam recall with fewer
    # distance evaluations than the fixed-beam curve at that recall
    from scipy.stats import spearmanr
    from paper_2203_13601_amd import learned
    from paper_2203_13601_amd.metrics import recall_at_k
    w = synth.small(30000, 64, 2400, seed=93, integer=True, n_centres=16, zipf=True, wildcard_arity=True)
    ix = nhq.nhq_build_index(_dev(w.x), _dev(w.attrs), degree=32, cand=64, n_entry=1024, seed=7)
    qtr, qatr = _dev(w.q[:1600]), _dev(w.qattrs[:1600])
    qte, qate = _dev(w.q[1600:]), _dev(w.qattrs[1600:])
    params, info = learned.train_pool_network(ix, qtr, qatr, k=10, beam=256, epochs=60, seed=1,
                                              check_every=1, n_init=8)
    nhq.nhq_mlp_load(ix, params)
    # the prediction at the first checkpoint against the held-out targets
    need = learned.pool_labels(ix, qte, qate, 10, 256, (10, 12, 16, 20, 24, 32, 40, 48, 64, 96, 128, 192),
                               n_init=8).cpu().numpy()
    tr = nhq.TraceBuffers(qte.shape[0], 1)
    nhq.nhq_hybrid_search(ix, qte, qate, 10, 256, n_init=8, check_every=1, trace=tr)
    has = tr.count.cpu().numpy() > 0
    Z = nhq.nhq_mlp_eval(ix, tr.feat[:, 0, :][torch.from_numpy(has).cuda()].contiguous())
    rho = spearmanr(Z[:, 1].cpu().numpy(), need[has]).correlation
    assert rho > 0.3, rho
    gi, gd = oracle.bruteforce(w.x, w.attrs, w.q[1600:], w.qattrs[1600:], 10)[:2]

    def run(**kw):
        ids, _, cnt = nhq.nhq_hybrid_search(ix, qte, qate, 10, kw.pop("beam"), n_init=8, counters=True, **kw)
        r = recall_at_k(ids.cpu().numpy(), w.x, w.q[1600:], w.attrs, w.qattrs[1600:], gi, 10).mean()
        return r, cnt.cpu().numpy()[:, 0].mean()
    fixed = [run(beam=b) for b in (12, 16, 24, 32, 48, 64, 96, 128, 192, 256)]
    fr = np.array([f[0] for f in fixed])
    fn = np.array([f[1] for f in fixed])
    gain = False
    for cf in (1.0, 1.5, 2.0, 3.0):
        r, ndc = run(beam=256, learned=3, check_every=1, cap_factor=cf)
        if r <= fr[0] or r > fr[-1]:
            continue
        j = int(np.searchsorted(fr, r))             # fixed beams bracketing r
        t = (r - fr[j - 1]) / max(fr[j] - fr[j - 1], 1e-12)
        gain = gain or ndc < fn[j - 1] + t * (fn[j] - fn[j - 1])
    nhq.nhq_mlp_load(ix, None)
    assert gain
