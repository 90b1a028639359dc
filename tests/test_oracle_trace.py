"""Pins of the oracle's checkpoint traces and learned stop (the stop
network's inputs): every feature worked out by hand on small hand-built walks
(tests/hand_walks.py), and properties that hold whatever the data."""
import math

import numpy as np
import pytest

import hand_walks
import oracle
import synth


@pytest.fixture(scope="module")
def traced():
    w = synth.small(4000, 16, 60, seed=81, integer=True, n_centres=6)
    adj = oracle.build_graph(w.x, w.attrs, l=32, R=16)
    entry = oracle.entry_points(3, w.n, 128)
    out = oracle.search(adj, w.x, w.attrs, w.q, w.qattrs, 10, 96, entry, key_mode=oracle.KEY32,
                        check_every=4, trace_cap=64)
    return w, adj, entry, out


def test_trace_counters_and_closed_forms(traced):
    w, adj, entry, (ids, gam, ndc, hops, flag, tr) = traced
    for q in range(w.nq):
        c = tr["count"][q]
        assert c == min(64, max(0, (hops[q] - 1) // 4))   # checkpoints at 4, 8, ... < H
        for t in range(c):
            h = tr["hop"][q, t]
            assert h == 4 * (t + 1)
            f = tr["feat"][q, t]
            assert f[0] == pytest.approx(math.log1p(h) / 8)
            assert 0.0 <= f[3] <= 1.0 and 0.0 <= f[6] <= 1.0 and 0.0 <= f[7] <= 1.0
            assert f[1] >= 0.0


def test_selectivity_feature_is_log_frequency(traced):
    w, adj, entry, (ids, gam, ndc, hops, flag, tr) = traced
    for q in range(w.nq):
        if tr["count"][q] == 0:
            continue
        want = 0.0
        for i in range(w.m):
            c = int(w.qattrs[q, i])
            if c != 255:
                cnt = int((w.attrs[:, i] == c).sum())
                want += math.log((cnt if cnt else 0.5) / w.n)
        assert tr["feat"][q, 0, 2] == pytest.approx(want / 8, abs=1e-12)


def test_kth_key_only_improves(traced):
    # the pool keeps the best keys seen, so the k-th eligible key never grows
    # while k eligible entries exist (f5 <= 0 and non-increasing)
    w, adj, entry, (ids, gam, ndc, hops, flag, tr) = traced
    for q in range(w.nq):
        c = tr["count"][q]
        f5 = tr["feat"][q, :c, 4]
        f6 = tr["feat"][q, :c, 5]
        real = f5[f5 != 1.0]
        if len(real) and real[0] != 0.0:
            continue  # first defined value is the reference: 0
        assert (real <= 1e-12).all()
        assert (f6[f5 == 1.0] == -1.0).all()


def test_fingerprint_is_the_set_of_returned_ids(traced):
    w, adj, entry, (ids, gam, ndc, hops, flag, tr) = traced
    def fmix32(h):
        h ^= h >> 16; h = (h * 0x85EBCA6B) & 0xFFFFFFFF
        h ^= h >> 13; h = (h * 0xC2B2AE35) & 0xFFFFFFFF
        return h ^ (h >> 16)
    for q in range(w.nq):
        want = sum(fmix32((int(v) + 0x9E3779B9) & 0xFFFFFFFF) for v in ids[q] if v >= 0) & 0xFFFFFFFF
        assert int(tr["final_hash"][q]) == want


def test_learned_stop_extremes(traced):
    w, adj, entry, (ids, gam, ndc, hops, flag, tr) = traced
    p = oracle.MLPRef.init(0)
    flat = np.concatenate([p[k].ravel() for k in ("W1", "b1", "W2", "b2", "W3", "b3")])
    never = flat.copy()
    never[4864] = -1e6            # stop logit always very negative
    always = flat.copy()
    always[4864] = 1e6
    a = oracle.search(adj, w.x, w.attrs, w.q, w.qattrs, 10, 96, entry, key_mode=oracle.KEY32,
                      check_every=4, mlp=never)
    assert np.array_equal(a[0], ids) and np.array_equal(a[3], hops)
    b = oracle.search(adj, w.x, w.attrs, w.q, w.qattrs, 10, 96, entry, key_mode=oracle.KEY32,
                      check_every=4, mlp=always)
    assert (b[3] == np.minimum(hops, 4)).all()


def test_learned_hop_budget_and_single_checkpoint(traced):
    # a network whose outputs are its biases: stop logit b3[0], beam output
    # b3[1].  The budget cap_factor * 2^b3[1] bounds the hops before every
    # step; mode 2 takes one checkpoint only.
    w, adj, entry, (ids, gam, ndc, hops, flag, tr) = traced
    net = np.zeros(oracle.MLPRef.SIZE if hasattr(oracle.MLPRef, "SIZE") else 4866)
    net[4864] = -1e6   # never stops by the stop logit
    net[4865] = 4.0    # beam output: 2^4 = 16
    for mode in (1, 2):
        for cf, want in ((1.0, 16), (1.5, 24), (0.5, 8)):
            o = oracle.search(adj, w.x, w.attrs, w.q, w.qattrs, 10, 96, entry, key_mode=oracle.KEY32,
                              check_every=4, mlp=net, cap_factor=cf, learned_mode=mode)
            # E = 1: one hop per step, so the search ends at exactly the budget
            # unless it has converged before (budget set at the checkpoint at hop 4)
            assert (o[3] == np.minimum(hops, max(want, 4))).all(), (mode, cf)
    # the number of checkpoints: every 4 hops (mode 1) or one (mode 2)
    o1 = oracle.search(adj, w.x, w.attrs, w.q, w.qattrs, 10, 96, entry, key_mode=oracle.KEY32,
                       check_every=4, trace_cap=64, mlp=net, cap_factor=8.0, learned_mode=1)
    o2 = oracle.search(adj, w.x, w.attrs, w.q, w.qattrs, 10, 96, entry, key_mode=oracle.KEY32,
                       check_every=4, trace_cap=64, mlp=net, cap_factor=8.0, learned_mode=2)
    assert np.array_equal(o1[3], o2[3]) and np.array_equal(o1[0], o2[0])
    reached = o2[3] > 4
    assert (o2[5]["count"][reached] == 1).all()
    assert (o1[5]["count"][reached] == np.minimum(64, (o1[3][reached] - 1) // 4)).all()


# ---- every feature pinned exactly on hand-built walks (tests/hand_walks.py)

def _run_hand(walk, key_mode):
    x = np.asarray(walk["x"], np.float32)[:, None]
    attrs = np.asarray(walk["attrs"], np.uint8)[:, None]
    adj = np.asarray(walk["adj"], np.int32)
    q = np.zeros((1, 1), np.float32)
    qa = np.zeros((1, 1), np.uint8)
    return oracle.search(adj, x, attrs, q, qa, walk["k"], walk["L"], np.asarray(walk["seeds"], np.int32),
                         n_init=len(walk["seeds"]), key_mode=key_mode, check_every=walk["check_every"],
                         trace_cap=64, expand=walk["expand"])


@pytest.mark.parametrize("walk", [hand_walks.chain(), hand_walks.wide_step(1), hand_walks.wide_step(2)],
                         ids=["chain", "wide_step_S1", "wide_step_S2"])
@pytest.mark.parametrize("key_mode", [oracle.KEY64, oracle.KEY32])
def test_features_exact_on_hand_walks(walk, key_mode):
    ids, gam, ndc, hops, flag, tr = _run_hand(walk, key_mode)
    assert ids[0].tolist() == walk["ids"]
    assert np.allclose(gam[0], walk["gamma"], rtol=1e-12)
    assert int(ndc[0]) == walk["ndc"] and int(hops[0]) == walk["hops"]
    nck = len(walk["feat"])
    assert tr["count"][0] >= nck
    assert tr["hop"][0, :nck].tolist() == walk["hop"]
    for t in range(nck):
        assert np.allclose(tr["feat"][0, t], walk["feat"][t], rtol=0, atol=1e-12), (t, tr["feat"][0, t])
        assert int(tr["hash"][0, t]) == hand_walks.fingerprint(walk["topk"][t])
    assert int(tr["final_hash"][0]) == hand_walks.fingerprint(walk["ids"])


def test_joined_counts_survivors_of_the_whole_step():
    # the wide step offers 128 neighbours, of which the first 64 are all
    # pushed out by the last 64: f7 counts 64 joins, whatever the batching
    walk = hand_walks.wide_step(1)
    _, _, _, _, _, tr = _run_hand(walk, oracle.KEY32)
    assert tr["feat"][0, 0, 6] == 1.0


# ---- learned mode 3: the beam output chooses the pool size

def _bias_net(stop_bias, beam_bias):
    """A network whose outputs are its output biases (all weights zero)."""
    net = np.zeros(4866)
    net[4864] = stop_bias
    net[4865] = beam_bias
    return net


def test_pool_size_predictor_on_the_chain_walk():
    # chain (tests/hand_walks.py): k = 2, L = 3, one checkpoint per hop.  With
    # beam output 0 and factor 2 the pool size is ceil(2 * 2^0) = 2 from the
    # checkpoint at H = 1: the pool v2 v0* v1 is cut to v2 v0*; expanding v2
    # offers v4(36) and v3(49), leaving v4 v3; v4 offers v5(16, mismatch)
    # -> v5 v4*; v5 offers v6(9) (v2 was visited) -> v6 v5*; v6 has no
    # neighbours.  H = 5, NDC = 6, and the only eligible entry is v6 (the
    # fixed search also returns v4, which the cut pushed out at step 3).
    walk = hand_walks.chain()
    x = np.asarray(walk["x"], np.float32)[:, None]
    attrs = np.asarray(walk["attrs"], np.uint8)[:, None]
    adj = np.asarray(walk["adj"], np.int32)
    q = np.zeros((1, 1), np.float32)
    qa = np.zeros((1, 1), np.uint8)
    seeds = np.asarray(walk["seeds"], np.int32)
    kw = dict(n_init=1, key_mode=oracle.KEY64, expand=1, check_every=1, learned_mode=3)
    ids, gam, ndc, hops, flag = oracle.search(adj, x, attrs, q, qa, 2, 3, seeds, mlp=_bias_net(-1e6, 0.0),
                                              cap_factor=2.0, **kw)
    assert ids[0].tolist() == [6, -1] and ndc[0] == 6 and hops[0] == 5
    assert gam[0][0] == pytest.approx(3.0) and np.isinf(gam[0][1])
    # a pool size of at least L leaves the search as it was
    ids, gam, ndc, hops, flag = oracle.search(adj, x, attrs, q, qa, 2, 3, seeds, mlp=_bias_net(-1e6, 0.0),
                                              cap_factor=3.0, **kw)
    assert ids[0].tolist() == walk["ids"] and ndc[0] == walk["ndc"] and hops[0] == walk["hops"]
    # the size is clamped below at k
    low = oracle.search(adj, x, attrs, q, qa, 2, 3, seeds, mlp=_bias_net(-1e6, -10.0), cap_factor=1.0, **kw)
    assert low[0][0].tolist() == [6, -1] and low[2][0] == 6 and low[3][0] == 5


def _beam_with_cut(adj, keys, seeds, L, ckpt, Lp):
    """Beam search with E = 1 written out plainly: the pool holds the L best
    (key, id) seen, the best unexpanded entry is expanded next, each vertex is
    scored once; before the step that follows hop `ckpt` the pool is cut to
    its Lp best entries and holds Lp from then on.  Returns the final pool
    (ids), NDC and H."""
    pool = sorted(set(int(s) for s in seeds), key=lambda v: (keys[v], v))[:L]
    seen = set(pool)
    expanded = set()
    cap, ndc, hops, cut = L, 0, 0, False
    while True:
        if not cut and hops >= ckpt:
            cut = True
            cap = min(cap, Lp)
            pool = pool[:cap]
        nxt = [v for v in pool if v not in expanded]
        if not nxt:
            break
        u = nxt[0]
        expanded.add(u)
        hops += 1
        for v in adj[u]:
            if v < 0 or v in seen:
                continue
            seen.add(v)
            ndc += 1
            pool.append(int(v))
            pool.sort(key=lambda t: (keys[t], t))
            pool = pool[:cap]
    return pool, ndc, hops


@pytest.mark.parametrize("Lp", [10, 13, 24, 40])
def test_pool_size_predictor_matches_a_plain_beam_search_with_a_cut(Lp):
    # integer data (every key exact in FP64), E = 1, one checkpoint at H = 3
    w = synth.small(1500, 8, 25, seed=202, integer=True, n_centres=5)
    adj = oracle.build_graph(w.x, w.attrs, l=24, R=12)
    entry = oracle.entry_points(5, w.n, 64)
    L, k, ce = 40, 10, 3
    beam_bias = math.log2(Lp)          # pool size ceil(2^log2(Lp)) = Lp
    ids, gam, ndc, hops, flag = oracle.search(adj, w.x, w.attrs, w.q, w.qattrs, k, L, entry, n_init=4,
                                              key_mode=oracle.KEY64, out_mode=1, check_every=ce,
                                              mlp=_bias_net(-1e6, beam_bias), cap_factor=1.0, learned_mode=3)
    for i in range(w.nq):
        con = w.qattrs[i] != 255
        mq = int(con.sum())
        d2 = ((w.x.astype(np.float64) - w.q[i].astype(np.float64)) ** 2).sum(1)
        chi = (w.attrs[:, con] != w.qattrs[i][con]).sum(1)
        keys = d2 * (mq + chi) ** 2 if mq else d2
        seeds = sorted(entry.tolist(), key=lambda v: (keys[v], v))[:4]
        pool, rndc, rhops = _beam_with_cut(adj, keys, seeds, L, ce, max(Lp, k))
        assert ids[i].tolist() == pool[:k] and ndc[i] == rndc and hops[i] == rhops, i
