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
