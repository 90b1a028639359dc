"""Pins of the oracle's joint pruning (Alg. 2) in beam form, of its output
rule (Def. 4) and of the literal form on the Example 2 graph."""
import json
import os

import numpy as np
import pytest

import oracle
import synth
from tests.conftest import GOLDEN


def _ex2():
    with open(os.path.join(GOLDEN, "ex2_joint_pruning.json")) as f:
        g = json.load(f)
    names = [v["name"] for v in g["vertices"]]
    idx = {nm: i for i, nm in enumerate(names)}
    x = np.array([v["vec"] for v in g["vertices"]], np.float32)
    attrs = np.array([v["attrs"] for v in g["vertices"]], np.uint8)
    R = max(len(v) for v in g["neighbours"].values())
    adj = np.full((len(names), R), -1, np.int32)
    for nm, nb in g["neighbours"].items():
        adj[idx[nm], : len(nb)] = [idx[b] for b in nb]
    q = np.array([g["query"]["vec"]], np.float32)
    qa = np.array([g["query"]["attrs"]], np.uint8)
    return g, names, idx, x, attrs, adj, q, qa


def test_example2_fixture_gammas():
    g, names, idx, x, attrs, adj, q, qa = _ex2()
    for v in g["vertices"]:
        i = idx[v["name"]]
        dl = oracle.delta(q[0], x[i])
        c = oracle.chi(qa[0], attrs[i])
        assert oracle.gamma(dl, c, g["m"]) == pytest.approx(v["gamma"], abs=1e-6)  # float32 inputs


def test_example2_literal_walk():
    g, names, idx, x, attrs, adj, q, qa = _ex2()
    gam = {i: oracle.gamma(oracle.delta(q[0], x[i]), oracle.chi(qa[0], attrs[i]), g["m"])
           for i in range(len(names))}
    nb = {i: [int(v) for v in adj[i] if v >= 0] for i in range(len(names))}
    res, order = oracle.alg2_literal(nb, gam.__getitem__, [idx[s] for s in g["seeds"]], g["k"])
    assert [names[v] for v in res] == g["expected_result"]
    assert [names[v] for v in order] == g["expected_expansions"]
    assert not set(g["never_expanded"]) & set(names[v] for v in order)
    # vector distance alone would expand u1 (delta 0.4 < 0.5) right after u0:
    # the attribute term is what prunes it
    dl = {i: oracle.delta(q[0], x[i]) for i in range(len(names))}
    _, order_v = oracle.alg2_literal(nb, dl.__getitem__, [idx["u0"]], 1)
    assert names[order_v[1]] == "u1"


def test_example2_beam_form_agrees_with_literal():
    g, names, idx, x, attrs, adj, q, qa = _ex2()
    seeds = np.array([idx[s] for s in g["seeds"]], np.int32)
    ids, gam, ndc, hops, flag = oracle.search(adj, x, attrs, q, qa, k=1, L=1, seeds=seeds, n_init=1)
    assert names[ids[0, 0]] == "u5"
    assert hops[0] == 3                     # u0, u4, u5
    assert gam[0, 0] == pytest.approx(0.1414213562373095, abs=1e-6)
    # neighbour evaluations: u1..u4, then u5, then u6 (the seed is not counted)
    assert ndc[0] == 6


def test_complete_graph_gives_exact_answer():
    w = synth.small(300, 8, 30, seed=31)
    n = w.n
    adj = np.array([[j for j in range(n) if j != i] for i in range(n)], np.int32)
    seeds = oracle.entry_points(5, n, 4)
    gt, gd, _ = oracle.bruteforce(w.x, w.attrs, w.q, w.qattrs, 10)
    ids, gam, ndc, hops, _ = oracle.search(adj, w.x, w.attrs, w.q, w.qattrs, 10, n, seeds, n_init=4)
    assert (ids == gt).all()
    fin = np.isfinite(gd)
    assert np.allclose(gam[fin], gd[fin], rtol=1e-12)
    assert (ndc == n - 4).all()             # every vertex but the seeds scored once


def test_exhaustive_beam_reaches_every_answer():
    # L >= |V| on a connected graph: the search scores every vertex, so the
    # answer is exact (recall 1) whatever the graph looks like.
    w = synth.small(400, 12, 25, seed=32, wildcard_arity=True)
    adj = synth.random_graph(w.n, 6, seed=3)
    adj[:, 0] = (np.arange(w.n) + 1) % w.n   # a ring makes every vertex reachable
    seeds = oracle.entry_points(9, w.n, 32)
    gt, gd, _ = oracle.bruteforce(w.x, w.attrs, w.q, w.qattrs, 10)
    ids, gam, ndc, _, _ = oracle.search(adj, w.x, w.attrs, w.q, w.qattrs, 10, 512, seeds)
    rec = oracle.recall(ids, w.x, w.attrs, w.q, w.qattrs, gt, gd, 10)
    assert rec.min() == 1.0
    assert (ndc == w.n - 32).all()


def test_row_order_does_not_change_results():
    # The pool keeps the L best of (pool + batch), so the order in which one
    # vertex's neighbours are scored changes nothing (ids, NDC, hops).
    w = synth.small(2000, 16, 30, seed=33)
    adj = synth.random_graph(w.n, 16, seed=4, pad_frac=0.3)
    rng = np.random.default_rng(0)
    adj2 = adj.copy()
    for r in adj2:
        rng.shuffle(r)
    seeds = oracle.entry_points(1, w.n)
    a = oracle.search(adj, w.x, w.attrs, w.q, w.qattrs, 10, 48, seeds)
    b = oracle.search(adj2, w.x, w.attrs, w.q, w.qattrs, 10, 48, seeds)
    for u, v in zip(a[:4], b[:4]):
        assert np.array_equal(u, v)


def test_output_rule_and_raw_mode():
    w = synth.small(3000, 16, 40, seed=34)
    adj = oracle.build_graph(w.x, w.attrs, l=32, R=16)
    seeds = oracle.entry_points(2, w.n)
    ids, gam, _, _, _ = oracle.search(adj, w.x, w.attrs, w.q, w.qattrs, 10, 64, seeds)
    raw, rgam, _, _, _ = oracle.search(adj, w.x, w.attrs, w.q, w.qattrs, 10, 64, seeds, out_mode=1)
    for i in range(w.nq):
        for v, gv in zip(ids[i], gam[i]):
            if v >= 0:   # Def. 4: every returned object matches the query
                assert oracle.chi(w.qattrs[i], w.attrs[v]) == 0
                assert gv == pytest.approx(oracle.delta(w.q[i], w.x[v]), rel=1e-12)
        g = [x for x in gam[i] if np.isfinite(x)]
        assert g == sorted(g)
        rg = rgam[i]
        assert list(rg) == sorted(rg)       # raw mode: first k by Gamma

def test_entry_sample_seeds_the_pool_with_its_best_members():
    # The initial pool (seed set B) is the n_init best of the entry sample:
    # with no edges at all, the answer is exactly the best matches inside the
    # sample, so it equals the brute-force answer over the sample alone.
    w = synth.small(3000, 16, 30, seed=38)
    adj = np.full((w.n, 4), -1, np.int32)
    entry = oracle.entry_points(11, w.n, 500)
    ids, gam, ndc, hops, _ = oracle.search(adj, w.x, w.attrs, w.q, w.qattrs, 5, 200, entry, n_init=200)
    sub_ids, sub_d, _ = oracle.bruteforce(w.x[entry], w.attrs[entry], w.q, w.qattrs, 5)
    want = np.where(sub_ids >= 0, entry[np.maximum(sub_ids, 0)], -1)
    assert (ids == want).all()
    assert (ndc == 0).all() and (hops == 200).all()


def test_key32_matches_key64_on_integer_data_without_near_ties():
    w = synth.small(3000, 32, 40, seed=35, integer=True)
    adj = synth.random_graph(w.n, 16, seed=5)
    seeds = oracle.entry_points(3, w.n)
    a = oracle.search(adj, w.x, w.attrs, w.q, w.qattrs, 10, 64, seeds, key_mode=oracle.KEY64)
    b = oracle.search(adj, w.x, w.attrs, w.q, w.qattrs, 10, 64, seeds, key_mode=oracle.KEY32)
    # keys below 2^24 are exact in float: both modes take identical decisions
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[2], b[2])


def test_hop_cap_sets_flag():
    w = synth.small(500, 8, 3, seed=36)
    adj = synth.random_graph(w.n, 8, seed=6)
    seeds = oracle.entry_points(4, w.n)
    ids, _, _, hops, flag = oracle.search(adj, w.x, w.attrs, w.q, w.qattrs, 5, 32, seeds, max_hops=3)
    assert (ids >= -1).all()
    assert (hops == 3).all() and (flag == 1).all()


def test_rerank_uses_the_exact_vectors():
    # scoring with perturbed vectors, re-scoring the first 4k from the exact
    # copy: returned distances are exact deltas and sorted
    w = synth.small(2000, 16, 20, seed=37)
    adj = oracle.build_graph(w.x, w.attrs, l=32, R=16)
    seeds = oracle.entry_points(5, w.n)
    xs = w.x + np.random.default_rng(1).normal(0, 0.05, w.x.shape).astype(np.float32)
    ids, gam, _, _, _ = oracle.search(adj, xs, w.attrs, w.q, w.qattrs, 10, 64, seeds,
                                      rerank_n=40, xr=w.x)
    for i in range(w.nq):
        for v, gv in zip(ids[i], gam[i]):
            if v >= 0:
                assert gv == pytest.approx(oracle.delta(w.q[i], w.x[v]), rel=1e-12)
        g = [x for x in gam[i] if np.isfinite(x)]
        assert g == sorted(g)


def test_multi_expansion_is_exhaustive_with_a_large_beam():
    w = synth.small(400, 12, 25, seed=39, wildcard_arity=True)
    adj = synth.random_graph(w.n, 6, seed=3)
    adj[:, 0] = (np.arange(w.n) + 1) % w.n
    seeds = oracle.entry_points(9, w.n, 32)
    gt, gd, _ = oracle.bruteforce(w.x, w.attrs, w.q, w.qattrs, 10)
    for E in (1, 2, 5):
        ids, gam, ndc, hops, _ = oracle.search(adj, w.x, w.attrs, w.q, w.qattrs, 10, 512, seeds,
                                               expand=E)
        assert oracle.recall(ids, w.x, w.attrs, w.q, w.qattrs, gt, gd, 10).min() == 1.0
        assert (ndc == w.n - 32).all() and (hops == w.n).all()


def test_example2_with_two_expansions_per_step():
    g, names, idx, x, attrs, adj, q, qa = _ex2()
    seeds = np.array([idx[s] for s in g["seeds"]], np.int32)
    ids, gam, ndc, hops, flag = oracle.search(adj, x, attrs, q, qa, k=1, L=2, seeds=seeds, n_init=1,
                                              expand=2)
    assert names[ids[0, 0]] == "u5"
