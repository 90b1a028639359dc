"""Pins of the oracle's composite-index build (Alg. 1 in degree-bounded
form, edge selection of Sec. 4.1 with the landing zone of Def. 7, Gamma in
the build per Sec. 5.1) and of graph quality (Def. 8, Eq. 7)."""
import json
import os

import numpy as np
import pytest
from scipy.spatial.distance import cdist
from sklearn.neighbors import NearestNeighbors

import oracle
import synth
from tests.conftest import GOLDEN


def test_example6_landing_zone_selection():
    with open(os.path.join(GOLDEN, "ex6_landing_zone.json")) as f:
        g = json.load(f)
    names = list(g["candidates"].keys())
    pts = np.array([g["u_i"]] + [g["candidates"][n] for n in names], np.float32)
    attrs = np.zeros((len(pts), 2), np.uint8)
    adj = oracle.build_graph(pts, attrs, l=len(names), R=g["max_degree"], rows=np.array([0]))
    got = [names[v - 1] for v in adj[0] if v >= 0]
    assert got == g["expected_neighbours"]


def _fusion_matrix(x, attrs):
    """(m Gamma)^2 for all pairs from scipy distances and numpy equality."""
    m = attrs.shape[1]
    D2 = cdist(x.astype(np.float64), x.astype(np.float64), "sqeuclidean")
    C = (attrs[:, None, :] != attrs[None, :, :]).sum(-1)
    return D2 * (m + C) ** 2


def test_candidates_are_exact_l_nearest():
    w = synth.small(600, 8, 1, seed=21)
    adj, cand = oracle.build_graph(w.x, w.attrs, l=24, R=8, want_cand=True)
    K = _fusion_matrix(w.x, w.attrs)
    for i in range(w.n):
        order = [j for j in np.lexsort((np.arange(w.n), K[i])) if j != i][:24]
        assert cand[i].tolist() == order
    # without attributes in play the candidates are the plain k-NN lists
    attrs0 = np.zeros_like(w.attrs)
    _, cand0 = oracle.build_graph(w.x, attrs0, l=10, R=4, want_cand=True)
    nn = NearestNeighbors(n_neighbors=11, algorithm="brute").fit(w.x.astype(np.float64))
    _, ri = nn.kneighbors(w.x.astype(np.float64))
    assert (cand0 == ri[:, 1:]).all()


def test_every_kept_and_rejected_candidate_obeys_def7():
    w = synth.small(500, 6, 1, seed=22)
    l, R = 30, 12
    adj, cand = oracle.build_graph(w.x, w.attrs, l=l, R=R, want_cand=True)
    K = _fusion_matrix(w.x, w.attrs)
    for i in range(w.n):
        kept = [v for v in adj[i] if v >= 0]
        assert len(set(kept)) == len(kept) and i not in kept
        # kept edges appear in candidate order
        pos = [cand[i].tolist().index(v) for v in kept]
        assert pos == sorted(pos)
        sel = []
        for p in cand[i]:
            if len(sel) == R:
                break
            inside = all(K[p, i] < K[p, j] for j in sel)   # p in every L(i, j)
            if p in kept:
                assert inside
                sel.append(p)
            else:
                assert not inside
        assert sel == kept


def test_rng_edges_are_kept_when_uncapped():
    # Every edge of the relative neighbourhood graph (Def. 6) whose far end is
    # among the candidates survives the landing-zone selection (uncapped).
    w = synth.small(160, 3, 1, seed=23)
    attrs = np.zeros_like(w.attrs)
    n = w.n
    adj = oracle.build_graph(w.x, attrs, l=n - 1, R=n - 1)
    D = cdist(w.x.astype(np.float64), w.x.astype(np.float64))
    for i in range(n):
        for j in range(n):
            if i == j:
                continue
            blocked = any(max(D[i, k], D[k, j]) < D[i, j] for k in range(n) if k != i and k != j)
            # Def. 6 wording: edge iff no k is closer to both ends than they are to each other
            if not blocked:
                assert j in adj[i].tolist(), (i, j)


def test_reverse_pass_rows_are_valid_selections():
    w = synth.small(400, 6, 1, seed=24)
    R = 8
    fwd = oracle.build_graph(w.x, w.attrs, l=16, R=R)
    rev = oracle.build_graph(w.x, w.attrs, l=16, R=R, reverse=True)
    K = _fusion_matrix(w.x, w.attrs)
    into = [set() for _ in range(w.n)]
    for i in range(w.n):
        for v in fwd[i]:
            if v >= 0:
                into[v].add(i)
    for j in range(w.n):
        pool = sorted(set(int(v) for v in fwd[j] if v >= 0) | into[j], key=lambda v: (K[j, v], v))
        sel = []
        for p in pool:
            if len(sel) == R:
                break
            if all(K[p, j] < K[p, s] for s in sel):
                sel.append(p)
        assert [int(v) for v in rev[j] if v >= 0] == sel
    # reverse edges only add reachability: in-degree coverage grows
    assert (rev >= 0).sum() >= (fwd >= 0).sum() * 0.9


def test_rows_subset_matches_full_build():
    w = synth.small(700, 10, 1, seed=25)
    full = oracle.build_graph(w.x, w.attrs, l=20, R=10)
    rows = np.array([0, 5, 699, 123])
    part = oracle.build_graph(w.x, w.attrs, l=20, R=10, rows=rows)
    assert (part == full[rows]).all()


def test_graph_quality_eq7():
    w = synth.small(300, 5, 1, seed=26)
    rows = np.arange(w.n)
    knn = oracle.knn_rows(w.x, w.attrs, rows, 10)
    assert oracle.graph_quality(knn, knn) == 1.0
    half = knn.copy()
    half[:, 5:] = -1
    assert oracle.graph_quality(half, knn) == pytest.approx(0.5)
    # vector-only kNN against sklearn
    knn_v = oracle.knn_rows(w.x, w.attrs, rows, 6, use_attrs=False)
    nn = NearestNeighbors(n_neighbors=7, algorithm="brute").fit(w.x.astype(np.float64))
    _, ri = nn.kneighbors(w.x.astype(np.float64))
    assert (knn_v == ri[:, 1:]).all()
