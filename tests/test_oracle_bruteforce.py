"""Pins of the exact hybrid top-k (Def. 4 with Def. 2) and of Recall@k
(Eq. 3 with the hybrid rule of Sec. 6.1)."""
import numpy as np
import pytest
from scipy.spatial.distance import cdist
from sklearn.neighbors import NearestNeighbors

import oracle
import synth


def _lexsort_answer(x, attrs, q, qa, k):
    """Independent answer: numpy equality filter, scipy distances, lexsort."""
    ids = np.full((q.shape[0], k), -1, np.int64)
    dist = np.full((q.shape[0], k), np.inf)
    D = cdist(q.astype(np.float64), x.astype(np.float64))
    for i in range(q.shape[0]):
        cons = qa[i] != 255
        ok = np.all(attrs[:, cons] == qa[i, cons], axis=1)
        cand = np.nonzero(ok)[0]
        order = np.lexsort((cand, D[i, cand]))[:k]
        ids[i, : len(order)] = cand[order]
        dist[i, : len(order)] = D[i, cand[order]]
    return ids, dist


@pytest.mark.parametrize("wild", [False, True])
def test_bruteforce_equals_filter_then_lexsort(wild):
    w = synth.small(3000, 24, 40, seed=11, wildcard_arity=wild)
    ids, dist, nm = oracle.bruteforce(w.x, w.attrs, w.q, w.qattrs, 10)
    ref_ids, ref_dist = _lexsort_answer(w.x, w.attrs, w.q, w.qattrs, 10)
    assert (ids == ref_ids).all()
    fin = np.isfinite(ref_dist)
    assert np.allclose(dist[fin], ref_dist[fin], rtol=1e-12)
    assert np.isinf(dist[~fin]).all()
    for i in range(w.nq):
        cons = w.qattrs[i] != 255
        assert nm[i] == np.all(w.attrs[:, cons] == w.qattrs[i, cons], axis=1).sum()


def test_bruteforce_ties_broken_by_id_on_integer_data():
    # integer vectors produce many equal distances: the order is (delta, id)
    w = synth.small(4000, 4, 50, seed=12, integer=True, n_centres=2)
    ids, _, _ = oracle.bruteforce(w.x, w.attrs, w.q, w.qattrs, 20)
    ref_ids, _ = _lexsort_answer(w.x, w.attrs, w.q, w.qattrs, 20)
    assert (ids == ref_ids).all()


def test_unconstrained_query_is_plain_knn():
    # arity 0 reduces the hybrid query to exact vector kNN (Def. 2)
    w = synth.small(2000, 16, 30, seed=13)
    qa = np.full_like(w.qattrs, 255)
    ids, dist, nm = oracle.bruteforce(w.x, w.attrs, w.q, qa, 7)
    nn = NearestNeighbors(n_neighbors=7, algorithm="brute").fit(w.x.astype(np.float64))
    rd, ri = nn.kneighbors(w.q.astype(np.float64))
    assert (ids == ri).all()
    assert np.allclose(dist, rd, rtol=1e-10)
    assert (nm == w.n).all()


def test_empty_and_short_answers():
    w = synth.small(500, 8, 5, seed=14)
    qa = w.qattrs.copy()
    qa[0] = [2, 3, 4]
    attrs = w.attrs.copy()
    attrs[np.all(attrs == [2, 3, 4], axis=1)] = [0, 0, 0]   # nobody matches query 0
    attrs[7] = [2, 3, 4]
    attrs[9] = [2, 3, 4]                                    # ...except two objects
    ids, dist, nm = oracle.bruteforce(w.x, attrs, w.q, qa, 10)
    assert nm[0] == 2
    assert sorted(ids[0, :2].tolist()) == [7, 9]
    assert (ids[0, 2:] == -1).all() and np.isinf(dist[0, 2:]).all()
    ids0, dist0, _ = oracle.bruteforce(w.x, attrs, w.q, qa, 0)
    assert ids0.shape == (5, 0)


def test_by_gamma_ranking_equals_knn_when_all_match():
    w = synth.small(1500, 12, 20, seed=15)
    attrs = np.zeros_like(w.attrs)
    qa = np.zeros_like(w.qattrs)
    a, _, _ = oracle.bruteforce(w.x, attrs, w.q, qa, 10, by_gamma=True)
    b, _, _ = oracle.bruteforce(w.x, attrs, w.q, qa, 10, by_gamma=False)
    assert (a == b).all()


def test_recall_hand_cases():
    # 1-D points: distances are |x|.  Query at 0, attribute constraint 0.
    x = np.array([[1.0], [2.0], [2.0], [3.0], [0.5]], np.float32)
    attrs = np.array([[0], [0], [0], [0], [1]], np.uint8)
    q = np.zeros((1, 1), np.float32)
    qa = np.zeros((1, 1), np.uint8)
    gt, gd, nm = oracle.bruteforce(x, attrs, q, qa, 2)
    assert gt[0].tolist() == [0, 1] and nm[0] == 4
    r = lambda ids: oracle.recall(np.array([ids], np.int32), x, attrs, q, qa, gt, gd, 2)[0]
    assert r([0, 1]) == 1.0
    assert r([0, 2]) == 1.0          # tie at the k-th distance counts
    assert r([1, 2]) == 1.0          # both at the k-th distance
    assert r([0, 3]) == 0.5          # farther than the k-th
    assert r([0, 4]) == 0.5          # closer but mismatched attributes (Def. 4)
    assert r([0, 0]) == 0.5          # a repeated id counts once
    assert r([-1, -1]) == 0.0
    # |P| < k: denominator is |P|
    gt3, gd3, _ = oracle.bruteforce(x, attrs, q, np.ones((1, 1), np.uint8), 3)
    assert gt3[0].tolist() == [4, -1, -1]
    assert oracle.recall(np.array([[4, 0, 1]], np.int32), x, attrs, q, np.ones((1, 1), np.uint8), gt3, gd3, 3)[0] == 1.0
