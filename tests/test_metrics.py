"""The benchmark's Recall@k (Eq. 3, hybrid rule of Sec. 6.1) against the
oracle's per-query definition, on data with ties, repeats, wildcards, short
answers and wrong returned distances (the metric must not read them)."""
import numpy as np

import oracle
import synth
from paper_2203_13601_amd import metrics


def test_recall_equals_oracle_definition():
    w = synth.small(3000, 16, 80, seed=31, integer=True, n_centres=3, wildcard_arity=True)
    gi, gd, _ = oracle.bruteforce(w.x, w.attrs, w.q, w.qattrs, 10)
    rng = np.random.default_rng(3)
    # perturbed answers: some exact ids, some random ids, repeats, padding
    ids = gi.copy()
    flip = rng.random(ids.shape) < 0.3
    ids[flip] = rng.integers(0, w.n, size=int(flip.sum()))
    ids[:, 9] = ids[:, 0]                       # a repeat in every row
    ids[rng.random(ids.shape) < 0.1] = -1
    want = oracle.recall(ids, w.x, w.attrs, w.q, w.qattrs, gi, gd, 10)
    got = metrics.recall_at_k(ids, w.x, w.q, w.attrs, w.qattrs, gi, 10)
    assert np.array_equal(got, want)
    assert np.array_equal(metrics.recall_at_k(gi, w.x, w.q, w.attrs, w.qattrs, gi, 10),
                          np.ones(w.nq))


def test_gamma_error_uses_fp64_gamma():
    w = synth.small(2000, 24, 40, seed=32, wildcard_arity=True)
    gi, gd, _ = oracle.bruteforce(w.x, w.attrs, w.q, w.qattrs, 10, by_gamma=True)
    err = metrics.gamma_rel_error(gi, gd, w.x, w.q, w.attrs, w.qattrs)
    assert err.size == (gi >= 0).sum() and err.max() < 1e-12
    bad = gd.copy()
    bad[:, 0] *= 1.001
    assert metrics.gamma_rel_error(gi, bad, w.x, w.q, w.attrs, w.qattrs).max() > 9e-4


def test_qps_at_recall_interpolates_in_log_qps():
    assert abs(metrics.qps_at_recall([1, 2], [0.9, 1.0], [100.0, 10.0], 0.95) - np.sqrt(1000.0)) < 1e-9
    assert metrics.qps_at_recall([1, 2], [0.96, 0.99], [100.0, 10.0], 0.95) == 100.0
    assert metrics.qps_at_recall([1, 2], [0.9, 0.94], [100.0, 10.0], 0.95) is None
