"""Pins of the oracle's weight settings of Eq. 6 (Sec. 6.5, Fig. 10 (i)):
hand-computed values, the properties the paper states for each setting,
the float32 key against the FP64 one, and limits in which the build and the
search reduce to something simpler."""
import math

import numpy as np
import pytest

import oracle
import synth

MODES = [("default", 0.0), ("harmonic", 0.0), ("harmonic_c", 100.0), ("normalised", 500.0),
         ("fixed", 230.0)]


def test_hand_computed_values():
    # delta = 3, chi = 2, m_q = 3
    want = {("default", 0.0): 5.0, ("harmonic", 0.0): 2.4, ("harmonic_c", 100.0): 1200.0 / 203.0,
            ("normalised", 10.0): 0.3 + 2.0 / 3.0, ("fixed", 10.0): 23.0}
    for (mode, p), g in want.items():
        with oracle.weights(mode, p):
            assert oracle.gamma(3.0, 2, 3) == pytest.approx(g, rel=1e-15)
    # chi = 0 under Eq. 8 becomes 1: 2 * 3 * 1 / (3 + 1)
    with oracle.weights("harmonic_c", 100.0):
        assert oracle.gamma(3.0, 0, 3) == pytest.approx(1.5, rel=1e-15)
    # the setting is restored after the block
    assert oracle.gamma(3.0, 2, 3) == pytest.approx(5.0, rel=1e-15)


def test_harmonic_defect_and_mean_bounds():
    # curve i: Gamma = 0 whenever chi = 0, whatever delta (the defect the
    # paper reports); otherwise a harmonic mean lies between min and max
    rng = np.random.default_rng(0)
    with oracle.weights("harmonic"):
        for dl in rng.uniform(0, 1000, 50):
            assert oracle.gamma(dl, 0, 3) == 0.0
            for c in (1, 2, 3):
                g = oracle.gamma(dl, c, 3)
                assert min(dl, c) - 1e-12 <= g <= max(dl, c) + 1e-12
    with oracle.weights("harmonic_c", 100.0):
        for dl in rng.uniform(0, 1000, 50):
            # Eq. 8: chi = 0 counts as 1, so Gamma = 2 delta / (delta + 1) < 2;
            # chi >= 1 counts as c * chi
            assert oracle.gamma(dl, 0, 3) < 2.0
            assert oracle.gamma(dl, 1, 3) == pytest.approx(200 * dl / (dl + 100), rel=1e-12)


def test_normalised_and_fixed_are_linear():
    with oracle.weights("normalised", 400.0):
        assert oracle.gamma(400.0, 3, 3) == pytest.approx(2.0)
        assert oracle.gamma(0.0, 0, 3) == 0.0
        assert oracle.gamma(200.0, 1, 0) == pytest.approx(0.5)   # no constrained attribute
    with oracle.weights("fixed", 7.0):
        for c in range(4):
            assert oracle.gamma(10.0, c, 3) - oracle.gamma(10.0, 0, 3) == pytest.approx(7.0 * c)


@pytest.mark.parametrize("mode,p", MODES)
def test_keys_order_like_gamma(mode, p):
    rng = np.random.default_rng(1)
    d2 = rng.integers(0, 200000, 400).astype(np.float64)
    c = rng.integers(0, 4, 400)
    with oracle.weights(mode, p):
        g = np.array([oracle.gamma(math.sqrt(a), int(b), 3) for a, b in zip(d2, c)])
        k64 = np.array([oracle.order_key(a, int(b), 3, oracle.KEY64) for a, b in zip(d2, c)])
        k32 = np.array([oracle.order_key(a, int(b), 3, oracle.KEY32) for a, b in zip(d2, c)])
    # the key is a monotone function of Gamma
    o = np.lexsort((np.arange(400), g))
    assert (np.diff(k64[o]) >= 0).all()
    # float32 key: Gamma rounded, within a few float32 ulps
    ref = k64 if mode == "default" else g
    assert np.allclose(k32, ref, rtol=4e-7, atol=1e-30)


def test_fixed_ratio_limit_build_and_search():
    # w_l / w_v -> infinity: chi decides first, delta second.  The build's
    # candidate lists are then the nearest objects with identical attributes
    # (when there are enough), and the search's answers rank matches first.
    w = synth.small(1200, 16, 20, seed=71, integer=True, n_centres=4, cards=(2, 3))
    with oracle.weights("fixed", 1e9):
        adj, cand = oracle.build_graph(w.x, w.attrs, l=16, R=8, want_cand=True)
    for i in range(0, w.n, 97):
        same = np.flatnonzero((w.attrs == w.attrs[i]).all(axis=1))
        same = same[same != i]
        d = ((w.x[same].astype(np.float64) - w.x[i]) ** 2).sum(1)
        want = same[np.lexsort((same, d))][:16]
        assert np.array_equal(cand[i], want), i
    entry = oracle.entry_points(3, w.n, 64)
    with oracle.weights("fixed", 1e9):
        ids, gam, _, _, _ = oracle.search(adj, w.x, w.attrs, w.q, w.qattrs, 10, 64, entry,
                                          out_mode=1)
    for i in range(w.nq):
        chis = [oracle.chi(w.qattrs[i], w.attrs[v]) for v in ids[i] if v >= 0]
        assert chis == sorted(chis)


def test_default_mode_unchanged_by_the_switch():
    w = synth.small(800, 16, 10, seed=72, integer=True)
    a = oracle.build_graph(w.x, w.attrs, l=16, R=8)
    with oracle.weights("default"):
        b = oracle.build_graph(w.x, w.attrs, l=16, R=8)
    assert np.array_equal(a, b)
