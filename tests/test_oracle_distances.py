"""Pins of the oracle's distances: chi (Eq. 4-5), delta (Eq. 1), Gamma
(Eq. 6 with the default weights of Sec. 3.2) and the ordering keys.

Each check compares the oracle with something other than itself: a library
routine, exact integer arithmetic, or a property the paper states."""
import itertools
import json
import math
import os

import numpy as np
import pytest
from scipy.spatial import distance as spd

import oracle
from tests.conftest import GOLDEN


def test_splitmix64_published_outputs():
    with open(os.path.join(GOLDEN, "splitmix64.json")) as f:
        g = json.load(f)
    for case in g["cases"]:
        gen = oracle.splitmix64(case["seed"])
        if "outputs_hex" in case:
            want = [int(h, 16) for h in case["outputs_hex"]]
        else:
            want = [int(s) for s in case["outputs_dec"]]
        got = [next(gen) for _ in want]
        assert got == want


def test_entry_points_distinct_in_range():
    for n in (1, 5, 31, 32, 33, 1000, 10**6):
        s = oracle.entry_points(12345, n, 32)
        assert len(s) == min(32, n)
        assert len(set(s.tolist())) == len(s)
        assert s.min() >= 0 and s.max() < n
    # the list is a prefix-stable function of the seed
    a = oracle.entry_points(7, 10**6, 32)
    b = oracle.entry_points(7, 10**6, 16)
    assert (a[:16] == b).all()


def test_chi_is_hamming_distance_on_full_constraints():
    # For two objects (every attribute constrained) chi is the Hamming
    # distance of the code vectors: scipy computes it independently.
    rng = np.random.default_rng(0)
    for m in (1, 2, 3, 4):
        for _ in range(200):
            a = rng.integers(0, 4, size=m).astype(np.uint8)
            b = rng.integers(0, 4, size=m).astype(np.uint8)
            assert oracle.chi(a, b) == round(spd.hamming(a, b) * m)


def test_chi_wildcards_exhaustive():
    # Exhaustive over m <= 3, cardinality 3, every wildcard pattern:
    # chi = 0 exactly when the object satisfies the constraint (Def. 4), chi
    # never exceeds the arity, chi is a metric on the constrained positions.
    card = 3
    for m in (1, 2, 3):
        codes = list(itertools.product(range(card), repeat=m))
        qcodes = list(itertools.product(list(range(card)) + [255], repeat=m))
        for qa in qcodes:
            mq = oracle.arity(qa)
            assert mq == sum(1 for c in qa if c != 255)
            for ea in codes:
                c = oracle.chi(qa, ea)
                match = all(qq == 255 or qq == ee for qq, ee in zip(qa, ea))
                assert (c == 0) == match
                assert 0 <= c <= mq
    # triangle inequality of the Hamming metric (full constraints)
    codes = list(itertools.product(range(2), repeat=3))
    for a, b, c in itertools.product(codes, repeat=3):
        assert oracle.chi(a, c) <= oracle.chi(a, b) + oracle.chi(b, c)


def test_delta_matches_library_and_exact_integers():
    rng = np.random.default_rng(1)
    for d in (1, 2, 7, 128, 960):
        x = rng.standard_normal(d).astype(np.float32)
        y = rng.standard_normal(d).astype(np.float32)
        assert oracle.delta(x, y) == pytest.approx(spd.euclidean(x.astype(np.float64), y.astype(np.float64)), rel=1e-13)
        xi = rng.integers(0, 256, size=d)
        yi = rng.integers(0, 256, size=d)
        exact = sum(int(a - b) ** 2 for a, b in zip(xi, yi))
        got = oracle.delta(xi.astype(np.float32), yi.astype(np.float32)) ** 2
        assert abs(got - exact) <= 1e-9 * max(1, exact)
    # delta2 on integer data is the exact integer (no rounding at all)
    xi = np.full(128, 255, np.float32)
    yi = np.zeros(128, np.float32)
    assert oracle.lib().or_delta2(xi.ctypes.data, yi.ctypes.data, 128) == 255 * 255 * 128


def test_gamma_properties_from_the_paper():
    rng = np.random.default_rng(2)
    for _ in range(2000):
        mq = int(rng.integers(1, 5))
        dl = float(rng.uniform(0, 100))
        # an exact attribute match leaves the vector distance unchanged
        assert oracle.gamma(dl, 0, mq) == dl
        prev = -1.0
        for c in range(mq + 1):
            g = oracle.gamma(dl, c, mq)
            # delta <= Gamma <= 2 delta with the default weights
            assert dl <= g <= 2 * dl * (1 + 1e-15)
            # Gamma grows with the mismatch count (strictly when delta > 0)
            assert g > prev
            prev = g
        # a full mismatch doubles the distance
        assert oracle.gamma(dl, mq, mq) == pytest.approx(2 * dl, rel=1e-15)
    # no constrained attribute: Gamma is delta
    assert oracle.gamma(3.5, 0, 0) == 3.5
    # delta = 0 gives Gamma = 0 whatever chi is (the weight w_l = delta/m)
    assert oracle.gamma(0.0, 2, 3) == 0.0


def test_order_key_orders_like_gamma():
    # key = delta^2 (m_q + chi)^2 = (m_q Gamma)^2 is a monotone transform of
    # Gamma; check against Gamma computed by the oracle on random pairs.
    rng = np.random.default_rng(3)
    for mq in (0, 1, 2, 3, 4):
        pts = []
        for _ in range(400):
            d2 = float(rng.integers(0, 10**6))
            c = int(rng.integers(0, mq + 1))
            pts.append((d2, c))
        for (a2, ca), (b2, cb) in zip(pts[::2], pts[1::2]):
            ga = oracle.gamma(math.sqrt(a2), ca, mq)
            gb = oracle.gamma(math.sqrt(b2), cb, mq)
            ka = oracle.order_key(a2, ca, mq)
            kb = oracle.order_key(b2, cb, mq)
            if abs(ga - gb) > 1e-9 * max(ga, gb, 1.0):
                assert (ga < gb) == (ka < kb)


def test_key32_is_one_float_multiply():
    # On integer delta^2 below 2^24 the float key is a single correctly
    # rounded float32 product; numpy's float32 multiply computes the same.
    rng = np.random.default_rng(4)
    for _ in range(5000):
        d2 = int(rng.integers(0, 1 << 24))
        mq = int(rng.integers(0, 5))
        c = int(rng.integers(0, mq + 1))
        mult = 1 if mq == 0 else (mq + c) ** 2
        want = float(np.float32(d2) * np.float32(mult))
        assert oracle.order_key(float(d2), c, mq, oracle.KEY32) == want
        assert oracle.order_key(float(d2), c, mq, oracle.KEY64) == float(d2 * mult)
