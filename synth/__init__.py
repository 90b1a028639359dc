"""Seeded synthetic workloads for native hybrid queries.

This module only draws random inputs: feature vectors, ordinal attribute
codes, query vectors, query constraints, arrival times and (for tests that
need a graph that no builder produced) random adjacency lists.  It holds
none of the method's arithmetic: no distance, no attribute distance, no
ordering.  Both the CPU oracle side and the GPU side of the tests, the
benchmark and the smoke check draw their inputs from here.

Shapes follow the paper's setting: an object set of n objects, each with a
d-dimensional feature vector and m ordinal-encoded attributes (Def. 1 and
the ordinal encoding of Sec. 3.2).  A query carries a vector and one code
per attribute; the code 0xFF marks an unconstrained attribute (wildcard).

All generators use ``numpy.random.default_rng(seed)``; vectors are drawn in
fixed-size chunks so that a workload is identical on every machine.
"""
from __future__ import annotations

import dataclasses
from typing import Optional, Sequence, Tuple

import numpy as np

WILDCARD = 0xFF
_CHUNK = 1 << 16  # rows per generation chunk (fixed: part of the recipe)


@dataclasses.dataclass
class Workload:
    name: str
    x: np.ndarray          # float32 [n, d] feature vectors
    attrs: np.ndarray      # uint8   [n, m] ordinal attribute codes
    cards: Tuple[int, ...]  # cardinality of each attribute
    q: np.ndarray          # float32 [nq, d] query vectors
    qattrs: np.ndarray     # uint8   [nq, m] query codes, WILDCARD = unconstrained
    k: int
    beams: Tuple[int, ...]
    degree: int            # graph out-degree R
    cand: int              # candidate-list size l of the edge selection
    build_seed: int        # seed of the index build (entry-point list)
    integer: bool          # vectors hold small non-negative integers

    @property
    def n(self) -> int:
        return int(self.x.shape[0])

    @property
    def d(self) -> int:
        return int(self.x.shape[1])

    @property
    def m(self) -> int:
        return int(self.attrs.shape[1])

    @property
    def nq(self) -> int:
        return int(self.q.shape[0])


# --------------------------------------------------------------------------
# vectors
# --------------------------------------------------------------------------
def gaussian_mixture(n: int, d: int, n_centres: int, seed: int,
                     centre_std: float = 2.0, noise_std: float = 1.0,
                     centres: Optional[np.ndarray] = None,
                     centre_seed: Optional[int] = None) -> np.ndarray:
    """n points x = mu_z + noise_std * N(0, I), z uniform over the centres,
    centres mu ~ N(0, centre_std^2 I) drawn from ``centre_seed`` (defaults to
    ``seed``).  Queries pass the same centre_seed as the base set so that
    they come from the same mixture."""
    if centres is None:
        crng = np.random.default_rng(centre_seed if centre_seed is not None else seed)
        centres = (crng.standard_normal((n_centres, d), dtype=np.float32)
                   * np.float32(centre_std))
    rng = np.random.default_rng(seed + 7919)
    out = np.empty((n, d), dtype=np.float32)
    for s in range(0, n, _CHUNK):
        e = min(n, s + _CHUNK)
        z = rng.integers(0, n_centres, size=e - s)
        out[s:e] = centres[z]
        out[s:e] += rng.standard_normal((e - s, d), dtype=np.float32) * np.float32(noise_std)
    return out


def integer_clusters(n: int, d: int, n_centres: int, seed: int, sigma: float,
                     centre_seed: int) -> np.ndarray:
    """Clustered vectors holding integers in [0, 255] (the value range of
    SIFT-like descriptors): centre coordinates round(255 * Beta(0.5, 2)),
    points clip(round(c_z + N(0, sigma^2)), 0, 255), stored as float32."""
    crng = np.random.default_rng(centre_seed)
    centres = np.round(255.0 * crng.beta(0.5, 2.0, size=(n_centres, d))).astype(np.float32)
    rng = np.random.default_rng(seed + 7919)
    out = np.empty((n, d), dtype=np.float32)
    for s in range(0, n, _CHUNK):
        e = min(n, s + _CHUNK)
        z = rng.integers(0, n_centres, size=e - s)
        v = centres[z] + rng.standard_normal((e - s, d), dtype=np.float32) * np.float32(sigma)
        np.clip(np.rint(v), 0.0, 255.0, out=out[s:e])
    return out


# --------------------------------------------------------------------------
# attributes
# --------------------------------------------------------------------------
def uniform_attrs(n: int, cards: Sequence[int], seed: int) -> np.ndarray:
    rng = np.random.default_rng(seed)
    a = np.empty((n, len(cards)), dtype=np.uint8)
    for i, c in enumerate(cards):
        a[:, i] = rng.integers(0, c, size=n)
    return a


def zipf_attrs(n: int, cards: Sequence[int], seed: int, s: float = 1.1) -> np.ndarray:
    """Code r-1 with probability proportional to r^-s, r = 1..card, drawn
    independently per attribute."""
    rng = np.random.default_rng(seed)
    a = np.empty((n, len(cards)), dtype=np.uint8)
    for i, c in enumerate(cards):
        p = np.arange(1, c + 1, dtype=np.float64) ** (-s)
        p /= p.sum()
        a[:, i] = rng.choice(c, size=n, p=p)
    return a


def partial_constraints(nq: int, cards: Sequence[int], seed: int,
                        arity: Optional[Sequence[int]] = None) -> np.ndarray:
    """Queries that constrain a random subset of the attributes: arity r
    uniform over ``arity`` (default 1..m), the subset uniform among the
    C(m, r) subsets, values uniform; the rest are wildcards."""
    m = len(cards)
    arity = tuple(arity) if arity is not None else tuple(range(1, m + 1))
    rng = np.random.default_rng(seed)
    qa = np.full((nq, m), WILDCARD, dtype=np.uint8)
    r = rng.choice(np.asarray(arity), size=nq)
    for i in range(nq):
        sub = rng.permutation(m)[: r[i]]
        for j in sub:
            qa[i, j] = rng.integers(0, cards[j])
    return qa


# --------------------------------------------------------------------------
# graphs and streams that no builder made (for search-only tests)
# --------------------------------------------------------------------------
def random_graph(n: int, degree: int, seed: int, pad_frac: float = 0.0) -> np.ndarray:
    """int32 [n, degree] adjacency: each row holds ``degree`` distinct ids
    other than its own, drawn uniformly; when ``pad_frac`` > 0 a random
    number (up to pad_frac * degree) of trailing slots per row is padding
    (-1).  Requires n > degree."""
    if n <= degree:
        raise ValueError("random_graph needs n > degree")
    rng = np.random.default_rng(seed)
    adj = np.empty((n, degree), dtype=np.int32)
    for s in range(0, n, _CHUNK):
        e = min(n, s + _CHUNK)
        own = np.arange(s, e, dtype=np.int64)[:, None]
        v = rng.integers(0, n - 1, size=(e - s, degree), dtype=np.int64)
        v += (v >= own)                      # skip the row's own id
        while True:                           # redraw repeated ids
            srt = np.sort(v, axis=1)
            dup_rows = np.nonzero((srt[:, 1:] == srt[:, :-1]).any(axis=1))[0]
            if dup_rows.size == 0:
                break
            for r in dup_rows:
                _, first = np.unique(v[r], return_index=True)
                mask = np.ones(degree, dtype=bool)
                mask[first] = False
                w = rng.integers(0, n - 1, size=int(mask.sum()), dtype=np.int64)
                v[r, mask] = w + (w >= own[r, 0])
        adj[s:e] = v
    if pad_frac > 0.0:
        npad = rng.integers(0, int(round(degree * pad_frac)) + 1, size=n)
        cols = np.arange(degree)[None, :]
        adj[cols >= (degree - npad)[:, None]] = -1
    return adj


def poisson_arrivals(n: int, rate_per_s: float, seed: int) -> np.ndarray:
    """Arrival times in seconds of a Poisson stream (exponential gaps)."""
    rng = np.random.default_rng(seed)
    return np.cumsum(rng.exponential(1.0 / rate_per_s, size=n))


# --------------------------------------------------------------------------
# the five workloads
# --------------------------------------------------------------------------
CONFIG2_SIGMA = 19.5  # within-cluster spread: median 20-NN distance ~230 at n = 1M


def config1(n: int = 10_000, nq: int = 100) -> Workload:
    """Plain method, small: 16-component Gaussian mixture, d = 128,
    3 uniform attributes of cardinality 3/4/5, full constraints."""
    cards = (3, 4, 5)
    x = gaussian_mixture(n, 128, 16, seed=101, centre_seed=1101)
    a = uniform_attrs(n, cards, 102)
    q = gaussian_mixture(nq, 128, 16, seed=103, centre_seed=1101)
    qa = uniform_attrs(nq, cards, 104)
    return Workload("config1-gmm16-n%d-d128" % n, x, a, cards, q, qa, k=10,
                    beams=(64,), degree=32, cand=64, build_seed=105, integer=False)


def config2(n: int = 1_000_000, nq: int = 10_000) -> Workload:
    """Plain method at scale: integer-valued d = 128 vectors from 256
    clusters (SIFT-like value range), attributes 3/4/5 uniform, full
    constraints, beam sweep 32..512."""
    cards = (3, 4, 5)
    x = integer_clusters(n, 128, 256, seed=201, sigma=CONFIG2_SIGMA, centre_seed=1201)
    a = uniform_attrs(n, cards, 202)
    q = integer_clusters(nq, 128, 256, seed=203, sigma=CONFIG2_SIGMA, centre_seed=1201)
    qa = uniform_attrs(nq, cards, 204)
    return Workload("config2-int256c-n%d-d128" % n, x, a, cards, q, qa, k=10,
                    beams=(32, 64, 128, 256, 512), degree=32, cand=64,
                    build_seed=205, integer=True)


def config2_train_queries(nq: int = 20_000):
    """Training queries of the config-2 distribution (same clusters and
    attribute law, seeds disjoint from the evaluation queries): for the
    stop network, which is evaluated on the held-out config-2 queries."""
    q = integer_clusters(nq, 128, 256, seed=206, sigma=CONFIG2_SIGMA, centre_seed=1201)
    qa = uniform_attrs(nq, (3, 4, 5), 207)
    return q, qa


def config3(n: int = 1_000_000, nq: int = 10_000) -> Workload:
    """Precision form: d = 960 Gaussian mixture (64 centres), 4 uniform
    attributes of cardinality 2/3/5/10, all four constrained."""
    cards = (2, 3, 5, 10)
    x = gaussian_mixture(n, 960, 64, seed=301, centre_seed=1301)
    a = uniform_attrs(n, cards, 302)
    q = gaussian_mixture(nq, 960, 64, seed=303, centre_seed=1301)
    qa = uniform_attrs(nq, cards, 304)
    return Workload("config3-gmm64-n%d-d960" % n, x, a, cards, q, qa, k=10,
                    beams=(32, 64, 128, 256, 512), degree=32, cand=64,
                    build_seed=305, integer=False)


def config3_train_queries(nq: int = 20_000):
    """Training queries of the precision-form distribution (same mixture
    and attribute law, seeds disjoint from the evaluation queries): for the
    stop network, evaluated on the held-out precision-form queries."""
    q = gaussian_mixture(nq, 960, 64, seed=306, centre_seed=1301)
    qa = uniform_attrs(nq, (2, 3, 5, 10), 307)
    return q, qa


def config4(n: int = 10_000_000, nq: int = 10_000, train: bool = False) -> Workload:
    """Learned-stop form: d = 96 Gaussian mixture (1024 centres), attributes
    3/4/5 Zipf(1.1)-skewed, full constraints with combinations drawn from
    the data distribution.  ``train`` selects the training query set."""
    cards = (3, 4, 5)
    x = gaussian_mixture(n, 96, 1024, seed=401, centre_seed=1401)
    a = zipf_attrs(n, cards, 402)
    qseed = 403 if train else 404
    q = gaussian_mixture(nq, 96, 1024, seed=qseed, centre_seed=1401)
    qa = zipf_attrs(nq, cards, qseed + 1000)
    return Workload("config4-gmm1024-zipf-n%d-d96" % n, x, a, cards, q, qa, k=10,
                    beams=(32, 64, 128, 256, 512), degree=32, cand=64,
                    build_seed=405, integer=False)


def config4_train_queries(nq: int = 200_000):
    """Training queries of the learned-stop form (same mixture and Zipf
    attribute law as its base set, the training seeds 403 / 1403)."""
    q = gaussian_mixture(nq, 96, 1024, seed=403, centre_seed=1401)
    qa = zipf_attrs(nq, (3, 4, 5), 1403)
    return q, qa


def config5_stream(nq: int, cards: Sequence[int] = (2, 3, 5, 10), d: int = 960,
                   rate_per_s: float = 50_000.0):
    """Serving stream: query vectors from the precision-form mixture,
    per-query k uniform over {1, 10, 50, 100}, constraint arity 1..4 with the
    rest wildcards, Poisson arrival times."""
    q = gaussian_mixture(nq, d, 64, seed=503, centre_seed=1301)
    qa = partial_constraints(nq, cards, 504)
    rng = np.random.default_rng(502)
    ks = rng.choice(np.array([1, 10, 50, 100], dtype=np.int32), size=nq)
    t = poisson_arrivals(nq, rate_per_s, 501)
    return q, qa, ks, t


def small(n: int, d: int, nq: int, cards: Sequence[int] = (3, 4, 5), seed: int = 7,
          integer: bool = False, n_centres: int = 8, wildcard_arity: bool = False,
          zipf: bool = False) -> Workload:
    """Small workloads for tests: same recipes at chosen sizes."""
    if integer:
        x = integer_clusters(n, d, n_centres, seed=seed, sigma=CONFIG2_SIGMA,
                             centre_seed=seed + 1000)
        q = integer_clusters(nq, d, n_centres, seed=seed + 2, sigma=CONFIG2_SIGMA,
                             centre_seed=seed + 1000)
    else:
        x = gaussian_mixture(n, d, n_centres, seed=seed, centre_seed=seed + 1000)
        q = gaussian_mixture(nq, d, n_centres, seed=seed + 2, centre_seed=seed + 1000)
    a = (zipf_attrs if zipf else uniform_attrs)(n, cards, seed + 1)
    if wildcard_arity:
        qa = partial_constraints(nq, cards, seed + 3)
    else:
        qa = (zipf_attrs if zipf else uniform_attrs)(nq, cards, seed + 3)
    return Workload("small-n%d-d%d" % (n, d), x, a, tuple(cards), q, qa, k=10,
                    beams=(64,), degree=32, cand=64, build_seed=seed + 4,
                    integer=integer)
