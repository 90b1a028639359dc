"""Pins of the stratified seed sets (the flagged entry-sample option): each
block holds only its attribute pattern, is the per-pattern minimum of the
published splitmix64 hash, and a search seeded from the query's block finds
answers that a random global sample cannot reach when the graph has no edge
between patterns."""
import numpy as np

import oracle
import synth


def test_blocks_are_the_smallest_hashes_of_their_pattern():
    rng = np.random.default_rng(1)
    attrs = rng.integers(0, 3, size=(300, 2)).astype(np.uint8)
    seed, per = 77, 7
    st = oracle.entry_strata(seed, attrs, per)
    pats = {tuple(int(c) for c in r) for r in attrs}
    assert set(st) == pats
    for t, ids in st.items():
        members = [i for i in range(len(attrs)) if tuple(int(c) for c in attrs[i]) == t]
        assert all(tuple(int(c) for c in attrs[i]) == t for i in ids)
        # brute force with the scalar generator: first output from state
        # (seed ^ salt) ^ (i * C) mod 2^64
        def h(i):
            s = (seed ^ 0x8F14E45FCEEA167A) ^ ((i * 0xD1B54A32D192ED03) & 0xFFFFFFFFFFFFFFFF)
            return next(oracle.splitmix64(s))
        want = sorted(members, key=lambda i: (h(i), i))[:per]
        assert ids.tolist() == want
        assert len(ids) == min(per, len(members))


def test_pattern_blocks_reach_answers_a_global_sample_misses():
    # four patterns, each its own far-apart cluster, a graph with edges only
    # inside a pattern: a query can reach its answers only from a seed of
    # its own pattern.  The block seeds find them all (exhaustive beam); a
    # global sample drawn from the first pattern's objects alone cannot.
    rng = np.random.default_rng(2)
    npp, d = 60, 8
    x = np.concatenate([rng.standard_normal((npp, d)) + 40.0 * p for p in range(4)]).astype(np.float32)
    attrs = np.repeat(np.arange(4), npp)[:, None].astype(np.uint8)
    n = 4 * npp
    adj = np.full((n, 16), -1, np.int32)
    for p in range(4):
        ids = np.arange(p * npp, (p + 1) * npp)
        for i in ids:
            nb = rng.choice(ids[ids != i], size=16, replace=False)
            adj[i] = nb
    q = (x[rng.integers(0, n, 40)] + 0.1).astype(np.float32)
    qa = attrs[rng.integers(0, n, 40)]
    strata = oracle.entry_strata(5, attrs, 4)
    glob = np.arange(4, dtype=np.int32)            # four seeds, all of pattern 0
    gi, gd, _ = oracle.bruteforce(x, attrs, q, qa, 5)
    a = oracle.search_strata(adj, x, attrs, q, qa, 5, n, glob, strata, n_init=4)
    b = oracle.search(adj, x, attrs, q, qa, 5, n, glob, n_init=4)
    ra = oracle.recall(a[0], x, attrs, q, qa, gi, gd, 5)
    rb = oracle.recall(b[0], x, attrs, q, qa, gi, gd, 5)
    assert (ra == 1.0).all()
    assert (rb[qa[:, 0] != 0] == 0.0).all() and (rb[qa[:, 0] == 0] == 1.0).all()


def test_partial_constraints_use_the_global_sample():
    w = synth.small(2000, 16, 60, seed=4, integer=True, wildcard_arity=True)
    adj = oracle.build_graph(w.x, w.attrs, l=24, R=12)
    glob = oracle.entry_points(3, w.n, 64)
    strata = oracle.entry_strata(3, w.attrs, 16)
    part = (w.qattrs == oracle.WILDCARD).any(axis=1)
    a = oracle.search_strata(adj, w.x, w.attrs, w.q, w.qattrs, 10, 48, glob, strata, n_init=8,
                             key_mode=oracle.KEY32)
    b = oracle.search(adj, w.x, w.attrs, w.q, w.qattrs, 10, 48, glob, n_init=8, key_mode=oracle.KEY32)
    assert part.any() and np.array_equal(a[0][part], b[0][part])
