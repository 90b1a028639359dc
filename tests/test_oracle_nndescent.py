"""Pins of the oracle's NN-descent (NPG_kgraph's candidate lists, Sec. 4.3):
the random start drawn from splitmix64 (pinned separately by its published
values), the list invariants, monotone improvement, the update count, the
special cases that reduce to the exact l nearest, and convergence toward the
brute-force lists."""
import numpy as np
import pytest

import oracle
import synth

M64 = (1 << 64) - 1


@pytest.fixture(scope="module")
def small():
    return synth.small(2500, 16, 4, seed=64, integer=True, n_centres=6, cards=(2, 3))


def _keys(w, i, ids):
    out = []
    for v in ids:
        d2 = float(((w.x[i].astype(np.float64) - w.x[v]) ** 2).sum())
        out.append((oracle.order_key(d2, oracle.chi(w.attrs[i], w.attrs[v]), w.m, oracle.KEY32),
                    int(v)))
    return out


def test_round_zero_is_the_splitmix_start(small):
    w = small
    l, seed = 24, 77
    ids, upd = oracle.nndescent(w.x, w.attrs, l, 8, 0, seed)
    for i in (0, 1, 999, w.n - 1):
        want = []
        for z in oracle.splitmix64((seed ^ (i * 0xD1B54A32D192ED03)) & M64):
            v = z % w.n
            if v != i and v not in want:
                want.append(v)
            if len(want) == l:
                break
        assert sorted(ids[i].tolist()) == sorted(want)
        # ordered by (key, id)
        k = _keys(w, i, ids[i])
        assert k == sorted(k)


def test_list_invariants_and_monotone_improvement(small):
    w = small
    l = 20
    prev = None
    for r in range(0, 5):
        ids, _ = oracle.nndescent(w.x, w.attrs, l, 6, r, 5)
        for i in range(0, w.n, 61):
            row = ids[i].tolist()
            assert i not in row and len(set(row)) == l
            k = _keys(w, i, row)
            assert k == sorted(k)
            if prev is not None:
                # every position's key can only fall: the list keeps the l
                # best of a superset of the previous list
                kp = _keys(w, i, prev[i])
                assert all(a <= b for a, b in zip(k, kp))
        prev = ids


def test_update_count_is_the_set_difference(small):
    w = small
    l, s = 16, 5
    a, _ = oracle.nndescent(w.x, w.attrs, l, s, 2, 9)
    b, upd = oracle.nndescent(w.x, w.attrs, l, s, 3, 9)
    diff = sum(len(set(b[i]) - set(a[i])) for i in range(w.n))
    assert upd[2] == diff


def test_no_sampling_means_no_change(small):
    w = small
    a, _ = oracle.nndescent(w.x, w.attrs, 16, 0, 0, 3)
    b, upd = oracle.nndescent(w.x, w.attrs, 16, 0, 4, 3)
    assert np.array_equal(a, b) and (upd == 0).all()


def test_tiny_set_is_exact_from_the_start():
    # n = l + 1: the start already holds every other vertex
    w = synth.small(33, 8, 2, seed=65, integer=True)
    ids, _ = oracle.nndescent(w.x, w.attrs, 32, 4, 2, 1)
    knn = oracle.knn_rows(w.x, w.attrs, np.arange(w.n), 32)
    assert np.array_equal(ids, knn)


def test_converges_toward_the_exact_lists(small):
    w = small
    ids, upd = oracle.nndescent(w.x, w.attrs, 24, 8, 10, 11)
    knn = oracle.knn_rows(w.x, w.attrs, np.arange(w.n), 24)
    q = np.mean([len(set(a) & set(b)) / 24 for a, b in zip(ids, knn)])
    assert q >= 0.95, q
    assert upd[-1] < upd[0] / 20
    # edge selection over the exact lists equals the reference build
    adj = oracle.select_lists(w.x, w.attrs, knn, 12)
    assert np.array_equal(adj, oracle.build_graph(w.x, w.attrs, l=24, R=12))


# ---------------------------------------------------------------- NPG_nsw
def test_nsw_single_batch_is_the_reference_build_with_reverse_edges(small):
    # one batch holding every vertex: exact candidates within it, then every
    # named vertex re-selects with its offers -- the reference build with
    # its reverse pass
    w = small
    adj = oracle.build_nsw(w.x, w.attrs, 24, 12, w.n, 48, 1)
    assert np.array_equal(adj, oracle.build_graph(w.x, w.attrs, l=24, R=12, reverse=True))


@pytest.mark.parametrize("batch", [1, 7, 400])
def test_nsw_rows_are_valid_and_searchable(small, batch):
    w = small
    n = 700 if batch == 1 else w.n
    x, at = w.x[:n], w.attrs[:n]
    adj = oracle.build_nsw(x, at, 16, 8, batch, 32, 2)
    for i in range(n):
        row = [int(v) for v in adj[i] if v >= 0]
        assert i not in row and len(set(row)) == len(row) and all(0 <= v < n for v in row)
        assert (adj[i][len(row):] == -1).all()
    # nearly every row has edges, and the search finds most answers
    assert ((adj >= 0).sum(1) > 0).mean() > 0.99
    entry = oracle.entry_points(5, n, 64)
    gi, gd, _ = oracle.bruteforce(x, at, w.q, w.qattrs, 10)
    ids, gam, _, _, _ = oracle.search(adj, x, at, w.q, w.qattrs, 10, 64, entry)
    got = np.mean([len(set(a[a >= 0]) & set(b[b >= 0])) / max(1, (b >= 0).sum()) for a, b in zip(ids, gi)])
    assert got >= 0.5


def test_nsw_batches_see_only_earlier_vertices(small):
    # a batch sees only earlier vertices, and nothing is inserted after the
    # last batch: its rows name only vertices of the earlier batches
    w = small
    n = 1200
    adj = oracle.build_nsw(w.x[:n], w.attrs[:n], 16, 8, 300, 32, 4)
    for i in range(900, 1200):
        assert (adj[i][adj[i] >= 0] < 1200).all()
        assert (adj[i][adj[i] >= 0] < 900).all()


def test_nsw_insert_continues_the_build(small):
    # inserting the rest of the set into an NSW graph of a batch-aligned
    # prefix is the NSW build of the whole set
    w = small
    n0, B = 900, 300
    pre = oracle.build_nsw(w.x[:n0], w.attrs[:n0], 16, 8, B, 32, 6)
    got = oracle.nsw_insert(w.x, w.attrs, pre, 16, B, 32, 6)
    assert np.array_equal(got, oracle.build_nsw(w.x, w.attrs, 16, 8, B, 32, 6))
