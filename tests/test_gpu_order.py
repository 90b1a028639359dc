"""The launch order by selectivity (nhq_query_order, search param `order`):
a permutation of the queries, least selective first, that changes which
wavefront searches which query and nothing else -- ids, distances and
counters are bit-identical to the natural order, for the plain search and
the learned modes."""
import math

import numpy as np
import pytest
import torch

import synth

pytestmark = pytest.mark.gpu
nhq = pytest.importorskip("paper_2203_13601_amd")
from paper_2203_13601_amd.learned import init_params  # noqa: E402


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


@pytest.fixture(scope="module")
def mixed():
    w = synth.small(20000, 64, 600, seed=131, integer=True, n_centres=8, wildcard_arity=True, zipf=True)
    ix = nhq.nhq_build_index(_dev(w.x), _dev(w.attrs), degree=32, cand=64, n_entry=512, seed=w.build_seed)
    return w, ix


def _logsel(w):
    """sum over the constrained attributes of ln(count(code) / n), count 0 read as 0.5"""
    ls = np.zeros(w.nq)
    for i in range(w.m):
        cnt = np.bincount(w.attrs[:, i], minlength=256).astype(np.float64)
        c = w.qattrs[:, i]
        on = c != 255
        ls[on] += np.log(np.maximum(cnt[c[on]], 0.5) / w.n)
    return ls


def test_order_is_a_permutation_by_decreasing_selectivity(mixed):
    w, ix = mixed
    order = nhq.nhq_query_order(ix, _dev(w.qattrs)).cpu().numpy()
    assert np.array_equal(np.sort(order), np.arange(w.nq))
    ls = _logsel(w)[order]
    # buckets of 1/16 (float32 sums on the device): never increasing by more
    # than one bucket plus rounding along the order
    assert (np.diff(ls) <= 1.0 / 16 + 1e-4).all()
    assert ls[0] >= ls[-1]
    # the order does depend on the codes: unconstrained queries come first
    un = (w.qattrs == 255).all(axis=1)
    if un.any():
        assert un[order[: int(un.sum())]].all()


@pytest.mark.parametrize("mode", [0, 2, 3])
def test_order_leaves_results_unchanged(mixed, mode):
    w, ix = mixed
    q, qa = _dev(w.q), _dev(w.qattrs)
    kw = dict(n_init=8, expand=2, counters=True)
    if mode:
        nhq.nhq_mlp_load(ix, init_params(5))
        kw.update(learned=mode, check_every=2, stop_threshold=0.7, cap_factor=24.0)
    order = nhq.nhq_query_order(ix, qa)
    a = nhq.nhq_hybrid_search(ix, q, qa, 10, 96, **kw)
    b = nhq.nhq_hybrid_search(ix, q, qa, 10, 96, order=order, **kw)
    rev = torch.flip(order, [0]).contiguous()
    c = nhq.nhq_hybrid_search(ix, q, qa, 10, 96, order=rev, **kw)
    torch.cuda.synchronize()
    if mode:
        nhq.nhq_mlp_load(ix, None)
    for x in (b, c):
        assert torch.equal(a[0], x[0])
        assert torch.equal(a[1].view(torch.int32), x[1].view(torch.int32))
        assert torch.equal(a[2], x[2])
    assert nhq.nhq_index_device_error(ix) == 0


def test_order_entry_out_of_range_is_skipped_and_reported(mixed):
    w, ix = mixed
    q, qa = _dev(w.q[:64]), _dev(w.qattrs[:64])
    order = torch.arange(64, dtype=torch.int32, device="cuda")
    order[63] = 64 + 7
    ids, dists = nhq.nhq_hybrid_search(ix, q, qa, 10, 64, n_init=8, order=order)
    ref, _ = nhq.nhq_hybrid_search(ix, q, qa, 10, 64, n_init=8)
    torch.cuda.synchronize()
    assert nhq.nhq_index_device_error(ix) & nhq.DEVERR_BADID
    # every listed query was searched as in the natural order
    assert torch.equal(ids[:63], ref[:63])
