"""Precision form: bf16 / OCP fp8-e4m3 storage with float32 accumulation and
an exact float32 re-score of the first 4k eligible pool entries, against the
CPU oracle run on the decoded storage values (FP64)."""
import numpy as np
import pytest
import torch

import oracle
from parity import assert_float_parity
import synth

pytestmark = pytest.mark.gpu
nhq = pytest.importorskip("paper_2203_13601_amd")


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


@pytest.fixture(scope="module")
def gmm():
    w = synth.small(6000, 96, 120, seed=71, n_centres=12, cards=(2, 3, 5))
    adj = oracle.build_graph(w.x, w.attrs, l=48, R=32)
    return w, adj


def test_bf16_codes_bit_exact(gmm):
    w, adj = gmm
    ix = nhq.nhq_index_create(_dev(w.x), _dev(w.attrs), storage="bf16", n_entry=64)
    rows, _ = nhq.nhq_index_get_storage(ix)
    got = rows.cpu().numpy().view(np.uint16)[:, : w.d]
    assert np.array_equal(got, oracle.to_bf16_bits(w.x))
    assert (rows.cpu().numpy()[:, w.d:] == 0).all()


def test_fp8_codes_and_scales_bit_exact(gmm):
    w, adj = gmm
    x = w.x.copy()
    x[5] = 0.0                      # an all-zero row takes scale 1
    x[7, :3] = [-0.0, 1e-9, -3e-3]  # signed zero, tiny and subnormal-range values
    ix = nhq.nhq_index_create(_dev(x), _dev(w.attrs), storage="fp8", n_entry=64)
    rows, scales = nhq.nhq_index_get_storage(ix)
    codes, s = oracle.fp8_rows(x)
    assert np.array_equal(scales.cpu().numpy(), s)
    assert np.array_equal(rows.cpu().numpy()[:, : w.d], codes)


@pytest.mark.parametrize("storage", ["bf16", "fp8"])
def test_reduced_storage_search_matches_oracle_on_decoded_vectors(gmm, storage):
    w, adj = gmm
    if storage == "bf16":
        xs = oracle.from_bf16_bits(oracle.to_bf16_bits(w.x)).astype(np.float32)
    else:
        codes, s = oracle.fp8_rows(w.x)
        xs = oracle.fp8_decode_rows(codes, s).astype(np.float32)
    ix = nhq.nhq_index_create(_dev(w.x), _dev(w.attrs), storage=storage, n_entry=256,
                              seed=w.build_seed, degree=32)
    nhq.nhq_index_set_graph(ix, _dev(adj))
    entry = oracle.entry_points(w.build_seed, w.n, 256)
    ids, dist = nhq.nhq_hybrid_search(ix, _dev(w.q), _dev(w.qattrs), 10, 64, rerank=4)
    ids, dist = ids.cpu().numpy(), dist.cpu().numpy()
    oi, og, _, _, _ = oracle.search(adj, xs, w.attrs, w.q, w.qattrs, 10, 64, entry,
                                    rerank_n=40, xr=w.x)
    assert_float_parity(ids, oi, w.x, w.attrs, w.q, w.qattrs)
    # every returned distance is the exact delta of the returned object (the
    # re-score reads the float32 copy): error against FP64 per result
    rel = []
    for i in range(w.nq):
        for v, g in zip(ids[i], dist[i]):
            if v >= 0:
                assert oracle.chi(w.qattrs[i], w.attrs[v]) == 0
                want = oracle.delta(w.q[i], w.x[v])
                rel.append(abs(g - want) / want)
    assert max(rel) <= 1e-4
    # re-scored results are sorted by exact distance
    for row in dist:
        fin = row[np.isfinite(row)]
        assert (np.diff(fin) >= 0).all()


def test_bf16_on_integer_vectors_is_lossless():
    # integers 0..255 are exact in bf16: the bf16 path equals the fp32 path
    w = synth.small(5000, 128, 64, seed=72, integer=True)
    adj = oracle.build_graph(w.x, w.attrs, l=48, R=32)
    out = {}
    for st in ("fp32", "bf16"):
        ix = nhq.nhq_index_create(_dev(w.x), _dev(w.attrs), storage=st, n_entry=128, seed=4, degree=32)
        nhq.nhq_index_set_graph(ix, _dev(adj))
        ids, dist, cnt = nhq.nhq_hybrid_search(ix, _dev(w.q), _dev(w.qattrs), 10, 48, counters=True)
        out[st] = (ids.cpu().numpy(), dist.cpu().numpy(), cnt.cpu().numpy())
    for a, b in zip(out["fp32"], out["bf16"]):
        assert np.array_equal(a, b)
