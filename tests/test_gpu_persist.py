"""Index files (nhq_index_save / nhq_index_load): a loaded index answers
every call as the saved one did -- graph, entry sample, stored rows, seed
ranking, search results and counters, exact answers, the learned stop and
later insertions -- bit for bit, for every storage form; damaged files are
refused with NHQ_EIO and create no index."""
import os

import numpy as np
import pytest
import torch

import oracle
import synth

pytestmark = pytest.mark.gpu

nhq = pytest.importorskip("paper_2203_13601_amd")


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


@pytest.fixture(scope="module")
def data():
    return synth.small(3000, 40, 48, seed=91, integer=True, n_centres=6, cards=(2, 3, 4))


def _answers(ix, w, **kw):
    ids, dist, cnt = nhq.nhq_hybrid_search(ix, _dev(w.q), _dev(w.qattrs), 10, 48, expand=2, counters=True, **kw)
    cand = nhq.nhq_seed_rank(ix, _dev(w.q), _dev(w.qattrs), 20)
    gi, gd = nhq.nhq_bruteforce_hybrid_knn(ix, _dev(w.q), _dev(w.qattrs), 10)
    torch.cuda.synchronize()
    return [t.cpu().numpy() for t in (ids, dist, cnt, cand, gi, gd)]


@pytest.mark.parametrize("storage", ["fp32", "bf16", "fp8"])
def test_round_trip_answers_every_call_alike(data, storage, tmp_path):
    w = data
    ix = nhq.nhq_build_index(_dev(w.x), _dev(w.attrs), degree=16, cand=32, n_entry=128, seed=3,
                             storage=storage)
    path = str(tmp_path / ("ix_%s.nhq" % storage))
    nhq.nhq_index_save(ix, path)
    iy = nhq.nhq_index_load(path)
    assert nhq.nhq_index_info(iy) == nhq.nhq_index_info(ix)
    assert torch.equal(nhq.nhq_index_get_graph(iy), nhq.nhq_index_get_graph(ix))
    assert torch.equal(nhq.nhq_index_get_entry(iy), nhq.nhq_index_get_entry(ix))
    for a, b in zip(nhq.nhq_index_get_storage(ix), nhq.nhq_index_get_storage(iy)):
        if a is None:
            assert b is None
        else:
            assert torch.equal(a, b)
    for a, b in zip(_answers(ix, w), _answers(iy, w)):
        assert np.array_equal(a, b, equal_nan=True)
    # and the loaded index still equals the oracle on its graph
    adj = nhq.nhq_index_get_graph(iy).cpu().numpy()
    entry = oracle.entry_points(3, w.n, 128)
    if storage == "fp32":
        oi, _, ondc, ohops, _ = oracle.search(adj, w.x, w.attrs, w.q, w.qattrs, 10, 48, entry,
                                              key_mode=oracle.KEY32, expand=2)
        got = _answers(iy, w)
        assert np.array_equal(got[0], oi)
        assert np.array_equal(got[2][:, 0], ondc) and np.array_equal(got[2][:, 1], ohops)


def test_round_trip_keeps_weights_and_stop_network(data, tmp_path):
    w = data
    ix = nhq.nhq_build_index(_dev(w.x), _dev(w.attrs), degree=16, cand=32, n_entry=128, seed=4,
                             weights="normalised", weight_param=900.0)
    p = oracle.MLPRef.init(7)
    flat = np.concatenate([p[k].ravel() for k in ("W1", "b1", "W2", "b2", "W3", "b3")]).astype(np.float32)
    assert flat.size == nhq.MLP_PARAMS
    flat[4864] = -1.0
    nhq.nhq_mlp_load(ix, _dev(flat))
    path = str(tmp_path / "ix_w.nhq")
    nhq.nhq_index_save(ix, path)
    iy = nhq.nhq_index_load(path)
    for kw in (dict(), dict(learned=1, stop_threshold=0.5, check_every=4),
               dict(learned=2, stop_threshold=0.5, check_every=4, cap_factor=1.5)):
        for a, b in zip(_answers(ix, w, **kw), _answers(iy, w, **kw)):
            assert np.array_equal(a, b, equal_nan=True)


def test_loaded_index_takes_insertions_like_the_saved_one(data, tmp_path):
    w = data
    n0 = 2000
    kw = dict(degree=12, cand=24, n_entry=64, seed=21, builder="nsw", nsw_batch=500, nsw_beam=48,
              capacity=w.n)
    ix = nhq.nhq_build_index(_dev(w.x[:n0]), _dev(w.attrs[:n0]), **kw)
    path = str(tmp_path / "ix_cap.nhq")
    nhq.nhq_index_save(ix, path)
    iy = nhq.nhq_index_load(path)
    for index in (ix, iy):
        nhq.nhq_index_insert(index, _dev(w.x[n0:]), _dev(w.attrs[n0:]))
    assert torch.equal(nhq.nhq_index_get_graph(iy), nhq.nhq_index_get_graph(ix))
    assert np.array_equal(nhq.nhq_index_get_graph(iy).cpu().numpy(),
                          oracle.build_nsw(w.x, w.attrs, 24, 12, 500, 48, 21))


def test_damaged_files_are_refused(data, tmp_path):
    w = data
    ix = nhq.nhq_build_index(_dev(w.x[:500]), _dev(w.attrs[:500]), degree=12, cand=24, n_entry=32)
    path = str(tmp_path / "ok.nhq")
    nhq.nhq_index_save(ix, path)
    raw = open(path, "rb").read()
    cases = {"missing": None, "not_an_index": b"hello world" * 40, "truncated": raw[:-7],
             "trailing": raw + b"\0", "bad_version": raw[:8] + b"\x09" + raw[9:]}
    for name, blob in cases.items():
        p = str(tmp_path / (name + ".nhq"))
        if blob is not None:
            open(p, "wb").write(blob)
        with pytest.raises(nhq.NHQError) as e:
            nhq.nhq_index_load(p)
        assert e.value.code == -6, name  # NHQ_EIO
    with pytest.raises(nhq.NHQError):
        nhq.nhq_index_save(ix, str(tmp_path / "no_such_dir" / "x.nhq"))
    assert os.path.getsize(path) == len(raw)
    assert not os.path.exists(path + ".partial")
    # a save over an existing file replaces it whole
    iy = nhq.nhq_build_index(_dev(w.x[:300]), _dev(w.attrs[:300]), degree=12, cand=24, n_entry=32)
    nhq.nhq_index_save(iy, path)
    assert nhq.nhq_index_info(nhq.nhq_index_load(path))["n"] == 300
    assert not os.path.exists(path + ".partial")
