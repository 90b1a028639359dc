"""nhq_seed_rank_ws: the seed ranking with the caller's scratch.  Its
candidates must equal nhq_seed_rank's bit for bit on every ranking path
(matrix-core keys of a plain entry sample, a stratified sample, and the
float32 tiles of a sample over 8,192), also when two batches run at once on
two streams of one index with two workspaces; a short or misaligned
workspace is refused."""
import numpy as np
import pytest
import torch

import synth

pytestmark = pytest.mark.gpu
nhq = pytest.importorskip("paper_2203_13601_amd")


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def _ws(ix, nq, n_cand, extra=0):
    b = nhq.nhq_seed_rank_workspace_size(ix, nq, n_cand)
    return torch.empty(b + extra, dtype=torch.uint8, device="cuda")


@pytest.mark.parametrize("kind", ["dense", "strata", "tiles"])
def test_workspace_ranking_equals_index_workspace(kind):
    w = synth.small(30000, 96, 700, seed=141, n_centres=12, cards=(2, 3, 5), zipf=kind == "strata")
    kw = dict(n_entry=1024)
    if kind == "strata":
        kw = dict(n_entry=256, entry_per_pattern=512)
    elif kind == "tiles":
        kw = dict(n_entry=9000)
    ix = nhq.nhq_index_create(_dev(w.x), _dev(w.attrs), seed=w.build_seed, degree=32, **kw)
    q, qa = _dev(w.q), _dev(w.qattrs)
    want = nhq.nhq_seed_rank(ix, q, qa, 12).cpu().numpy()
    got = nhq.nhq_seed_rank(ix, q, qa, 12, workspace=_ws(ix, w.nq, 12)).cpu().numpy()
    assert np.array_equal(got, want)
    ix.free()


def test_two_streams_two_workspaces():
    w = synth.small(30000, 128, 2000, seed=142, n_centres=12)
    ix = nhq.nhq_index_create(_dev(w.x), _dev(w.attrs), seed=w.build_seed, degree=32, n_entry=2048)
    adj = synth.random_graph(w.n, 32, seed=7)
    nhq.nhq_index_set_graph(ix, _dev(adj))
    q, qa = _dev(w.q), _dev(w.qattrs)
    half = w.nq // 2
    parts = [(q[:half], qa[:half]), (q[half:], qa[half:])]
    want = []
    for pq, pa in parts:
        c = nhq.nhq_seed_rank(ix, pq, pa, 12)
        want.append(nhq.nhq_search_seeded(ix, pq, pa, c, 10, 64, n_init=4, expand=2)[0].cpu().numpy())
    streams = [torch.cuda.Stream(), torch.cuda.Stream()]
    ws = [_ws(ix, half, 12), _ws(ix, w.nq - half, 12)]
    torch.cuda.synchronize()
    outs = []
    for rep in range(3):
        res = []
        for j, (pq, pa) in enumerate(parts):
            with torch.cuda.stream(streams[j]):
                c = nhq.nhq_seed_rank(ix, pq, pa, 12, stream=streams[j], workspace=ws[j])
                res.append(nhq.nhq_search_seeded(ix, pq, pa, c, 10, 64, n_init=4, expand=2,
                                                 stream=streams[j])[0])
        torch.cuda.synchronize()
        outs.append([r.cpu().numpy() for r in res])
    for res in outs:
        for j in range(2):
            assert np.array_equal(res[j], want[j]), j
    assert nhq.nhq_index_device_error(ix) == 0
    ix.free()


def test_short_or_misaligned_workspace_is_refused():
    w = synth.small(5000, 64, 100, seed=143)
    ix = nhq.nhq_index_create(_dev(w.x), _dev(w.attrs), seed=w.build_seed, degree=32, n_entry=512)
    q, qa = _dev(w.q), _dev(w.qattrs)
    need = nhq.nhq_seed_rank_workspace_size(ix, w.nq, 12)
    assert need > 0
    short = torch.empty(need - 4, dtype=torch.uint8, device="cuda")
    with pytest.raises(nhq.NHQError):
        nhq.nhq_seed_rank(ix, q, qa, 12, workspace=short)
    big = torch.empty(need + 512, dtype=torch.uint8, device="cuda")
    with pytest.raises(nhq.NHQError):
        nhq.nhq_seed_rank(ix, q, qa, 12, workspace=big[1:])
    with pytest.raises(ValueError):
        nhq.nhq_seed_rank(ix, q, qa, 12, workspace=torch.empty(need, dtype=torch.float32, device="cuda"))
    ix.free()
