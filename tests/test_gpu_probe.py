"""The random-row gather probe reads the rows it reports, from every part of
the object set, for each storage form."""
import numpy as np
import pytest
import torch

import synth

pytestmark = pytest.mark.gpu

nhq = pytest.importorskip("paper_2203_13601_amd")


@pytest.mark.parametrize("storage,d", [("fp32", 128), ("bf16", 96), ("fp8", 960)])
def test_gather_probe_counts_and_sums(storage, d):
    w = synth.small(3000, d, 4, seed=71)
    x = np.abs(w.x) + 1.0  # positive rows: every lane's sum is positive
    ix = nhq.nhq_index_create(torch.from_numpy(x).cuda(), torch.from_numpy(w.attrs).cuda(), storage=storage,
                              n_entry=16)
    from paper_2203_13601_amd._binding import _padded_dim
    dp = _padded_dim(d)
    rb = 2 if dp <= 128 else 1
    sink, rows = nhq.nhq_gather_probe(ix, 64, 4 * rb)
    torch.cuda.synchronize()
    g = 8 if dp <= 512 else 16
    assert rows == 64 * 4 * rb * (64 // g)
    s = sink.cpu().numpy()
    assert np.isfinite(s).all() and (s > 0).all()
    with pytest.raises(nhq.NHQError):
        nhq.nhq_gather_probe(ix, 6, 4)
