"""The binding checks every query tensor against the index before a pointer
reaches the library (the C calls take no widths, so a narrower tensor would
be read past its end).  Runs on the CPU: the checks raise before any call,
on an index handle that is never dereferenced."""
import ctypes

import pytest
import torch

import paper_2203_13601_amd._binding as b


@pytest.fixture
def ix():
    h = b.Index(ctypes.c_void_p(1), device=torch.device("cuda", 0), d=128, m=3)
    yield h
    h._h = None  # never freed through the library


def _q(nq=4, d=128, m=3):
    return torch.zeros((nq, d), dtype=torch.float32), torch.zeros((nq, m), dtype=torch.uint8)


@pytest.mark.parametrize("call", ["search", "seed_rank", "seeded", "bruteforce"])
@pytest.mark.parametrize("bad", ["narrow_d", "wide_d", "narrow_m", "rows"])
def test_query_widths_are_checked(ix, call, bad):
    q, qa = _q()
    if bad == "narrow_d":
        q = q[:, :96].contiguous()
    elif bad == "wide_d":
        q = torch.zeros((4, 960), dtype=torch.float32)
    elif bad == "narrow_m":
        qa = qa[:, :2].contiguous()
    else:
        qa = qa[:3]
    with pytest.raises(ValueError):
        if call == "search":
            b.nhq_hybrid_search(ix, q, qa, 10, 32)
        elif call == "seed_rank":
            b.nhq_seed_rank(ix, q, qa, 12)
        elif call == "seeded":
            b.nhq_search_seeded(ix, q, qa, torch.zeros((4, 12), dtype=torch.int32), 10, 32)
        else:
            b.nhq_bruteforce_hybrid_knn(ix, q, qa, 10)


def test_tensors_off_the_index_device_are_rejected(ix):
    q, qa = _q()                       # right shapes, but host tensors
    with pytest.raises(ValueError, match="device"):
        b.nhq_hybrid_search(ix, q, qa, 10, 32)


def test_dtypes_are_checked(ix):
    q, qa = _q()
    with pytest.raises(TypeError):
        b.nhq_hybrid_search(ix, q.double(), qa, 10, 32)
    with pytest.raises(TypeError):
        b.nhq_hybrid_search(ix, q, qa.int(), 10, 32)


def test_caller_outputs_are_checked(ix):
    nq, k = 4, 10
    good = (torch.zeros((nq, k), dtype=torch.int32), torch.zeros((nq, k), dtype=torch.float32))
    bad = {
        "short": (torch.zeros((nq, k - 1), dtype=torch.int32), good[1]),
        "rows": (good[0], torch.zeros((nq - 1, k), dtype=torch.float32)),
        "strided": (torch.zeros((nq, 2 * k), dtype=torch.int32)[:, ::2], good[1]),
        "host": good,
    }
    for name, out in bad.items():
        with pytest.raises(ValueError):
            b._out_pair(ix, out, nq, k)
    with pytest.raises(TypeError):
        b._out_pair(ix, (good[1], good[0]), nq, k)   # dtypes swapped


def test_mlp_inputs_are_checked():
    with pytest.raises(ValueError):
        b._samples(torch.zeros((5, 7)), torch.zeros(5), torch.zeros(5), torch.device("cpu"))


@pytest.mark.parametrize("bad", ["dtype", "length", "device", "strided"])
def test_launch_order_is_checked(ix, bad):
    # the launch order must be an int32 [nq] tensor on the index's device
    order = {"dtype": torch.zeros(4, dtype=torch.int64), "length": torch.zeros(3, dtype=torch.int32),
             "device": torch.zeros(4, dtype=torch.int32),
             "strided": torch.zeros(8, dtype=torch.int32)[::2]}[bad]
    with pytest.raises(ValueError):
        b._order(ix, order, 4)


def test_query_order_checks_its_codes(ix):
    with pytest.raises(ValueError):
        b.nhq_query_order(ix, torch.zeros((4, 2), dtype=torch.uint8))
    with pytest.raises(ValueError):
        b.nhq_query_order(ix, torch.zeros((4, 3), dtype=torch.float32))
