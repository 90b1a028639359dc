"""Pins of the oracle's storage conversions (bf16, OCP fp8 e4m3 with a
per-vector scale) and of the FP64 reference of the stop/beam network."""
import numpy as np
import pytest
import torch

import oracle


def test_bf16_matches_torch_rounding():
    rng = np.random.default_rng(0)
    x = np.concatenate([rng.standard_normal(20000).astype(np.float32) * 100,
                        np.array([0.0, -0.0, 1.0, 255.0, 3.0e38, 1e-40, np.inf, -np.inf], np.float32)])
    # ties: values exactly half-way between two bf16 numbers
    base = rng.integers(0, 1 << 15, size=1000).astype(np.uint32) << 16
    ties = (base | 0x8000).view(np.float32)
    x = np.concatenate([x, ties])
    ours = oracle.to_bf16_bits(x)
    ref = torch.from_numpy(x.copy()).to(torch.bfloat16).view(torch.int16).numpy().view(np.uint16)
    nan = np.isnan(x)                       # NaN payloads are not compared
    assert np.array_equal(ours[~nan], ref[~nan])
    assert np.isnan(oracle.from_bf16_bits(ours[nan])).all()
    back = oracle.from_bf16_bits(ours)
    fin = np.isfinite(x) & (np.abs(x) > 1e-37) & (np.abs(x) < 3e38)
    # 8 significant bits: unit roundoff 2^-8
    assert np.all(np.abs(back[fin] - x[fin]) <= np.abs(x[fin]) * 2.0 ** -8)
    # integers 0..255 are exact in bf16
    ints = np.arange(256, dtype=np.float32)
    assert np.array_equal(oracle.from_bf16_bits(oracle.to_bf16_bits(ints)), ints)


def test_e4m3_decode_all_codes_against_torch():
    codes = np.arange(256, dtype=np.uint8)
    ref = torch.from_numpy(codes.copy()).view(torch.float8_e4m3fn).to(torch.float64).numpy()
    ours = oracle.e4m3_table()
    nan = np.isnan(ref)
    assert np.array_equal(np.isnan(ours), nan)
    assert nan.sum() == 2                       # 0x7F and 0xFF
    assert np.array_equal(ours[~nan], ref[~nan])
    assert np.nanmax(ours) == 448.0


def test_e4m3_encode_matches_torch_and_round_trips():
    rng = np.random.default_rng(1)
    x = np.concatenate([rng.uniform(-460, 460, 20000), rng.standard_normal(5000) * 0.01,
                        oracle.e4m3_table()[:0x7F]])
    x = x[np.isfinite(x)]
    ours = oracle.to_e4m3(x)
    ref = torch.from_numpy(np.clip(x, -448, 448)).to(torch.float8_e4m3fn).view(torch.uint8).numpy()
    assert np.array_equal(ours, ref)
    # every finite code round-trips
    t = oracle.e4m3_table()
    fin = np.arange(256)[np.isfinite(t)]
    assert np.array_equal(oracle.to_e4m3(t[fin]), fin.astype(np.uint8))
    # relative error in the normal range is at most 2^-4
    normal = (np.abs(x) >= 2 ** -6) & (np.abs(x) <= 448)
    dec = t[ours[normal]]
    assert np.all(np.abs(dec - x[normal]) <= np.abs(x[normal]) * 2.0 ** -4)


def test_fp8_rows_scale_and_error():
    rng = np.random.default_rng(2)
    x = rng.standard_normal((50, 96)).astype(np.float32) * 3
    x[3] = 0.0
    codes, s = oracle.fp8_rows(x)
    assert s[3] == 1.0 and (codes[3] == 0).all()
    dec = oracle.fp8_decode_rows(codes, s)
    mx = np.abs(x).max(1)
    # the largest element of each row maps to +-448 exactly
    for i in range(50):
        if mx[i] > 0:
            j = np.abs(x[i]).argmax()
            assert abs(dec[i, j]) == pytest.approx(mx[i], rel=1e-6)
    assert np.all(np.abs(dec - x) <= np.maximum(np.abs(x) * 2.0 ** -4, (s[:, None] * 2.0 ** -9) + 1e-12))


def _params(seed=0):
    p = oracle.MLPRef.init(seed)
    rng = np.random.default_rng(seed + 1)
    for k in p:
        p[k] = p[k] + rng.standard_normal(p[k].shape) * 0.1
    return p


def test_mlp_backward_finite_differences():
    rng = np.random.default_rng(3)
    p = _params()
    X = rng.standard_normal((16, 8))
    ys = (rng.uniform(size=16) > 0.5).astype(np.float64)
    yb = rng.uniform(5, 9, size=16)
    z, cache = oracle.MLPRef.forward(p, X)
    g = oracle.MLPRef.backward(p, cache, z, ys, yb)
    h = 1e-6
    for name in p:
        flat = p[name].reshape(-1)
        for idx in rng.choice(flat.size, size=min(12, flat.size), replace=False):
            old = flat[idx]
            flat[idx] = old + h
            lp = oracle.MLPRef.loss(oracle.MLPRef.forward(p, X)[0], ys, yb)
            flat[idx] = old - h
            lm = oracle.MLPRef.loss(oracle.MLPRef.forward(p, X)[0], ys, yb)
            flat[idx] = old
            fd = (lp - lm) / (2 * h)
            an = g[name].reshape(-1)[idx]
            assert abs(fd - an) <= 1e-6 * max(1.0, abs(an)) + 1e-9, (name, idx, fd, an)


def test_mlp_matches_torch_autograd_and_adam():
    rng = np.random.default_rng(4)
    p = _params(5)
    X = rng.standard_normal((64, 8))
    ys = (rng.uniform(size=64) > 0.3).astype(np.float64)
    yb = rng.uniform(5, 9, size=64)
    tp = {k: torch.tensor(v, dtype=torch.float64, requires_grad=True) for k, v in p.items()}
    Xt = torch.tensor(X)
    h1 = torch.relu(Xt @ tp["W1"].T + tp["b1"])
    h2 = torch.relu(h1 @ tp["W2"].T + tp["b2"])
    z = h2 @ tp["W3"].T + tp["b3"]
    bce = torch.nn.functional.binary_cross_entropy_with_logits(z[:, 0], torch.tensor(ys))
    hub = torch.nn.functional.huber_loss(z[:, 1], torch.tensor(yb), delta=1.0)
    loss = bce + hub
    loss.backward()
    zo, cache = oracle.MLPRef.forward(p, X)
    assert np.allclose(zo, z.detach().numpy(), rtol=1e-12, atol=1e-12)
    assert oracle.MLPRef.loss(zo, ys, yb) == pytest.approx(loss.item(), rel=1e-12)
    g = oracle.MLPRef.backward(p, cache, zo, ys, yb)
    for k in p:
        assert np.allclose(g[k], tp[k].grad.numpy(), rtol=1e-10, atol=1e-13), k
    # three Adam steps against torch.optim.Adam
    opt = torch.optim.Adam(list(tp.values()), lr=1e-2)
    st = {}
    pc = {k: v.copy() for k, v in p.items()}
    for _ in range(3):
        opt.zero_grad()
        h1 = torch.relu(Xt @ tp["W1"].T + tp["b1"])
        h2 = torch.relu(h1 @ tp["W2"].T + tp["b2"])
        z = h2 @ tp["W3"].T + tp["b3"]
        l = (torch.nn.functional.binary_cross_entropy_with_logits(z[:, 0], torch.tensor(ys))
             + torch.nn.functional.huber_loss(z[:, 1], torch.tensor(yb), delta=1.0))
        l.backward()
        opt.step()
        zo, cache = oracle.MLPRef.forward(pc, X)
        gg = oracle.MLPRef.backward(pc, cache, zo, ys, yb)
        pc = oracle.MLPRef.adam(pc, gg, st, lr=1e-2)
    for k in p:
        assert np.allclose(pc[k], tp[k].detach().numpy(), rtol=1e-9, atol=1e-12), k
