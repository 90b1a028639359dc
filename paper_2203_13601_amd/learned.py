"""Training driver of the learned stop network (argument marshalling only:
traces, labels, forward, backward and Adam all run in the library's
kernels).

The network reads 8 search-state features at every checkpoint (every
`check_every` expansions) and outputs a stop logit and log2 of a hop budget
(learned modes 1 and 2), or, trained on pool-size targets, log2 of the pool
size a query needs (mode 3, the beam-width predictor); fixed-beam search is
both its fallback (the pool of `beam` entries still bounds the search) and
the judge of its recall loss.
"""
from __future__ import annotations

import math
from typing import Dict, Tuple

import torch

from ._binding import (MLP_PARAMS, Index, TraceBuffers, nhq_hybrid_search, nhq_mlp_train,
                       nhq_trace_samples)


def init_params(seed: int = 0, device="cuda") -> torch.Tensor:
    """He-normal weights, zero biases, in the library's parameter order."""
    g = torch.Generator().manual_seed(seed)
    parts = []
    for (rows, cols) in ((64, 8), (64, 64), (2, 64)):
        parts.append(torch.randn(rows * cols, generator=g, dtype=torch.float64) * math.sqrt(2.0 / cols))
        parts.append(torch.zeros(rows, dtype=torch.float64))
    return torch.cat(parts).to(torch.float32).to(device)


def collect(ix: Index, queries: torch.Tensor, qattrs: torch.Tensor, k: int, beam: int,
            check_every: int = 4, n_init: int = 32, trace_cap: int = 0, expand: int = 1):
    """Plain fixed-beam search of the training queries with traces; returns
    (X, y_stop, y_beam) device tensors."""
    cap = trace_cap or (2 * beam) // check_every + 16
    tr = TraceBuffers(queries.shape[0], cap, device=queries.device)
    _, _, cnt = nhq_hybrid_search(ix, queries, qattrs, k, beam, n_init=n_init, check_every=check_every,
                                  counters=True, trace=tr, expand=expand)
    return nhq_trace_samples(tr, cnt)


def train_stop_network(ix: Index, queries: torch.Tensor, qattrs: torch.Tensor, k: int, beam: int,
                       epochs: int = 30, check_every: int = 4, n_init: int = 32, lr: float = 2e-3,
                       lam: float = 0.5, batch: int = 1024, seed: int = 0, expand: int = 1
                       ) -> Tuple[torch.Tensor, Dict]:
    X, ys, yb = collect(ix, queries, qattrs, k, beam, check_every, n_init, expand=expand)
    params = init_params(seed, queries.device)
    state = torch.zeros(2 * MLP_PARAMS, dtype=torch.float32, device=queries.device)
    step, losses = nhq_mlp_train(params, state, 0, X, ys, yb, epochs, batch, lr, lam, seed)
    info = {"samples": int(X.shape[0]), "positive_rate": float(ys.mean().item()) if X.shape[0] else 0.0,
            "steps": step, "losses": losses.cpu().tolist()}
    return params, info


def pool_labels(ix: Index, queries: torch.Tensor, qattrs: torch.Tensor, k: int, beam: int, ladder,
                n_init: int = 32, expand: int = 1, rerank: int = 0) -> torch.Tensor:
    """Per query, log2 of the smallest pool size of `ladder` (sizes below
    `beam`) from which every larger size up to `beam` returns the same ids as
    the search at `beam`: the beam-width predictor's target."""
    ref, _ = nhq_hybrid_search(ix, queries, qattrs, k, beam, n_init=n_init, expand=expand, rerank=rerank)
    nq = queries.shape[0]
    smallest = torch.full((nq,), float(beam), dtype=torch.float32, device=queries.device)
    same = torch.ones(nq, dtype=torch.bool, device=queries.device)
    for size in sorted({int(s) for s in ladder if k <= int(s) < beam}, reverse=True):
        ids, _ = nhq_hybrid_search(ix, queries, qattrs, k, size, n_init=n_init, expand=expand, rerank=rerank)
        same &= (ids == ref).all(dim=1)
        smallest = torch.where(same, torch.full_like(smallest, float(size)), smallest)
    return torch.log2(smallest)


def train_pool_network(ix: Index, queries: torch.Tensor, qattrs: torch.Tensor, k: int, beam: int,
                       ladder=(10, 12, 16, 20, 24, 32, 40, 48, 64, 96, 128, 192, 256, 384, 512),
                       epochs: int = 30, check_every: int = 1, n_init: int = 32, lr: float = 2e-3,
                       lam: float = 4.0, batch: int = 1024, seed: int = 0, expand: int = 1, rerank: int = 0
                       ) -> Tuple[torch.Tensor, Dict]:
    """The beam-width predictor (learned mode 3): one sample per training
    query, its features at the first checkpoint of the search at `beam`, and
    the target log2 of the pool size it needs (pool_labels).  The stop
    output is trained towards 'continue' and is not read in mode 3."""
    tr = TraceBuffers(queries.shape[0], 1, device=queries.device)
    nhq_hybrid_search(ix, queries, qattrs, k, beam, n_init=n_init, check_every=check_every, trace=tr,
                      expand=expand, rerank=rerank)
    has = tr.count > 0
    X = tr.feat[:, 0, :][has].contiguous()
    yb = pool_labels(ix, queries, qattrs, k, beam, ladder, n_init=n_init, expand=expand,
                     rerank=rerank)[has].contiguous()
    ys = torch.zeros_like(yb)
    params = init_params(seed, queries.device)
    state = torch.zeros(2 * MLP_PARAMS, dtype=torch.float32, device=queries.device)
    step, losses = nhq_mlp_train(params, state, 0, X, ys, yb, epochs, batch, lr, lam, seed)
    info = {"samples": int(X.shape[0]), "steps": step, "losses": losses.cpu().tolist(),
            "pool_label_median": float(torch.exp2(yb.median()).item()) if X.shape[0] else 0.0}
    return params, info
