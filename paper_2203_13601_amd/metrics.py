"""Search-quality and cost metrics (Sec. 6.1, "Metrics").

Recall@k (Eq. 3) with the hybrid rule: the returned set and the exact set
both consist of objects whose attributes match the query; a returned id is a
hit when it matches, is not repeated, and lies no farther from the query than
the last exact answer (equal distances at the k-th place count, since several
answer sets can then be exact).  The denominator is min(k, |P|); a query that
no object satisfies scores 1.
"""
from __future__ import annotations

import numpy as np


def recall_at_k(ids: np.ndarray, dists: np.ndarray, gt_ids: np.ndarray, gt_dists: np.ndarray,
                attrs: np.ndarray, qattrs: np.ndarray, k: int, rtol: float = 1e-6) -> np.ndarray:
    """Per-query hybrid Recall@k.  ids/dists: returned [nq, >=k] (Gamma =
    delta for matching objects); gt_ids/gt_dists: exact answers [nq, >=k]."""
    nq = ids.shape[0]
    out = np.ones(nq, dtype=np.float64)
    cons = qattrs != 0xFF
    for i in range(nq):
        g = gt_ids[i, :k]
        ng = int((g >= 0).sum())
        if ng == 0:
            continue
        lim = float(gt_dists[i, ng - 1]) * (1.0 + rtol)
        seen = set()
        hits = 0
        for v, dv in zip(ids[i, :k], dists[i, :k]):
            v = int(v)
            if v < 0 or v in seen:
                continue
            seen.add(v)
            if not np.all(attrs[v, cons[i]] == qattrs[i, cons[i]]):
                continue
            if float(dv) <= lim:
                hits += 1
        out[i] = hits / ng
    return out


def qps_at_recall(beams, recalls, qps, target: float):
    """QPS at a target recall, interpolating log(QPS) linearly in recall
    between the two swept beams that bracket the target.  Returns None when
    no beam reaches the target; the QPS of the first beam when it already
    does (no extrapolation)."""
    pts = sorted(zip(beams, recalls, qps))
    prev = None
    for b, r, q in pts:
        if r >= target:
            if prev is None or prev[1] >= r:
                return float(q)
            _, r0, q0 = prev
            t = (target - r0) / (r - r0)
            return float(np.exp(np.log(q0) + t * (np.log(q) - np.log(q0))))
        prev = (b, r, q)
    return None


def search_bytes_per_query(d_pad: int, elem_bytes: int, R: int, k: int, n_cand: float, ndc: float,
                           hops: float, d: int, m: int, scale_bytes: int = 0,
                           out_rows: float = None) -> float:
    """Bytes the search kernel must move per query (HBM, algorithmic):
    the query vector and codes, the seed candidates (position, entry id,
    attribute word, stored row), one adjacency row per expansion, the
    attribute word and stored row of every scored neighbour, the float32
    rows re-read for the output distances, and the written ids/distances."""
    row = d_pad * elem_bytes + scale_bytes
    out_rows = k if out_rows is None else out_rows
    return (4.0 * d + m
            + n_cand * (4 + 4 + 4 + row)
            + hops * 4.0 * R
            + ndc * (4.0 + row)
            + out_rows * 4.0 * d_pad
            + 8.0 * k)
