"""Search-quality and cost metrics (Sec. 6.1, "Metrics").

Recall@k (Eq. 3) with the hybrid rule: the returned set and the exact set
both consist of objects whose attributes match the query; a returned id is a
hit when it matches, is not repeated, and lies no farther from the query than
the last exact answer (equal distances at the k-th place count, since several
answer sets can then be exact).  The denominator is min(k, |P|); a query that
no object satisfies scores 1.  Every distance it compares is recomputed here
in FP64 from the vectors (Eq. 1): neither the returned distances nor those of
the exact answers are trusted.
"""
from __future__ import annotations

import numpy as np

_CHUNK = 1024


def true_delta(ids: np.ndarray, x: np.ndarray, q: np.ndarray) -> np.ndarray:
    """FP64 Euclidean distance (Eq. 1) from query i to object ids[i, j];
    +inf where ids[i, j] < 0."""
    ids = np.asarray(ids)
    out = np.full(ids.shape, np.inf, dtype=np.float64)
    for s in range(0, ids.shape[0], _CHUNK):
        e = min(ids.shape[0], s + _CHUNK)
        blk = ids[s:e]
        ok = blk >= 0
        rows = x[np.where(ok, blk, 0)].astype(np.float64)          # [c, k, d]
        diff = rows - q[s:e, None, :].astype(np.float64)
        dl = np.sqrt(np.einsum("ckd,ckd->ck", diff, diff))
        out[s:e] = np.where(ok, dl, np.inf)
    return out


def matches(ids: np.ndarray, attrs: np.ndarray, qattrs: np.ndarray) -> np.ndarray:
    """ids[i, j] >= 0 and its codes equal query i's on every constrained
    attribute (Def. 4; code 255 marks an unconstrained query attribute)."""
    ok = ids >= 0
    a = attrs[np.where(ok, ids, 0)]                                # [nq, k, m]
    cons = (qattrs != 0xFF)[:, None, :]
    same = (a == qattrs[:, None, :]) | ~cons
    return ok & same.all(axis=2)


def recall_at_k(ids: np.ndarray, x: np.ndarray, q: np.ndarray, attrs: np.ndarray,
                qattrs: np.ndarray, gt_ids: np.ndarray, k: int, rtol: float = 1e-12) -> np.ndarray:
    """Per-query hybrid Recall@k of the returned ids [nq, >=k] against the
    exact answers gt_ids [nq, >=k] (-1 padded), every distance recomputed in
    FP64."""
    ids = np.asarray(ids)[:, :k]
    gt = np.asarray(gt_ids)[:, :k]
    ng = (gt >= 0).sum(axis=1)
    gd = true_delta(gt, x, q)
    lim = np.where(ng > 0, np.max(np.where(gt >= 0, gd, -np.inf), axis=1), 0.0)
    dl = true_delta(ids, x, q)
    hit = matches(ids, attrs, qattrs) & (dl <= (lim * (1.0 + rtol))[:, None])
    # distinct hit ids per query (a repeated id counts once)
    s = np.sort(np.where(hit, ids, -1), axis=1)
    first = np.ones_like(s, dtype=bool)
    first[:, 1:] = s[:, 1:] != s[:, :-1]
    hits = ((s >= 0) & first).sum(axis=1)
    return np.where(ng > 0, hits / np.maximum(ng, 1), 1.0)


def gamma_rel_error(ids: np.ndarray, dists: np.ndarray, x: np.ndarray, q: np.ndarray,
                    attrs: np.ndarray, qattrs: np.ndarray) -> np.ndarray:
    """|returned Gamma - FP64 Gamma| / FP64 Gamma for every returned id
    (Gamma = delta (1 + chi / m_q), Eq. 6 with the weights of Sec. 3.2)."""
    ids = np.asarray(ids)
    ok = ids >= 0
    dl = true_delta(ids, x, q)
    a = attrs[np.where(ok, ids, 0)]
    cons = (qattrs != 0xFF)[:, None, :]
    chi = ((a != qattrs[:, None, :]) & cons).sum(axis=2)
    mq = (qattrs != 0xFF).sum(axis=1)[:, None]
    g = np.where(mq > 0, dl * (1.0 + chi / np.maximum(mq, 1)), dl)
    with np.errstate(invalid="ignore"):  # padded places: inf - inf, dropped below
        err = np.abs(np.asarray(dists, dtype=np.float64) - g) / np.maximum(g, 1e-30)
    return err[ok]


def qps_at_recall(points, recalls, qps, target: float):
    """QPS at a target recall, interpolating log(QPS) linearly in recall
    between the two swept points (ordered by cost, cheapest first) that
    bracket the target.  Returns None when no point reaches the target; the
    QPS of the first point that reaches it when no cheaper one falls short
    (no extrapolation)."""
    pts = list(zip(points, recalls, qps))
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


def search_bytes_per_query(d: int, elem_bytes: int, R: int, k: int, ndc: float, hops: float,
                           scale_bytes: int = 0, rerank_rows: float = 0.0) -> float:
    """Bytes the search must move per query (HBM, algorithmic): the query
    vector, one adjacency row per expansion, the attribute word and the
    stored row (d * elem_bytes + scale) of every scored neighbour, the
    float32 rows of the exact re-score of the final candidates (precision
    form), and the written ids and distances:
      4d + H*4R + NDC*(4 + d*s_v + s_sc) + rerank_rows*4d + 8k."""
    return (4.0 * d + hops * 4.0 * R + ndc * (4.0 + d * elem_bytes + scale_bytes)
            + rerank_rows * 4.0 * d + 8.0 * k)


def search_extra_bytes_per_query(d_pad: int, elem_bytes: int, n_cand: float, out_rows: float,
                                 scale_bytes: int = 0, rerank: bool = False) -> dict:
    """Bytes the kernel moves beyond the algorithmic ones, reported apart:
    the seed candidates' re-score (position, entry id, attribute word and
    stored row of each of the n_init + margin candidates the dense ranking
    kept), the zero padding of rows to the kernel width, and -- without the
    precision form's re-score -- the float32 re-read of the output rows."""
    row = d_pad * elem_bytes + scale_bytes
    return {"seed_candidates": n_cand * (12.0 + row),
            "output_reread": 0.0 if rerank else out_rows * 4.0 * d_pad}
