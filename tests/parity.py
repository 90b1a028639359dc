"""Comparisons of GPU results with the oracle's for float data, where the
two orders may differ only at near-ties (float32 against FP64 keys)."""
import numpy as np

import oracle


def result_overlap(ids, oids):
    """Mean over queries of |A & B| / max(|A|, |B|) for the returned sets A
    (GPU) and B (oracle), -1 padding dropped; two empty answers agree."""
    out = []
    for a, b in zip(ids, oids):
        sa, sb = set(a[a >= 0].tolist()), set(b[b >= 0].tolist())
        out.append(1.0 if not sa and not sb else len(sa & sb) / max(len(sa), len(sb)))
    return float(np.mean(out))


def recalls(ids, oids, x, attrs, q, qa, k=10):
    """Recall@k (Eq. 3, hybrid rule) of both answers against the exact one."""
    gi, gd, _ = oracle.bruteforce(x, attrs, q, qa, k)
    return (float(oracle.recall(ids, x, attrs, q, qa, gi, gd, k).mean()),
            float(oracle.recall(oids, x, attrs, q, qa, gi, gd, k).mean()))


def assert_float_parity(ids, oids, x, attrs, q, qa, k=10, min_overlap=0.99, recall_tol=0.005):
    ov = result_overlap(ids, oids)
    assert ov >= min_overlap, ov
    rg, ro = recalls(ids, oids, x, attrs, q, qa, k)
    assert abs(rg - ro) <= recall_tol, (rg, ro)
    return ov, rg, ro
