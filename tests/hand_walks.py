"""Hand-built search walks whose checkpoint features are worked out by hand.

The eight search-state features read by the stop network (the library's own
design: the paper names learned routing only as prior art, Sec. 4.2) are, at
a checkpoint taken every S expansions before the next step:
  f1 = ln(1 + H) / 8                      H: expansions so far
  f2 = ln(1 + NDC) / 8                    NDC: neighbour distance evaluations
  f3 = sum of ln(count(code) / n) over the constrained attributes, / 8
  f4 = eligible entries (attribute matches) among the first k pool places / k
  f5 = ln(k-th eligible key / that key at its first checkpoint), 1 before
  f6 = ln(key of the next entry to expand / k-th eligible key), -1 before
  f7 = entries that joined the pool since the last checkpoint / (S R); an
       entry joins in a step when it is still pooled after all of that
       step's neighbours have been offered
  f8 = min((H - H at the last change of the eligible top-k) / 64, 1)
Keys are delta^2 (m_q + chi)^2 with m_q = 1 here, so a matching object at
distance x has key x^2 and a mismatched one 4 x^2.  Every walk below is a
one-dimensional object set with the query at 0; the comments follow each
step (pool entries are written vertex(key), * = expanded).
"""
import math

ln = math.log


def chain():
    """E = 1, S = 1, k = 2, L = 3, R = 2, seed v0.

    init: pool v0(100)
    step 1 expands v0: v1(324, mismatch) and v2(64) join -> v2 v0* v1; NDC 2
    ckpt H=1: top-2 eligible {v2, v0}, k-th key 100 (first); next v2(64)
    step 2 expands v2: v4(36), v3(49) join (v1, then v0 pushed out)
            -> v4 v3 v2*; NDC 4
    ckpt H=2: top-2 {v4, v3} changed; k-th 49; next v4(36)
    step 3 expands v4: v5(16, mismatch) joins -> v5 v4* v3; NDC 5
    ckpt H=3: eligible v4 (place 1), v3 (place 2): f4 = 1/2, top-2 {v4, v3}
            unchanged, k-th 49; next v5(16)
    step 4 expands v5: v6(9) joins, v2 already visited -> v6 v5* v4*; NDC 6
    ckpt H=4: top-2 {v6, v4} changed; k-th 36; next v6(9)
    step 5 expands v6 (no neighbours); every entry expanded: H = 5, NDC = 6.
    v1 was pushed out before its expansion, so v7 is never reached.
    """
    x = [10.0, 9.0, 8.0, 7.0, 6.0, 2.0, 3.0, 1.0]
    attrs = [0, 1, 0, 0, 0, 1, 0, 0]
    adj = [[1, 2], [7, -1], [4, 3], [-1, -1], [5, -1], [6, 2], [-1, -1], [-1, -1]]
    ls = ln(6 / 8) / 8  # six of the eight objects hold code 0
    feat = [
        [ln(2) / 8, ln(3) / 8, ls, 1.0, 0.0, ln(64 / 100), 2 / 2, 1 / 64],
        [ln(3) / 8, ln(5) / 8, ls, 1.0, ln(49 / 100), ln(36 / 49), 2 / 2, 0.0],
        [ln(4) / 8, ln(6) / 8, ls, 0.5, ln(49 / 100), ln(16 / 49), 1 / 2, 1 / 64],
        [ln(5) / 8, ln(7) / 8, ls, 0.5, ln(36 / 100), ln(9 / 36), 1 / 2, 0.0],
    ]
    return dict(x=x, attrs=attrs, adj=adj, k=2, L=3, seeds=[0], expand=1, check_every=1,
                feat=feat, hop=[1, 2, 3, 4], topk=[[2, 0], [4, 3], [4, 3], [6, 4]],
                ids=[6, 4], gamma=[3.0, 6.0], ndc=6, hops=5)


def wide_step(check_every=1):
    """E = 2, R = 64, k = 1, L = 64, seeds v0 (x 200) and v1 (x 201).

    v0's 64 neighbours F_i (ids 2..65, x = 100 + i) come first in the step,
    v1's 64 neighbours N_i (ids 66..129, x = 1 + i) after them.  Offered in
    that order, the F_i fill the pool and are then all pushed out by the N_i:
    the step ends with the pool N_0 .. N_63, so 64 entries joined (not 128).
    The N_i have no neighbours; they are expanded two per step.
    ckpt H=2: NDC 128, top-1 N_0 (key 1), next N_0: f6 = ln(1/1)
    ckpt H=4 (S = 1): nothing joined in the step, next N_2 (key 9), top-1
            unchanged since H = 0 (f8 = 4/64)
    The search ends after 33 steps: H = 66, NDC = 128.
    """
    n = 130
    x = [200.0, 201.0] + [100.0 + i for i in range(64)] + [1.0 + i for i in range(64)]
    attrs = [0] * n
    adj = [[-1] * 64 for _ in range(n)]
    adj[0] = list(range(2, 66))
    adj[1] = list(range(66, 130))
    S = check_every
    if S == 1:
        feat = [[ln(3) / 8, ln(129) / 8, 0.0, 1.0, 0.0, 0.0, 64 / 64, 2 / 64],
                [ln(5) / 8, ln(129) / 8, 0.0, 1.0, 0.0, ln(9), 0.0, 4 / 64]]
        hop = [2, 4]
    else:  # S = 2: checkpoints at H = 2, 4, ... as well
        feat = [[ln(3) / 8, ln(129) / 8, 0.0, 1.0, 0.0, 0.0, 64 / 128, 2 / 64],
                [ln(5) / 8, ln(129) / 8, 0.0, 1.0, 0.0, ln(9), 0.0, 4 / 64]]
        hop = [2, 4]
    return dict(x=x, attrs=attrs, adj=adj, k=1, L=64, seeds=[0, 1], expand=2, check_every=S,
                feat=feat, hop=hop, topk=[[66], [66]], ids=[66], gamma=[1.0], ndc=128, hops=66)


def fmix32(h):
    """MurmurHash3's 32-bit finaliser (the top-k fingerprint's mixer)."""
    h ^= h >> 16
    h = (h * 0x85EBCA6B) & 0xFFFFFFFF
    h ^= h >> 13
    h = (h * 0xC2B2AE35) & 0xFFFFFFFF
    return h ^ (h >> 16)


def fingerprint(ids):
    return sum(fmix32((int(v) + 0x9E3779B9) & 0xFFFFFFFF) for v in ids) & 0xFFFFFFFF
