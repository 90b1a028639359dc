"""CPU oracle for native hybrid queries -- TEST INFRASTRUCTURE ONLY.

Only the test suite, the smoke check and the CPU-baseline leg of the
benchmark import this package.  The product (the HIP library and its Python
binding) never imports, links or calls it; the two share no code.

Plain, slow, obviously correct FP64 reference of what the GPU path computes:

* ``nhq_oracle.c`` (built by ``oracle/build.py`` with gcc): attribute
  distance chi (Eq. 4-5), delta (Eq. 1), fusion distance Gamma (Eq. 6 with
  the default weights of Sec. 3.2), exact hybrid top-k (Def. 4), the
  composite-index build (Alg. 1 in degree-bounded form with the landing-zone
  edge selection of Sec. 4.1, Def. 7), joint pruning (Alg. 2 in beam form)
  and exact k-NN rows for graph quality (Def. 8, Eq. 7).
* this file: ctypes marshalling, the entry-point list (splitmix64),
  Recall@k (Eq. 3 with the hybrid rule of Sec. 6.1), graph quality (Eq. 7),
  the literal form of Alg. 2 for tiny hand-built graphs, the bf16 / fp8
  e4m3 storage conversions, and the FP64 reference of the small stop/beam
  network (forward, loss, analytic backward, Adam).

Readings of the paper that the oracle takes are listed in each docstring.
"""
from __future__ import annotations

import contextlib
import ctypes
import math
import os
import subprocess
import sys
from typing import Callable, Dict, List, Optional, Sequence, Tuple

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "libnhq_oracle.so")
_lib = None

KEY64 = 0
KEY32 = 1
WILDCARD = 0xFF


def build(force: bool = False) -> str:
    """Compile the C oracle with gcc (FP64, no contraction, OpenMP)."""
    src = os.path.join(_HERE, "nhq_oracle.c")
    if force or not os.path.exists(_SO) or os.path.getmtime(_SO) < os.path.getmtime(src):
        tmp = _SO + ".tmp%d" % os.getpid()
        cmd = ["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-fopenmp",
               "-ffp-contract=off", "-fno-fast-math", src, "-o", tmp, "-lm"]
        subprocess.check_call(cmd)
        os.replace(tmp, _SO)
    return _SO


def lib():
    global _lib
    if _lib is None:
        build()
        L = ctypes.CDLL(_SO)
        P = ctypes.c_void_p
        i64 = ctypes.c_int64
        i32 = ctypes.c_int
        L.or_delta2.restype = ctypes.c_double
        L.or_delta2.argtypes = [P, P, i32]
        L.or_chi.restype = i32
        L.or_chi.argtypes = [P, P, i32]
        L.or_arity.restype = i32
        L.or_arity.argtypes = [P, i32]
        L.or_gamma.restype = ctypes.c_double
        L.or_gamma.argtypes = [ctypes.c_double, i32, i32]
        L.or_order_key.restype = ctypes.c_double
        L.or_order_key.argtypes = [ctypes.c_double, i32, i32, i32]
        L.or_bruteforce.restype = None
        L.or_bruteforce.argtypes = [P, P, i64, i32, i32, P, P, i64, i32, i32, P, P, P, i32]
        L.or_build.restype = None
        L.or_build.argtypes = [P, P, i64, i32, i32, i32, i32, i32, P, i64, P, P, i32]
        L.or_knn_rows.restype = None
        L.or_knn_rows.argtypes = [P, P, i64, i32, i32, i32, P, i64, i32, P, i32]
        L.or_nndescent.restype = None
        L.or_nndescent.argtypes = [P, P, i64, i32, i32, i32, i32, i32, ctypes.c_uint64, i32, P, P, i32]
        L.or_select_lists.restype = None
        L.or_select_lists.argtypes = [P, P, i64, i32, i32, P, i32, i32, P, i32]
        L.or_nsw_insert.restype = None
        L.or_nsw_insert.argtypes = [P, P, i64, i32, i32, i32, i32, i64, i64, i32, ctypes.c_uint64, P,
                                    i32]
        L.or_build_nsw.restype = None
        L.or_build_nsw.argtypes = [P, P, i64, i32, i32, i32, i32, i64, i32, ctypes.c_uint64, P, i32]
        L.or_set_weights.restype = None
        L.or_set_weights.argtypes = [i32, ctypes.c_double]
        L.or_search.restype = None
        L.or_search.argtypes = [P, i32, P, P, P, i64, i32, i32, P, P, i64, i32, i32, P, i32,
                                i32, i32, i32, i32, i64, P, P, P, P, P, i32, P, P, P, P, P, i32,
                                P, ctypes.c_double, ctypes.c_double, i32, i32, i32, i32]
        _lib = L
    return _lib


def _threads(t: Optional[int]) -> int:
    return int(t) if t else (os.cpu_count() or 1)


def _p(a: Optional[np.ndarray]):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def _f32(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.float32)


def _u8(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.uint8)


# ------------------------------------------------------------ scalar pieces
def delta(x: np.ndarray, y: np.ndarray) -> float:
    """Eq. 1 in FP64 direct form."""
    x, y = _f32(x), _f32(y)
    return math.sqrt(lib().or_delta2(_p(x), _p(y), x.shape[0]))


def chi(qa: Sequence[int], ea: Sequence[int]) -> int:
    """Eq. 4-5 over the constrained attributes of ``qa``."""
    qa, ea = _u8(qa), _u8(ea)
    return int(lib().or_chi(_p(qa), _p(ea), qa.shape[0]))


def arity(qa: Sequence[int]) -> int:
    qa = _u8(qa)
    return int(lib().or_arity(_p(qa), qa.shape[0]))


def gamma(dlt: float, c: int, mq: int) -> float:
    """Eq. 6 under the current weight setting (default: w_v = 1 and
    w_l = delta / m_q, Sec. 3.2)."""
    return float(lib().or_gamma(float(dlt), int(c), int(mq)))


# weight settings of Sec. 6.5 (Fig. 10 (i), curves iv, i, ii, iii, v)
WEIGHTS = {"default": 0, "harmonic": 1, "harmonic_c": 2, "normalised": 3, "fixed": 4}


@contextlib.contextmanager
def weights(mode, param: float = 0.0):
    """Run the enclosed oracle calls under one weight setting of Eq. 6:
    'default' (curve iv), 'harmonic' (i), 'harmonic_c' (ii, Eq. 8 with
    c = param), 'normalised' (iii, delta_max = param) or 'fixed' (v, the
    ratio w_l / w_v = param)."""
    code = WEIGHTS[mode] if isinstance(mode, str) else int(mode)
    lib().or_set_weights(code, float(param))
    try:
        yield
    finally:
        lib().or_set_weights(0, 0.0)


def order_key(d2: float, c: int, mq: int, mode: int = KEY64) -> float:
    return float(lib().or_order_key(float(d2), int(c), int(mq), int(mode)))


# --------------------------------------------------------- exact hybrid top-k
def bruteforce(x, attrs, q, qa, k: int, by_gamma: bool = False,
               threads: Optional[int] = None):
    """Def. 4 exact answer: ids [nq,k] (-1 padded), distances [nq,k]
    (delta of each match, +inf padded), |P| per query.  by_gamma ranks every
    object by (Gamma, id) instead and returns Gamma."""
    x, attrs, q, qa = _f32(x), _u8(attrs), _f32(q), _u8(qa)
    n, d = x.shape
    m = attrs.shape[1]
    nq = q.shape[0]
    ids = np.empty((nq, k), dtype=np.int32)
    dist = np.empty((nq, k), dtype=np.float64)
    nmatch = np.empty(nq, dtype=np.int64)
    lib().or_bruteforce(_p(x), _p(attrs), n, d, m, _p(q), _p(qa), nq, k, int(by_gamma),
                        _p(ids), _p(dist), _p(nmatch), _threads(threads))
    return ids, dist, nmatch


# ------------------------------------------------------------ graph build
def build_graph(x, attrs, l: int, R: int, reverse: bool = False,
                rows: Optional[np.ndarray] = None, want_cand: bool = False,
                threads: Optional[int] = None):
    """Composite index (Alg. 1, degree-bounded; Sec. 4.1 edge selection;
    Sec. 5.1 fusion distance in the build).  Returns adj [rows, R] and, if
    asked, the candidate lists [rows, l]."""
    x, attrs = _f32(x), _u8(attrs)
    n, d = x.shape
    m = attrs.shape[1]
    rr = None if rows is None else np.ascontiguousarray(rows, dtype=np.int64)
    nr = n if rr is None else rr.shape[0]
    adj = np.empty((nr, R), dtype=np.int32)
    cand = np.empty((nr, l), dtype=np.int32) if want_cand else None
    lib().or_build(_p(x), _p(attrs), n, d, m, l, R, int(reverse), _p(rr), nr, _p(adj),
                   _p(cand), _threads(threads))
    return (adj, cand) if want_cand else adj


def nndescent(x, attrs, l: int, s: int, rounds: int, seed: int, key_mode: int = KEY32,
              threads: Optional[int] = None):
    """Candidate lists of NPG_kgraph (Sec. 4.3): random lists refined through
    neighbours of neighbours in synchronous rounds; see or_nndescent.
    Returns (ids [n, l] sorted by (key, id), updates [rounds])."""
    x, attrs = _f32(x), _u8(attrs)
    n, d = x.shape
    m = attrs.shape[1]
    if n <= l:
        raise ValueError("NN-descent needs n > l")
    ids = np.empty((n, l), dtype=np.int32)
    upd = np.zeros(max(rounds, 1), dtype=np.int64)
    lib().or_nndescent(_p(x), _p(attrs), n, d, m, int(l), int(s), int(rounds),
                       ctypes.c_uint64(int(seed) & 0xFFFFFFFFFFFFFFFF), int(key_mode), _p(ids),
                       _p(upd), _threads(threads))
    return ids, upd[:rounds]


def select_lists(x, attrs, lists, R: int, threads: Optional[int] = None) -> np.ndarray:
    """Edge selection (Sec. 4.1 (2)-(3)) over given candidate lists, each
    re-ordered by the exact FP64 key (forward pass only)."""
    x, attrs = _f32(x), _u8(attrs)
    n, d = x.shape
    m = attrs.shape[1]
    lists = np.ascontiguousarray(lists, dtype=np.int32)
    adj = np.empty((n, R), dtype=np.int32)
    lib().or_select_lists(_p(x), _p(attrs), n, d, m, _p(lists), lists.shape[1], int(R), _p(adj),
                          _threads(threads))
    return adj


def build_nsw(x, attrs, l: int, R: int, batch: int, beam: int, seed: int,
              threads: Optional[int] = None) -> np.ndarray:
    """NPG_nsw (Sec. 4.3) by insertion in batches of `batch` vertices (id
    order); see or_build_nsw.  batch = 1 inserts one vertex at a time."""
    x, attrs = _f32(x), _u8(attrs)
    n, d = x.shape
    m = attrs.shape[1]
    adj = np.empty((n, R), dtype=np.int32)
    lib().or_build_nsw(_p(x), _p(attrs), n, d, m, int(l), int(R), int(batch), int(beam),
                       ctypes.c_uint64(int(seed) & 0xFFFFFFFFFFFFFFFF), _p(adj), _threads(threads))
    return adj


def nsw_insert(x, attrs, adj_prefix, l: int, batch: int, beam: int, seed: int,
               threads: Optional[int] = None) -> np.ndarray:
    """Insertion of the rows after the prefix graph adj_prefix [s0, R] into
    it, in batches (the later batches of build_nsw).  Returns adj [n, R]."""
    x, attrs = _f32(x), _u8(attrs)
    n, d = x.shape
    m = attrs.shape[1]
    s0, R = adj_prefix.shape
    adj = np.full((n, R), -1, dtype=np.int32)
    adj[:s0] = adj_prefix
    lib().or_nsw_insert(_p(x), _p(attrs), n, d, m, int(l), int(R), int(s0), int(batch), int(beam),
                        ctypes.c_uint64(int(seed) & 0xFFFFFFFFFFFFFFFF), _p(adj), _threads(threads))
    return adj


def knn_rows(x, attrs, rows, k: int, use_attrs: bool = True,
             threads: Optional[int] = None) -> np.ndarray:
    x, attrs = _f32(x), _u8(attrs)
    n, d = x.shape
    m = attrs.shape[1]
    rr = np.ascontiguousarray(rows, dtype=np.int64)
    out = np.empty((rr.shape[0], k), dtype=np.int32)
    lib().or_knn_rows(_p(x), _p(attrs), n, d, m, int(use_attrs), _p(rr), rr.shape[0], k,
                      _p(out), _threads(threads))
    return out


def graph_quality(adj_rows: np.ndarray, knn: np.ndarray) -> float:
    """Eq. 7: mean over u of |N(u) & M(u)| / |M(u)|."""
    k = knn.shape[1]
    tot = 0.0
    for a, b in zip(adj_rows, knn):
        tot += len(set(int(v) for v in a if v >= 0) & set(int(v) for v in b if v >= 0)) / k
    return tot / max(1, adj_rows.shape[0])


# ------------------------------------------------------------ entry points
_M64 = (1 << 64) - 1


def splitmix64(state: int):
    """Steele, Lea and Flood's SplitMix64 generator (OOPSLA 2014), as a
    Python generator of 64-bit outputs."""
    while True:
        state = (state + 0x9E3779B97F4A7C15) & _M64
        z = state
        z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & _M64
        z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & _M64
        yield z ^ (z >> 31)


def entry_points(build_seed: int, n: int, n_seeds: int = 32) -> np.ndarray:
    """Seed set B of Alg. 2 (random seeds, Sec. 3.2): the
    first min(n_seeds, n) distinct values of splitmix64(build_seed) mod n."""
    want = min(n_seeds, n)
    out: List[int] = []
    seen = set()
    for z in splitmix64(build_seed):
        v = z % n
        if v not in seen:
            seen.add(v)
            out.append(v)
            if len(out) == want:
                break
    return np.asarray(out, dtype=np.int32)


def _splitmix64_first(states: np.ndarray) -> np.ndarray:
    """The first splitmix64 output (Steele, Lea and Flood) from each uint64
    state: z = s + 0x9E3779B97F4A7C15, then the two xor-shift-multiply
    rounds and a final xor-shift (wrapping uint64 arithmetic)."""
    with np.errstate(over="ignore"):
        z = states + np.uint64(0x9E3779B97F4A7C15)
        z = (z ^ (z >> np.uint64(30))) * np.uint64(0xBF58476D1CE4E5B9)
        z = (z ^ (z >> np.uint64(27))) * np.uint64(0x94D049BB133111EB)
        return z ^ (z >> np.uint64(31))


def entry_strata(build_seed: int, attrs, per_pattern: int):
    """Stratified seed sets (the flagged entry-sample option): for every code
    tuple the objects hold, the min(per_pattern, count) objects of that tuple
    with the smallest (h(i), i), h(i) = the first splitmix64 output from
    state (seed ^ 0x8F14E45FCEEA167A) ^ (i * 0xD1B54A32D192ED03) mod 2^64.
    Returns {code tuple: int32 ids in (h, id) order}.  Seeds stay random
    (Sec. 3.2), within each attribute pattern."""
    attrs = _u8(attrs)
    n = attrs.shape[0]
    i = np.arange(n, dtype=np.uint64)
    with np.errstate(over="ignore"):
        states = np.uint64((build_seed ^ 0x8F14E45FCEEA167A) & 0xFFFFFFFFFFFFFFFF) ^ (
            i * np.uint64(0xD1B54A32D192ED03))
    h = _splitmix64_first(states)
    out = {}
    tuples = [tuple(int(c) for c in row) for row in attrs]
    groups: Dict[Tuple[int, ...], List[int]] = {}
    for v, t in enumerate(tuples):
        groups.setdefault(t, []).append(v)
    for t, ids in groups.items():
        ids = sorted(ids, key=lambda v: (int(h[v]), v))[:per_pattern]
        out[t] = np.asarray(ids, dtype=np.int32)
    return out


def search_strata(adj, xs, attrs, q, qa, k: int, L: int, global_seeds, strata, **kw):
    """Joint pruning (``search``) where each query draws its seed set from
    the stratified sample: a query that constrains every attribute takes the
    block of its code tuple (when an object holds it), any other query the
    global sample.  Same outputs as ``search``."""
    q, qa = _f32(q), _u8(qa)
    nq = q.shape[0]
    key = [tuple(int(c) for c in row) if (row != WILDCARD).all() else None for row in qa]
    groups: Dict[object, List[int]] = {}
    for i, t in enumerate(key):
        groups.setdefault(t if t in strata else None, []).append(i)
    res = None
    for t, rows in groups.items():
        rows = np.asarray(rows)
        seeds = strata[t] if t is not None else np.asarray(global_seeds, dtype=np.int32)
        o = search(adj, xs, attrs, q[rows], qa[rows], k, L, seeds, **kw)
        if res is None:
            res = [np.empty((nq,) + a.shape[1:], dtype=a.dtype) if isinstance(a, np.ndarray) else None
                   for a in o]
        for r, a in zip(res, o):
            if isinstance(a, np.ndarray):
                r[rows] = a
    return tuple(res)


# ------------------------------------------------------------ Alg. 2
def search(adj, xs, attrs, q, qa, k: int, L: int, seeds, n_init: int = 32, key_mode: int = KEY64,
           out_mode: int = 0, rerank_n: int = 0, xr=None, max_hops: int = 1 << 40,
           threads: Optional[int] = None, check_every: int = 0, trace_cap: int = 0,
           mlp: Optional[np.ndarray] = None, stop_threshold: float = 0.5, cap_factor: float = 0.0,
           expand: int = 1, learned_mode: int = 1, route_h: int = 0):
    """Joint pruning in beam form; see ``or_search`` in nhq_oracle.c.
    Returns (ids [nq,k], gamma [nq,k], ndc [nq], hops [nq], flag [nq]); with
    trace_cap > 0 also a dict of checkpoint traces (feat [nq,cap,8], hop,
    hash, count, final_hash).  ``mlp`` (float64 [4866], weights as the GPU
    holds them) turns on the learned stop with threshold stop_threshold;
    learned_mode 2 evaluates it at the first checkpoint only, whose beam
    output (times cap_factor) then bounds the hops; learned_mode 3 (the
    beam-width predictor) evaluates it at the first checkpoint only and takes
    ceil(cap_factor * 2^z1), clamped to [k, L], as the pool size from there
    on (the pool keeps its best entries).
    ``expand`` E > 1 expands the E best unexpanded entries per step (a
    batched form of the algorithm's expansion loop; E = 1 is Alg. 2 itself).
    ``route_h`` h >= 2 runs two-stage routing (Sec. 4.2): a first stage that
    looks at a random 1-in-h subset of each expanded vertex's neighbours until
    a step adds nothing to the pool, then Alg. 2 over the whole pool."""
    adj = np.ascontiguousarray(adj, dtype=np.int32)
    xs, attrs, q, qa = _f32(xs), _u8(attrs), _f32(q), _u8(qa)
    xr = None if xr is None else _f32(xr)
    seeds = np.ascontiguousarray(seeds, dtype=np.int32)
    n, d = xs.shape
    m = attrs.shape[1]
    R = adj.shape[1]
    nq = q.shape[0]
    ids = np.empty((nq, k), dtype=np.int32)
    gam = np.empty((nq, k), dtype=np.float64)
    ndc = np.empty(nq, dtype=np.int64)
    hops = np.empty(nq, dtype=np.int64)
    flag = np.empty(nq, dtype=np.int32)
    tr = None
    if trace_cap > 0:
        tr = {"feat": np.zeros((nq, trace_cap, 8)), "hop": np.zeros((nq, trace_cap), np.uint32),
              "hash": np.zeros((nq, trace_cap), np.uint32), "count": np.zeros(nq, np.int32),
              "final_hash": np.zeros(nq, np.uint32)}
    w = None if mlp is None else np.ascontiguousarray(mlp, dtype=np.float64)
    logit = math.log(stop_threshold / (1.0 - stop_threshold))
    lib().or_search(_p(adj), R, _p(xs), _p(xr), _p(attrs), n, d, m, _p(q), _p(qa), nq, k, L,
                    _p(seeds), seeds.shape[0], int(n_init), key_mode, out_mode, rerank_n, max_hops,
                    _p(ids), _p(gam), _p(ndc), _p(hops), _p(flag), int(check_every),
                    _p(tr["feat"]) if tr else None, _p(tr["hop"]) if tr else None,
                    _p(tr["hash"]) if tr else None, _p(tr["count"]) if tr else None,
                    _p(tr["final_hash"]) if tr else None, int(trace_cap), _p(w), logit,
                    float(cap_factor), int(learned_mode), int(expand), int(route_h), _threads(threads))
    if tr is not None:
        return ids, gam, ndc, hops, flag, tr
    return ids, gam, ndc, hops, flag


def alg2_literal(neighbours: Dict[int, Sequence[int]], dist: Callable[[int], float],
                 seeds: Sequence[int], k: int):
    """Alg. 2 as printed, for tiny hand-built graphs: C and R start as the
    seed set; repeatedly take the vertex of C with the smallest Gamma out of
    C, add its neighbours to C, and let each neighbour replace the current
    worst member of R when strictly closer.  Stops after the first round that
    leaves R unchanged.  Readings: a vertex already in R is not added twice;
    ties broken by the smaller id.  Returns (R sorted by (Gamma, id), the
    expansion order)."""
    C = set(seeds)
    Rs = sorted(set(seeds), key=lambda v: (dist(v), v))[:k]
    order = []
    while C:
        ui = min(C, key=lambda v: (dist(v), v))
        C.discard(ui)
        order.append(ui)
        nb = list(neighbours.get(ui, ()))
        C.update(nb)
        changed = False
        for uj in nb:
            if uj in Rs:
                continue
            if len(Rs) < k:
                Rs.append(uj)
                changed = True
                continue
            ur = max(Rs, key=lambda v: (dist(v), v))
            if dist(uj) < dist(ur):
                Rs.remove(ur)
                Rs.append(uj)
                changed = True
        if not changed:
            break
    return sorted(Rs, key=lambda v: (dist(v), v)), order


# ------------------------------------------------------------ Recall@k
def recall(ids: np.ndarray, x, attrs, q, qa, gt_ids: np.ndarray, gt_dist: np.ndarray,
           k: int) -> np.ndarray:
    """Eq. 3 with the hybrid rule (Sec. 6.1, Metrics): per query,
    hits / min(k, |P|).  A returned id is a hit iff it matches the query's
    attributes, is not repeated, and its delta is <= the delta of the last
    exact answer (ties at the k-th distance count).  Queries with |P| = 0
    score 1."""
    x, attrs, q, qa = _f32(x), _u8(attrs), _f32(q), _u8(qa)
    nq = ids.shape[0]
    out = np.empty(nq, dtype=np.float64)
    for i in range(nq):
        gt = [int(v) for v in gt_ids[i, :k] if v >= 0]
        if not gt:
            out[i] = 1.0
            continue
        lim = float(gt_dist[i, len(gt) - 1])
        seen = set()
        hits = 0
        for v in ids[i, :k]:
            v = int(v)
            if v < 0 or v in seen:
                continue
            seen.add(v)
            if chi(qa[i], attrs[v]) != 0:
                continue
            if delta(q[i], x[v]) <= lim * (1.0 + 1e-12):
                hits += 1
        out[i] = hits / len(gt)
    return out


# ------------------------------------------------------------ conversions
def to_bf16_bits(x) -> np.ndarray:
    """float32 -> bfloat16 bit patterns, round to nearest even, NaN kept
    quiet."""
    u = np.ascontiguousarray(x, dtype=np.float32).view(np.uint32).astype(np.uint64)
    nan = (u & 0x7FFFFFFF) > 0x7F800000
    r = (u + 0x7FFF + ((u >> 16) & 1)) >> 16
    r = np.where(nan, (u >> 16) | 0x40, r)
    return r.astype(np.uint16)


def from_bf16_bits(b) -> np.ndarray:
    return (np.asarray(b, dtype=np.uint32) << 16).view(np.float32)


def e4m3_decode(code: int) -> float:
    """OCP FP8 E4M3 ("FN"): sign, 4 exponent bits (bias 7), 3 mantissa bits;
    no infinities; S.1111.111 is NaN; largest finite 448."""
    s = -1.0 if code & 0x80 else 1.0
    e = (code >> 3) & 0xF
    mnt = code & 0x7
    if e == 0xF and mnt == 0x7:
        return float("nan")
    if e == 0:
        return s * (mnt / 8.0) * 2.0 ** (-6)
    return s * (1.0 + mnt / 8.0) * 2.0 ** (e - 7)


_E4M3_POS = np.array([e4m3_decode(c) for c in range(0x7F)], dtype=np.float64)


def to_e4m3(x) -> np.ndarray:
    """float -> E4M3 codes: nearest representable value, ties to the even
    code, saturating to +-448 (no NaN produced for finite input)."""
    x = np.asarray(x, dtype=np.float64)
    a = np.minimum(np.abs(x), 448.0)
    idx = np.searchsorted(_E4M3_POS, a)           # first >= a
    idx = np.clip(idx, 1, 0x7E)
    lo, hi = idx - 1, idx
    dlo = a - _E4M3_POS[lo]
    dhi = _E4M3_POS[hi] - a
    pick = np.where(dlo < dhi, lo, np.where(dhi < dlo, hi, np.where(lo % 2 == 0, lo, hi)))
    pick = np.where(a >= 448.0, 0x7E, pick)
    pick = np.where(a == 0.0, 0, pick)
    sign = np.where(np.signbit(x), 0x80, 0)
    return (pick | sign).astype(np.uint8)


def e4m3_table() -> np.ndarray:
    return np.array([e4m3_decode(c) for c in range(256)], dtype=np.float64)


def fp8_rows(x) -> Tuple[np.ndarray, np.ndarray]:
    """Per-vector scaling: s = max|x| / 448 (1 for an all-zero row); codes
    e4m3(x / s).  Returns (codes [n,d], scales [n] float32)."""
    x = np.asarray(x, dtype=np.float32)
    mx = np.abs(x).max(axis=1).astype(np.float32)
    s = np.where(mx > 0, mx / np.float32(448.0), np.float32(1.0)).astype(np.float32)
    codes = to_e4m3(x.astype(np.float64) / s.astype(np.float64)[:, None])
    return codes, s


def fp8_decode_rows(codes, scales) -> np.ndarray:
    t = e4m3_table()
    return t[np.asarray(codes)] * np.asarray(scales, dtype=np.float64)[:, None]


# ------------------------------------------------------------ stop/beam network
class MLPRef:
    """FP64 reference of the 8 -> 64 -> 64 -> 2 network with ReLU.
    Output 0 is the stop logit (binary cross-entropy), output 1 the
    predicted log2 beam (Huber loss, weight lam).  Parameters are a dict of
    numpy float64 arrays: W1 [64,8], b1 [64], W2 [64,64], b2 [64],
    W3 [2,64], b3 [2]."""

    SHAPES = {"W1": (64, 8), "b1": (64,), "W2": (64, 64), "b2": (64,),
              "W3": (2, 64), "b3": (2,)}

    @staticmethod
    def forward(p, X):
        a1 = X @ p["W1"].T + p["b1"]
        h1 = np.maximum(a1, 0.0)
        a2 = h1 @ p["W2"].T + p["b2"]
        h2 = np.maximum(a2, 0.0)
        z = h2 @ p["W3"].T + p["b3"]
        return z, (X, a1, h1, a2, h2)

    @staticmethod
    def loss(z, y_stop, y_beam, lam: float = 1.0, hub: float = 1.0) -> float:
        z0, z1 = z[:, 0], z[:, 1]
        bce = np.logaddexp(0.0, z0) - y_stop * z0
        r = z1 - y_beam
        ar = np.abs(r)
        hl = np.where(ar <= hub, 0.5 * r * r, hub * (ar - 0.5 * hub))
        return float(np.mean(bce) + lam * np.mean(hl))

    @staticmethod
    def backward(p, cache, z, y_stop, y_beam, lam: float = 1.0, hub: float = 1.0):
        X, a1, h1, a2, h2 = cache
        B = X.shape[0]
        dz = np.empty_like(z)
        dz[:, 0] = (1.0 / (1.0 + np.exp(-z[:, 0])) - y_stop) / B
        r = z[:, 1] - y_beam
        dz[:, 1] = lam * np.clip(r, -hub, hub) / B
        g = {}
        g["W3"] = dz.T @ h2
        g["b3"] = dz.sum(0)
        dh2 = dz @ p["W3"]
        da2 = dh2 * (a2 > 0)
        g["W2"] = da2.T @ h1
        g["b2"] = da2.sum(0)
        dh1 = da2 @ p["W2"]
        da1 = dh1 * (a1 > 0)
        g["W1"] = da1.T @ X
        g["b1"] = da1.sum(0)
        return g

    @staticmethod
    def adam(p, g, state, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
        """Adam (Kingma and Ba, 2015) with bias correction; state holds t,
        m and v per parameter."""
        state["t"] = state.get("t", 0) + 1
        t = state["t"]
        for name in p:
            mo = state.setdefault("m_" + name, np.zeros_like(p[name]))
            ve = state.setdefault("v_" + name, np.zeros_like(p[name]))
            mo[...] = b1 * mo + (1 - b1) * g[name]
            ve[...] = b2 * ve + (1 - b2) * g[name] ** 2
            mh = mo / (1 - b1 ** t)
            vh = ve / (1 - b2 ** t)
            p[name] = p[name] - lr * mh / (np.sqrt(vh) + eps)
        return p

    @staticmethod
    def init(seed: int = 0):
        rng = np.random.default_rng(seed)
        p = {}
        for name, shp in MLPRef.SHAPES.items():
            if name.startswith("W"):
                p[name] = rng.standard_normal(shp) * math.sqrt(2.0 / shp[1])
            else:
                p[name] = np.zeros(shp)
        return p
