"""ctypes binding of libnhq: argument marshalling only.

Every function here has the name of the C entry point it calls and does no
arithmetic of the method: it checks shapes and dtypes, passes device
pointers and the current HIP stream of torch, and turns error codes into
``NHQError``.  Tensors must live on the GPU the index was created on.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional, Tuple

import numpy as np
import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libnhq.so")

STORAGE = {"fp32": 0, "bf16": 1, "fp8": 2}
DEVERR_HOPCAP = 0x1
DEVERR_BADID = 0x2


class NHQError(RuntimeError):
    def __init__(self, code: int, where: str, msg: str):
        super().__init__("%s failed (%d): %s" % (where, code, msg))
        self.code = code


class BuildParams(ctypes.Structure):
    _fields_ = [("degree", ctypes.c_int32), ("cand", ctypes.c_int32),
                ("reverse_edges", ctypes.c_int32), ("storage", ctypes.c_int32),
                ("n_entry", ctypes.c_int32), ("weights", ctypes.c_int32),
                ("seed", ctypes.c_uint64), ("weight_param", ctypes.c_double),
                ("builder", ctypes.c_int32), ("nnd_rounds", ctypes.c_int32),
                ("nnd_sample", ctypes.c_int32), ("nnd_stop", ctypes.c_float),
                ("nsw_batch", ctypes.c_int32), ("nsw_beam", ctypes.c_int32),
                ("capacity", ctypes.c_int64), ("entry_per_pattern", ctypes.c_int32)]


class Trace(ctypes.Structure):
    _fields_ = [("feat", ctypes.c_void_p), ("hop", ctypes.c_void_p), ("hash", ctypes.c_void_p),
                ("count", ctypes.c_void_p), ("final_hash", ctypes.c_void_p), ("cap", ctypes.c_int32)]


class SearchParams(ctypes.Structure):
    _fields_ = [("n_init", ctypes.c_int32), ("rerank", ctypes.c_int32),
                ("output_mode", ctypes.c_int32), ("max_hops", ctypes.c_int32),
                ("visited_log2", ctypes.c_int32), ("learned", ctypes.c_int32),
                ("stop_threshold", ctypes.c_float), ("check_every", ctypes.c_int32),
                ("counters", ctypes.c_void_p), ("cap_factor", ctypes.c_float),
                ("trace", ctypes.c_void_p), ("expand", ctypes.c_int32),
                ("route_h", ctypes.c_int32), ("order", ctypes.c_void_p)]


MLP_PARAMS = 4866
SERVE_RAW = 1
PENDING = 1


class ServerParams(ctypes.Structure):
    _fields_ = [("beam_small", ctypes.c_int32), ("beam_large", ctypes.c_int32),
                ("slots_small", ctypes.c_int32), ("slots_large", ctypes.c_int32),
                ("ring", ctypes.c_int32), ("max_k", ctypes.c_int32), ("n_init", ctypes.c_int32),
                ("expand", ctypes.c_int32), ("rerank", ctypes.c_int32), ("check_every", ctypes.c_int32),
                ("auto_beam", ctypes.c_int32), ("max_hops", ctypes.c_int32),
                ("stop_threshold", ctypes.c_float), ("cap_factor", ctypes.c_float),
                ("learned_mode", ctypes.c_int32), ("reserved1", ctypes.c_int32),
                ("lifetime_s", ctypes.c_double)]


_lib = None


def lib() -> ctypes.CDLL:
    """Load libnhq.so (after torch, so both use torch's HIP runtime).  Fails
    loudly when the library has not been built: there is no fallback."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError("libnhq.so is not built (run __graft_entry__.build() or "
                          "python -m paper_2203_13601_amd.build_lib)")
    L = ctypes.CDLL(LIB_PATH)
    P, i32, i64, u32 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_uint32
    sig = {
        "nhq_index_create": ([P, P, i64, i32, i32, P, P, P], i32),
        "nhq_index_build_graph": ([P, P], i32),
        "nhq_nndescent_lists": ([P, i32, i32, i32, ctypes.c_double, ctypes.c_uint64, P, P, P, P], i32),
        "nhq_index_build_report": ([P, P], i32),
        "nhq_index_insert": ([P, P, P, i64, P], i32),
        "nhq_build_index": ([P, P, i64, i32, i32, P, P, P], i32),
        "nhq_index_set_graph": ([P, P, i32, P], i32),
        "nhq_index_get_graph": ([P, P, P], i32),
        "nhq_index_get_entry": ([P, P, P], i32),
        "nhq_index_entry_blocks": ([P, P, P, P, P, P], i32),
        "nhq_index_info": ([P, P, P, P, P, P, P], i32),
        "nhq_index_get_storage": ([P, P, P, P, P], i32),
        "nhq_index_device_error": ([P, P, P], i32),
        "nhq_index_free": ([P], None),
        "nhq_index_save": ([P, ctypes.c_char_p, P], i32),
        "nhq_index_load": ([ctypes.c_char_p, P, P], i32),
        "nhq_hybrid_search": ([P, P, P, i64, i32, i32, P, P, P, P], i32),
        "nhq_bruteforce_hybrid_knn": ([P, P, P, i64, i32, P, P, P], i32),
        "nhq_hybrid_search_noalloc": ([P, P, P, i64, i32, i32, P, P, P, P], i32),
        "nhq_seed_rank": ([P, P, P, i64, i32, P, P], i32),
        "nhq_seed_rank_workspace_size": ([P, i64, i32, P], i32),
        "nhq_seed_rank_ws": ([P, P, P, i64, i32, P, P, ctypes.c_size_t, P], i32),
        "nhq_search_seeded": ([P, P, P, i64, P, i32, i32, i32, P, P, P, P], i32),
        "nhq_query_order": ([P, P, i64, P, P], i32),
        "nhq_seed_order": ([P, P, i32, i64, P, P, ctypes.c_size_t, P], i32),
        "nhq_trace_samples": ([P, i64, P, P, P, P, P, P], i32),
        "nhq_mlp_grad": ([P, P, P, P, i64, ctypes.c_float, P, P, P, P], i32),
        "nhq_mlp_train": ([P, P, P, P, P, P, i64, i32, i32, ctypes.c_float, ctypes.c_float,
                           ctypes.c_uint64, P, P], i32),
        "nhq_mlp_load": ([P, P, P], i32),
        "nhq_mlp_eval": ([P, P, i64, P, P], i32),
        "nhq_server_create": ([P, P, P], i32),
        "nhq_server_info": ([P, P, P, P, P], i32),
        "nhq_server_submit": ([P, P, P, i32, i32, i32, P], i32),
        "nhq_server_poll": ([P, ctypes.c_uint64, P, P, P, P], i32),
        "nhq_server_run": ([P, P, P, P, P, P, P, i64, P, P, P, P, P, P, ctypes.c_double], i32),
        "nhq_server_free": ([P], i32),
        "nhq_gather_probe": ([P, i64, i32, ctypes.c_uint64, P, P, P], i32),
        "nhq_strerror": ([i32], ctypes.c_char_p),
        "nhq_last_error": ([], ctypes.c_char_p),
        "nhq_version": ([], i32),
    }
    for name, (args, res) in sig.items():
        f = getattr(L, name)
        f.argtypes = args
        f.restype = res
    _lib = L
    return L


def _check(rc: int, where: str) -> None:
    if rc != 0:
        L = lib()
        raise NHQError(rc, where, L.nhq_last_error().decode() or L.nhq_strerror(rc).decode())


def _stream(stream=None) -> ctypes.c_void_p:
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def _query_inputs(ix: "Index", queries: torch.Tensor, qattrs: torch.Tensor):
    """Checks queries float32 [nq][d] and qattrs uint8 [nq][m] against the
    index (shapes first, then the device), returns contiguous tensors."""
    d, m = ix.dims()
    for name, t, dt, wd in (("queries", queries, torch.float32, d), ("qattrs", qattrs, torch.uint8, m)):
        if not isinstance(t, torch.Tensor):
            raise TypeError("%s must be a tensor" % name)
        if t.dtype != dt:
            raise TypeError("%s must be %s, got %s" % (name, dt, t.dtype))
        if t.dim() != 2 or t.shape[1] != wd:
            raise ValueError("%s must be [nq][%d] for this index, got %s" % (name, wd, tuple(t.shape)))
    if qattrs.shape[0] != queries.shape[0]:
        raise ValueError("queries and qattrs differ in rows")
    for name, t in (("queries", queries), ("qattrs", qattrs)):
        if t.device != ix.device:
            raise ValueError("%s must be on the index's device %s, got %s" % (name, ix.device, t.device))
    return queries.contiguous(), qattrs.contiguous()


def _out_pair(ix: "Index", out, nq: int, k: int):
    """The (ids int32 [nq][k], dists float32 [nq][k]) outputs: new tensors,
    or the caller's after checking shape, dtype, contiguity and device."""
    if out is None:
        return (torch.empty((nq, k), dtype=torch.int32, device=ix.device),
                torch.empty((nq, k), dtype=torch.float32, device=ix.device))
    ids, dists = out
    for name, t, dt in (("out ids", ids, torch.int32), ("out dists", dists, torch.float32)):
        if not isinstance(t, torch.Tensor) or t.dtype != dt:
            raise TypeError("%s must be a %s tensor" % (name, dt))
        if tuple(t.shape) != (nq, k):
            raise ValueError("%s must be [%d][%d], got %s" % (name, nq, k, tuple(t.shape)))
        if not t.is_contiguous():
            raise ValueError("%s must be contiguous" % name)
        if t.device != ix.device:
            raise ValueError("%s must be on the index's device %s" % (name, ix.device))
    return ids, dists


def _dev(t: torch.Tensor, dtype, name: str, ndim: int) -> torch.Tensor:
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError("%s must be a CUDA (HIP) tensor" % name)
    if t.dtype != dtype:
        raise TypeError("%s must be %s, got %s" % (name, dtype, t.dtype))
    if t.dim() != ndim:
        raise ValueError("%s must have %d dimensions" % (name, ndim))
    return t.contiguous()


class Index:
    """Owning handle of an nhq_index.  Remembers the device it lives on and
    (once read) its vector width d and attribute count m, against which the
    wrappers check every query tensor before a pointer reaches the library
    (the C calls take no widths)."""

    def __init__(self, handle: ctypes.c_void_p, keep=(), device=None, d=None, m=None):
        self._h = handle
        self._keep = keep
        if device is None:
            device = torch.device("cuda", torch.cuda.current_device())
        self.device = torch.device(device)
        self._d, self._m = d, m

    def dims(self) -> Tuple[int, int]:
        """(d, m) of the index."""
        if self._d is None:
            info = nhq_index_info(self)
            self._d, self._m = info["d"], info["m"]
        return self._d, self._m

    @property
    def handle(self) -> ctypes.c_void_p:
        if not self._h:
            raise ValueError("index was freed")
        return self._h

    def free(self) -> None:
        if self._h:
            lib().nhq_index_free(self._h)
            self._h = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


# weight settings of Gamma (Eq. 6; compared in Sec. 6.5)
WEIGHTS = {"default": 0, "harmonic": 1, "harmonic_c": 2, "normalised": 3, "fixed": 4}


BUILDERS = {"exact": 0, "nndescent": 1, "nsw": 2}


def _params(degree=32, cand=64, reverse_edges=False, storage="fp32", n_entry=1024, seed=0,
            weights="default", weight_param=0.0, builder="exact", nnd_rounds=0, nnd_sample=0,
            nnd_stop=0.0, nsw_batch=0, nsw_beam=0, capacity=0, entry_per_pattern=0):
    return BuildParams(int(degree), int(cand), int(bool(reverse_edges)),
                       STORAGE[storage] if isinstance(storage, str) else int(storage),
                       int(n_entry), WEIGHTS[weights] if isinstance(weights, str) else int(weights),
                       int(seed), float(weight_param),
                       BUILDERS[builder] if isinstance(builder, str) else int(builder),
                       int(nnd_rounds), int(nnd_sample), float(nnd_stop), int(nsw_batch),
                       int(nsw_beam), int(capacity), int(entry_per_pattern))


def nhq_index_create(vecs: torch.Tensor, attrs: torch.Tensor, stream=None, **params) -> Index:
    vecs = _dev(vecs, torch.float32, "vecs", 2)
    attrs = _dev(attrs, torch.uint8, "attrs", 2)
    if attrs.shape[0] != vecs.shape[0]:
        raise ValueError("vecs and attrs differ in rows")
    p = _params(**params)
    h = ctypes.c_void_p()
    _check(lib().nhq_index_create(vecs.data_ptr(), attrs.data_ptr(), vecs.shape[0], vecs.shape[1],
                                  attrs.shape[1], ctypes.byref(p), _stream(stream), ctypes.byref(h)),
           "nhq_index_create")
    return Index(h, device=vecs.device, d=vecs.shape[1], m=attrs.shape[1])


def nhq_nndescent_lists(ix: Index, l: int, s: int, rounds: int, seed: int, stop_frac: float = 0.0,
                        stream=None):
    """NN-descent candidate lists (Sec. 4.3): (ids int32 [n, l] on the
    device, updates per round as a numpy int64 array, rounds run)."""
    n = nhq_index_info(ix)["n"]
    dev = torch.device("cuda", torch.cuda.current_device())
    ids = torch.empty((n, l), dtype=torch.int32, device=dev)
    upd = np.zeros(max(rounds, 1), dtype=np.int64)
    done = ctypes.c_int32()
    _check(lib().nhq_nndescent_lists(ix.handle, int(l), int(s), int(rounds), float(stop_frac),
                                     ctypes.c_uint64(int(seed) & 0xFFFFFFFFFFFFFFFF), ids.data_ptr(),
                                     upd.ctypes.data, ctypes.byref(done), _stream(stream)),
           "nhq_nndescent_lists")
    return ids, upd[:done.value], done.value


def nhq_index_insert(ix: Index, vecs: torch.Tensor, attrs: torch.Tensor, stream=None) -> None:
    """Append objects (ids n .. n + nb - 1) and link them in by NSW insertion."""
    vecs = _dev(vecs, torch.float32, "vecs", 2)
    attrs = _dev(attrs, torch.uint8, "attrs", 2)
    if attrs.shape[0] != vecs.shape[0]:
        raise ValueError("vecs and attrs differ in rows")
    _check(lib().nhq_index_insert(ix.handle, vecs.data_ptr(), attrs.data_ptr(), vecs.shape[0],
                                  _stream(stream)), "nhq_index_insert")


def nhq_index_build_report(ix: Index) -> dict:
    r = ctypes.c_int32()
    _check(lib().nhq_index_build_report(ix.handle, ctypes.byref(r)), "nhq_index_build_report")
    return {"nnd_rounds_run": r.value}


def nhq_index_save(ix: Index, path: str, stream=None) -> None:
    """Write the index to a file (include/nhq.h: nhq_index_save)."""
    _check(lib().nhq_index_save(ix.handle, os.fsencode(path), _stream(stream)), "nhq_index_save")


def nhq_index_load(path: str, stream=None) -> Index:
    """A new index on the current device from a file written by
    nhq_index_save."""
    h = ctypes.c_void_p()
    _check(lib().nhq_index_load(os.fsencode(path), _stream(stream), ctypes.byref(h)), "nhq_index_load")
    return Index(h)


def nhq_index_build_graph(ix: Index, stream=None) -> None:
    _check(lib().nhq_index_build_graph(ix.handle, _stream(stream)), "nhq_index_build_graph")


def nhq_build_index(vecs: torch.Tensor, attrs: torch.Tensor, stream=None, **params) -> Index:
    vecs = _dev(vecs, torch.float32, "vecs", 2)
    attrs = _dev(attrs, torch.uint8, "attrs", 2)
    if attrs.shape[0] != vecs.shape[0]:
        raise ValueError("vecs and attrs differ in rows")
    p = _params(**params)
    h = ctypes.c_void_p()
    _check(lib().nhq_build_index(vecs.data_ptr(), attrs.data_ptr(), vecs.shape[0], vecs.shape[1],
                                 attrs.shape[1], ctypes.byref(p), _stream(stream), ctypes.byref(h)),
           "nhq_build_index")
    return Index(h, device=vecs.device, d=vecs.shape[1], m=attrs.shape[1])


def nhq_index_set_graph(ix: Index, adj: torch.Tensor, stream=None) -> None:
    adj = _dev(adj, torch.int32, "adj", 2)
    n = nhq_index_info(ix)["n"]
    if adj.shape[0] != n:
        raise ValueError("adj must have n rows")
    _check(lib().nhq_index_set_graph(ix.handle, adj.data_ptr(), adj.shape[1], _stream(stream)),
           "nhq_index_set_graph")


def nhq_index_info(ix: Index) -> dict:
    n = ctypes.c_int64()
    d, m, deg, st, ne = (ctypes.c_int32() for _ in range(5))
    _check(lib().nhq_index_info(ix.handle, ctypes.byref(n), ctypes.byref(d), ctypes.byref(m),
                                ctypes.byref(deg), ctypes.byref(st), ctypes.byref(ne)),
           "nhq_index_info")
    return {"n": n.value, "d": d.value, "m": m.value, "degree": deg.value,
            "storage": st.value, "n_entry": ne.value}


def nhq_index_get_graph(ix: Index, stream=None) -> torch.Tensor:
    info = nhq_index_info(ix)
    out = torch.empty((info["n"], info["degree"]), dtype=torch.int32, device=ix.device)
    _check(lib().nhq_index_get_graph(ix.handle, out.data_ptr(), _stream(stream)), "nhq_index_get_graph")
    return out


def nhq_index_get_entry(ix: Index, stream=None) -> torch.Tensor:
    info = nhq_index_info(ix)
    out = torch.empty((info["n_entry"],), dtype=torch.int32, device=ix.device)
    _check(lib().nhq_index_get_entry(ix.handle, out.data_ptr(), _stream(stream)), "nhq_index_get_entry")
    return out


def nhq_index_entry_blocks(ix: Index, stream=None):
    """Blocks of a stratified entry sample: (codes uint8 [B][m], offsets
    int32 [B + 1] in entry positions, member ids int32 tensor on the device),
    or None when the index has none."""
    nb = ctypes.c_int32()
    _check(lib().nhq_index_entry_blocks(ix.handle, ctypes.byref(nb), None, None, None, _stream(stream)),
           "nhq_index_entry_blocks")
    if nb.value == 0:
        return None
    m = ix.dims()[1]
    codes = np.empty((nb.value, m), dtype=np.uint8)
    offs = np.empty(nb.value + 1, dtype=np.int32)
    _check(lib().nhq_index_entry_blocks(ix.handle, ctypes.byref(nb), codes.ctypes.data, offs.ctypes.data, None,
                                        _stream(stream)), "nhq_index_entry_blocks")
    ids = torch.empty((int(offs[-1] - offs[0]),), dtype=torch.int32, device=ix.device)
    _check(lib().nhq_index_entry_blocks(ix.handle, ctypes.byref(nb), None, None, ids.data_ptr(), _stream(stream)),
           "nhq_index_entry_blocks")
    return codes, offs, ids


def nhq_index_get_storage(ix: Index, stream=None):
    """(rows [n, dp] as float32 / int16 bf16 bit patterns / uint8 e4m3 codes,
    scales float32 [n] or None)"""
    info = nhq_index_info(ix)
    st = info["storage"]
    dp = ctypes.c_int32()
    _d = _padded_dim(info["d"])
    dt = {0: torch.float32, 1: torch.int16, 2: torch.uint8}[st]
    rows = torch.empty((info["n"], _d), dtype=dt, device=ix.device)
    scales = torch.empty((info["n"],), dtype=torch.float32, device=ix.device) if st == 2 else None
    _check(lib().nhq_index_get_storage(ix.handle, rows.data_ptr(),
                                       scales.data_ptr() if scales is not None else None,
                                       ctypes.byref(dp), _stream(stream)), "nhq_index_get_storage")
    if dp.value != _d:
        raise RuntimeError("padded width mismatch")
    return rows, scales


def _padded_dim(d: int) -> int:
    for w in (32, 64, 96, 128, 256, 512, 960, 1024):
        if d <= w:
            return w
    raise ValueError("d > 1024")


def nhq_index_device_error(ix: Index, stream=None) -> int:
    bits = ctypes.c_uint32()
    _check(lib().nhq_index_device_error(ix.handle, _stream(stream), ctypes.byref(bits)),
           "nhq_index_device_error")
    return bits.value


def nhq_hybrid_search(ix: Index, queries: torch.Tensor, qattrs: torch.Tensor, k: int, beam: int,
                      n_init: int = 32, rerank: int = 0, output_mode: int = 0, max_hops: int = 0,
                      visited_log2: int = 0, learned: int = 0, stop_threshold: float = 0.0,
                      check_every: int = 0, counters: bool = False, stream=None,
                      out: Optional[Tuple[torch.Tensor, torch.Tensor]] = None,
                      cap_factor: float = 0.0, trace: Optional["TraceBuffers"] = None,
                      expand: int = 1, route_h: int = 0, order: Optional[torch.Tensor] = None):
    """Returns (ids int32 [nq,k], dists float32 [nq,k]) and, with
    counters=True, a uint32-valued int32 tensor [nq,2] of (NDC, H).
    route_h >= 2 turns on two-stage routing (Sec. 4.2); order (int32 [nq]
    permutation, see nhq_query_order) sets the launch order."""
    queries, qattrs = _query_inputs(ix, queries, qattrs)
    nq = queries.shape[0]
    ids, dists = _out_pair(ix, out, nq, int(k))
    if trace is not None and (trace.nq != nq or trace.feat.device != ix.device):
        raise ValueError("trace buffers must be for %d queries on %s" % (nq, ix.device))
    cnt = torch.zeros((nq, 2), dtype=torch.int32, device=queries.device) if counters else None
    sp = SearchParams(int(n_init), int(rerank), int(output_mode), int(max_hops), int(visited_log2),
                      int(learned), float(stop_threshold), int(check_every),
                      cnt.data_ptr() if cnt is not None else None, float(cap_factor),
                      ctypes.cast(ctypes.byref(trace.c), ctypes.c_void_p) if trace is not None else None,
                      int(expand), int(route_h), _order(ix, order, nq))
    _check(lib().nhq_hybrid_search(ix.handle, queries.data_ptr(), qattrs.data_ptr(), nq, int(k),
                                   int(beam), ctypes.byref(sp), ids.data_ptr(), dists.data_ptr(),
                                   _stream(stream)), "nhq_hybrid_search")
    return (ids, dists, cnt) if counters else (ids, dists)


NOALLOC_SCRATCH_BYTES = 64 << 20


def nhq_hybrid_search_noalloc(ix: Index, queries: torch.Tensor, qattrs: torch.Tensor, k: int, beam: int,
                              out: Tuple[torch.Tensor, torch.Tensor], n_init: int = 32,
                              counters: Optional[torch.Tensor] = None, stream=None, **kw):
    """nhq_hybrid_search through the allocation-free entry point: the caller
    passes the outputs (and, optionally, an int32 [nq][2] counters tensor);
    the library uses its fixed per-device scratch.  Other keywords as
    nhq_hybrid_search (rerank, output_mode, expand, ...)."""
    queries, qattrs = _query_inputs(ix, queries, qattrs)
    nq = queries.shape[0]
    ids, dists = _out_pair(ix, out, nq, int(k))
    if counters is not None and (counters.dtype != torch.int32 or tuple(counters.shape) != (nq, 2)
                                 or not counters.is_contiguous() or counters.device != ix.device):
        raise ValueError("counters must be a contiguous int32 [%d][2] tensor on %s" % (nq, ix.device))
    sp = SearchParams(int(n_init), int(kw.get("rerank", 0)), int(kw.get("output_mode", 0)),
                      int(kw.get("max_hops", 0)), int(kw.get("visited_log2", 0)), 0, 0.0, 0,
                      counters.data_ptr() if counters is not None else None, 0.0, None,
                      int(kw.get("expand", 1)), int(kw.get("route_h", 0)), _order(ix, kw.get("order"), nq))
    _check(lib().nhq_hybrid_search_noalloc(ix.handle, queries.data_ptr(), qattrs.data_ptr(), nq, int(k),
                                           int(beam), ctypes.byref(sp), ids.data_ptr(), dists.data_ptr(),
                                           _stream(stream)), "nhq_hybrid_search_noalloc")
    return ids, dists


def _order(ix: Index, order: Optional[torch.Tensor], nq: int):
    """The launch-order pointer for SearchParams (None: natural order)."""
    if order is None:
        return None
    if (not isinstance(order, torch.Tensor) or order.dtype != torch.int32 or tuple(order.shape) != (nq,)
            or not order.is_contiguous() or order.device != ix.device):
        raise ValueError("order must be a contiguous int32 [%d] tensor on %s" % (nq, ix.device))
    return order.data_ptr()


def nhq_query_order(ix: Index, qattrs: torch.Tensor, stream=None) -> torch.Tensor:
    """Launch order by decreasing selectivity fraction (least selective
    queries first): an int32 [nq] permutation for the searches' `order`."""
    if not isinstance(qattrs, torch.Tensor) or qattrs.dtype != torch.uint8 or qattrs.dim() != 2:
        raise ValueError("qattrs must be a uint8 [nq][m] tensor")
    _, m = ix.dims()
    if qattrs.shape[1] != m:
        raise ValueError("qattrs has %d attributes, the index %d" % (qattrs.shape[1], m))
    if qattrs.device != ix.device:
        raise ValueError("qattrs must be on the index's device %s" % ix.device)
    qattrs = qattrs.contiguous()
    nq = qattrs.shape[0]
    order = torch.empty((nq,), dtype=torch.int32, device=ix.device)
    _check(lib().nhq_query_order(ix.handle, qattrs.data_ptr(), nq, order.data_ptr(), _stream(stream)),
           "nhq_query_order")
    return order


def nhq_seed_order(ix: Index, cand: torch.Tensor, stream=None, out: Optional[torch.Tensor] = None,
                   workspace: Optional[torch.Tensor] = None) -> torch.Tensor:
    """Launch order grouping a batch by the lowest entry position among each
    query's seed candidates (cand from nhq_seed_rank), each group on one XCD;
    int32 [nq] on the index's device.  workspace: as for nhq_seed_rank (the
    same tensor serves both calls)."""
    if (not isinstance(cand, torch.Tensor) or cand.dtype != torch.int32 or cand.dim() != 2
            or cand.device != ix.device):
        raise ValueError("cand must be an int32 [nq][n_cand] tensor on %s" % ix.device)
    cand = cand.contiguous()
    nq = cand.shape[0]
    order = out if out is not None else torch.empty(nq, dtype=torch.int32, device=cand.device)
    if (order.dtype != torch.int32 or tuple(order.shape) != (nq,) or not order.is_contiguous()
            or order.device != ix.device):
        raise ValueError("out must be a contiguous int32 [%d] tensor on %s" % (nq, ix.device))
    if workspace is not None and (not isinstance(workspace, torch.Tensor) or workspace.dtype != torch.uint8
                                  or not workspace.is_contiguous() or workspace.device != ix.device):
        raise ValueError("workspace must be a contiguous uint8 tensor on %s" % ix.device)
    _check(lib().nhq_seed_order(ix.handle, cand.data_ptr(), cand.shape[1], nq, order.data_ptr(),
                                None if workspace is None else workspace.data_ptr(),
                                0 if workspace is None else workspace.numel(), _stream(stream)),
           "nhq_seed_order")
    return order


def nhq_seed_rank_workspace_size(ix: Index, nq: int, n_cand: int) -> int:
    """Bytes of device scratch nhq_seed_rank(..., workspace=) needs."""
    b = ctypes.c_size_t()
    _check(lib().nhq_seed_rank_workspace_size(ix.handle, int(nq), int(n_cand), ctypes.byref(b)),
           "nhq_seed_rank_workspace_size")
    return int(b.value)


def nhq_seed_rank(ix: Index, queries: torch.Tensor, qattrs: torch.Tensor, n_cand: int,
                  stream=None, out: Optional[torch.Tensor] = None,
                  workspace: Optional[torch.Tensor] = None) -> torch.Tensor:
    """Seed candidates [nq][n_cand]; with `workspace` (a contiguous uint8
    device tensor of at least nhq_seed_rank_workspace_size bytes, 256-byte
    aligned) the ranking's scratch is the caller's, so calls with different
    workspaces may run concurrently on different streams."""
    queries, qattrs = _query_inputs(ix, queries, qattrs)
    nq = queries.shape[0]
    if out is None:
        cand = torch.empty((nq, n_cand), dtype=torch.int32, device=queries.device)
    else:
        cand = out
        if (not isinstance(cand, torch.Tensor) or cand.dtype != torch.int32
                or tuple(cand.shape) != (nq, int(n_cand)) or not cand.is_contiguous()
                or cand.device != ix.device):
            raise ValueError("out must be a contiguous int32 [%d][%d] tensor on %s" % (nq, n_cand, ix.device))
    if workspace is None:
        _check(lib().nhq_seed_rank(ix.handle, queries.data_ptr(), qattrs.data_ptr(), nq, int(n_cand),
                                   cand.data_ptr(), _stream(stream)), "nhq_seed_rank")
        return cand
    if (not isinstance(workspace, torch.Tensor) or workspace.dtype != torch.uint8
            or not workspace.is_contiguous() or workspace.device != ix.device):
        raise ValueError("workspace must be a contiguous uint8 tensor on %s" % ix.device)
    _check(lib().nhq_seed_rank_ws(ix.handle, queries.data_ptr(), qattrs.data_ptr(), nq, int(n_cand),
                                  cand.data_ptr(), workspace.data_ptr(), workspace.numel(), _stream(stream)),
           "nhq_seed_rank_ws")
    return cand


def nhq_search_seeded(ix: Index, queries: torch.Tensor, qattrs: torch.Tensor, cand: torch.Tensor,
                      k: int, beam: int, n_init: int = 32, rerank: int = 0, output_mode: int = 0,
                      max_hops: int = 0, visited_log2: int = 0, learned: int = 0,
                      stop_threshold: float = 0.0, check_every: int = 0, counters: bool = False,
                      stream=None, out: Optional[Tuple[torch.Tensor, torch.Tensor]] = None,
                      cap_factor: float = 0.0, trace: Optional["TraceBuffers"] = None,
                      expand: int = 1, route_h: int = 0, order: Optional[torch.Tensor] = None):
    queries, qattrs = _query_inputs(ix, queries, qattrs)
    nq = queries.shape[0]
    if (not isinstance(cand, torch.Tensor) or cand.dtype != torch.int32 or cand.dim() != 2
            or cand.shape[0] != nq):
        raise ValueError("cand must be an int32 [nq][n_cand] tensor")
    if cand.device != ix.device:
        raise ValueError("cand must be on the index's device %s" % ix.device)
    cand = cand.contiguous()
    ids, dists = _out_pair(ix, out, nq, int(k))
    if trace is not None and (trace.nq != nq or trace.feat.device != ix.device):
        raise ValueError("trace buffers must be for %d queries on %s" % (nq, ix.device))
    cnt = torch.zeros((nq, 2), dtype=torch.int32, device=queries.device) if counters else None
    sp = SearchParams(int(n_init), int(rerank), int(output_mode), int(max_hops), int(visited_log2),
                      int(learned), float(stop_threshold), int(check_every),
                      cnt.data_ptr() if cnt is not None else None, float(cap_factor),
                      ctypes.cast(ctypes.byref(trace.c), ctypes.c_void_p) if trace is not None else None,
                      int(expand), int(route_h), _order(ix, order, nq))
    _check(lib().nhq_search_seeded(ix.handle, queries.data_ptr(), qattrs.data_ptr(), nq,
                                   cand.data_ptr(), cand.shape[1], int(k), int(beam), ctypes.byref(sp),
                                   ids.data_ptr(), dists.data_ptr(), _stream(stream)),
           "nhq_search_seeded")
    return (ids, dists, cnt) if counters else (ids, dists)


def nhq_bruteforce_hybrid_knn(ix: Index, queries: torch.Tensor, qattrs: torch.Tensor, k: int,
                              stream=None):
    queries, qattrs = _query_inputs(ix, queries, qattrs)
    nq = queries.shape[0]
    ids, dists = _out_pair(ix, None, nq, int(k))
    _check(lib().nhq_bruteforce_hybrid_knn(ix.handle, queries.data_ptr(), qattrs.data_ptr(), nq,
                                           int(k), ids.data_ptr(), dists.data_ptr(), _stream(stream)),
           "nhq_bruteforce_hybrid_knn")
    return ids, dists


class TraceBuffers:
    """Device buffers of nhq_trace for nq queries and up to `cap` checkpoints."""

    def __init__(self, nq: int, cap: int, device="cuda"):
        self.feat = torch.zeros((nq, cap, 8), dtype=torch.float32, device=device)
        self.hop = torch.zeros((nq, cap), dtype=torch.int32, device=device)
        self.hash = torch.zeros((nq, cap), dtype=torch.int32, device=device)
        self.count = torch.zeros((nq,), dtype=torch.int32, device=device)
        self.final_hash = torch.zeros((nq,), dtype=torch.int32, device=device)
        self.nq, self.cap = nq, cap
        self.c = Trace(self.feat.data_ptr(), self.hop.data_ptr(), self.hash.data_ptr(),
                       self.count.data_ptr(), self.final_hash.data_ptr(), cap)


def nhq_trace_samples(trace: TraceBuffers, counters: Optional[torch.Tensor] = None, stream=None):
    """(X [n,8], y_stop [n], y_beam [n]) training samples of a trace."""
    rows = trace.nq * trace.cap
    dev = trace.feat.device
    if counters is not None and (counters.dtype != torch.int32 or tuple(counters.shape) != (trace.nq, 2)
                                 or not counters.is_contiguous() or counters.device != dev):
        raise ValueError("counters must be a contiguous int32 [%d][2] tensor on %s" % (trace.nq, dev))
    X = torch.empty((max(rows, 1), 8), dtype=torch.float32, device=dev)
    ys = torch.empty((max(rows, 1),), dtype=torch.float32, device=dev)
    yb = torch.empty((max(rows, 1),), dtype=torch.float32, device=dev)
    n = ctypes.c_int64()
    _check(lib().nhq_trace_samples(ctypes.byref(trace.c), trace.nq,
                                   counters.data_ptr() if counters is not None else None,
                                   X.data_ptr(), ys.data_ptr(), yb.data_ptr(), ctypes.byref(n),
                                   _stream(stream)), "nhq_trace_samples")
    return X[: n.value], ys[: n.value], yb[: n.value]


def _samples(X: torch.Tensor, y_stop: torch.Tensor, y_beam: torch.Tensor, device):
    """Training samples X float32 [n][8], y_stop [n], y_beam [n] on `device`."""
    n = X.shape[0]
    if (X.dim() != 2 or X.shape[1] != 8 or tuple(y_stop.shape) != (n,)
            or tuple(y_beam.shape) != (n,)):
        raise ValueError("X must be [n][8] and y_stop, y_beam [n]")
    X = _dev(X, torch.float32, "X", 2)
    y_stop = _dev(y_stop, torch.float32, "y_stop", 1)
    y_beam = _dev(y_beam, torch.float32, "y_beam", 1)
    for name, t in (("X", X), ("y_stop", y_stop), ("y_beam", y_beam)):
        if t.device != device:
            raise ValueError("%s must be on %s" % (name, device))
    return X, y_stop, y_beam


def _mlp_params(t: torch.Tensor, name: str = "params") -> torch.Tensor:
    t = _dev(t, torch.float32, name, 1)
    if t.shape[0] != MLP_PARAMS:
        raise ValueError("%s must hold %d values" % (name, MLP_PARAMS))
    return t


def nhq_mlp_grad(params: torch.Tensor, X: torch.Tensor, y_stop: torch.Tensor, y_beam: torch.Tensor,
                 lam: float = 1.0, want_z: bool = False, stream=None):
    """(grad [4866], loss [1], z [n,2] or None) of the mean loss at params."""
    params = _mlp_params(params)
    X, y_stop, y_beam = _samples(X, y_stop, y_beam, params.device)
    n = X.shape[0]
    grad = torch.empty_like(params)
    loss = torch.empty((1,), dtype=torch.float32, device=params.device)
    z = torch.empty((n, 2), dtype=torch.float32, device=params.device) if want_z else None
    _check(lib().nhq_mlp_grad(params.data_ptr(), X.data_ptr(), y_stop.data_ptr(), y_beam.data_ptr(), n,
                              float(lam), grad.data_ptr(), loss.data_ptr(),
                              z.data_ptr() if z is not None else None, _stream(stream)), "nhq_mlp_grad")
    return grad, loss, z


def nhq_mlp_train(params: torch.Tensor, adam_state: torch.Tensor, step: int, X: torch.Tensor,
                  y_stop: torch.Tensor, y_beam: torch.Tensor, epochs: int, batch: int = 1024,
                  lr: float = 1e-3, lam: float = 1.0, seed: int = 0, stream=None):
    """Trains params in place; returns (new step count, loss per epoch)."""
    for name, t, size in (("params", params, MLP_PARAMS), ("adam_state", adam_state, 2 * MLP_PARAMS)):
        if not t.is_cuda or t.dtype != torch.float32 or not t.is_contiguous():
            raise TypeError("%s must be a contiguous float32 CUDA tensor" % name)
        if t.dim() != 1 or t.shape[0] != size or t.device != params.device:
            raise ValueError("%s must be [%d] on %s" % (name, size, params.device))
    X, y_stop, y_beam = _samples(X, y_stop, y_beam, params.device)
    st = ctypes.c_int64(int(step))
    losses = torch.zeros((max(epochs, 1),), dtype=torch.float32, device=params.device)
    _check(lib().nhq_mlp_train(params.data_ptr(), adam_state.data_ptr(), ctypes.byref(st), X.data_ptr(),
                               y_stop.data_ptr(), y_beam.data_ptr(), X.shape[0], int(epochs), int(batch),
                               float(lr), float(lam), int(seed), losses.data_ptr(), _stream(stream)),
           "nhq_mlp_train")
    return st.value, losses[:epochs]


def nhq_mlp_load(ix: Index, params: Optional[torch.Tensor], stream=None) -> None:
    if params is not None:
        params = _mlp_params(params)
        if params.device != ix.device:
            raise ValueError("params must be on the index's device %s" % ix.device)
    _check(lib().nhq_mlp_load(ix.handle, params.data_ptr() if params is not None else None,
                              _stream(stream)), "nhq_mlp_load")


def nhq_mlp_eval(ix: Index, X: torch.Tensor, stream=None) -> torch.Tensor:
    X = _dev(X, torch.float32, "X", 2)
    if X.shape[1] != 8 or X.device != ix.device:
        raise ValueError("X must be [n][8] on the index's device %s" % ix.device)
    Z = torch.empty((X.shape[0], 2), dtype=torch.float32, device=X.device)
    _check(lib().nhq_mlp_eval(ix.handle, X.data_ptr(), X.shape[0], Z.data_ptr(), _stream(stream)),
           "nhq_mlp_eval")
    return Z


# ------------------------------------------------------------------ serving

def _host(a, dtype, name: str):
    import numpy as np
    a = np.ascontiguousarray(a, dtype=dtype)
    return a, a.ctypes.data


class Server:
    """Owning handle of an nhq_server (host-side arrays are numpy)."""

    def __init__(self, ix: Index, **params):
        import numpy as np
        self._ix = ix
        p = ServerParams(**params)
        h = ctypes.c_void_p()
        _check(lib().nhq_server_create(ix.handle, ctypes.byref(p), ctypes.byref(h)), "nhq_server_create")
        self._h = h
        info = nhq_index_info(ix)
        self.d, self.m = info["d"], info["m"]
        slots = (ctypes.c_int32 * 2)()
        lds = (ctypes.c_int32 * 2)()
        bmax = (ctypes.c_int32 * 2)()
        hz = ctypes.c_double()
        _check(lib().nhq_server_info(h, slots, lds, bmax, ctypes.byref(hz)), "nhq_server_info")
        self.slots, self.lds_bytes, self.beam_max = list(slots), list(lds), list(bmax)
        self.tick_hz = hz.value
        self.max_k = params.get("max_k", 0) or 100
        self._np = np

    @property
    def handle(self):
        if not self._h:
            raise ValueError("server was freed")
        return self._h

    def submit(self, q, qa, k: int, beam: int, flags: int = 0) -> int:
        np = self._np
        q, qp = _host(q, np.float32, "q")
        qa, ap = _host(qa, np.uint8, "qattr")
        if q.shape != (self.d,) or qa.shape != (self.m,):
            raise ValueError("q must be [d] and qattr [m]")
        t = ctypes.c_uint64()
        rc = lib().nhq_server_submit(self.handle, qp, ap, int(k), int(beam), int(flags), ctypes.byref(t))
        if rc == -7:
            return -1
        _check(rc, "nhq_server_submit")
        return t.value

    def poll(self, ticket: int, k: int):
        """(ids, dists, counters, ticks) once finished, else None."""
        np = self._np
        ids = np.empty(k, np.int32)
        dists = np.empty(k, np.float32)
        cnt = np.empty(2, np.uint32)
        ticks = np.empty(2, np.uint64)
        rc = lib().nhq_server_poll(self.handle, ctypes.c_uint64(ticket), ids.ctypes.data, dists.ctypes.data,
                                   cnt.ctypes.data, ticks.ctypes.data)
        if rc == PENDING:
            return None
        _check(rc, "nhq_server_poll")
        return ids, dists, cnt, ticks

    def run(self, q, qa, k, beam, arrival_s, flags=None, timeout_s: float = 60.0):
        """Open-loop stream in native code; returns a dict of host arrays."""
        np = self._np
        n = len(arrival_s)
        q, qp = _host(q, np.float32, "q")
        qa, ap = _host(qa, np.uint8, "qattrs")
        k, kp = _host(k, np.int32, "k")
        beam, bp = _host(beam, np.int32, "beam")
        arr, tp = _host(arrival_s, np.float64, "arrival_s")
        fp = None
        if flags is not None:
            flags, fp = _host(flags, np.int32, "flags")
        if q.shape != (n, self.d) or qa.shape != (n, self.m) or k.shape != (n,) or beam.shape != (n,):
            raise ValueError("q [n][d], qattrs [n][m], k [n], beam [n] expected")
        ids = np.empty((n, self.max_k), np.int32)
        dists = np.empty((n, self.max_k), np.float32)
        cnt = np.empty((n, 2), np.uint32)
        ticks = np.empty((n, 2), np.uint64)
        lat = np.empty(n, np.float64)
        el = ctypes.c_double()
        _check(lib().nhq_server_run(self.handle, qp, ap, kp, bp, fp, tp, n, ids.ctypes.data, dists.ctypes.data,
                                    cnt.ctypes.data, ticks.ctypes.data, lat.ctypes.data, ctypes.byref(el),
                                    float(timeout_s)), "nhq_server_run")
        return {"ids": ids, "dists": dists, "counters": cnt, "ticks": ticks, "latency_s": lat,
                "elapsed_s": el.value}

    def free(self) -> None:
        if self._h:
            rc = lib().nhq_server_free(self._h)
            self._h = None
            _check(rc, "nhq_server_free")

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.free()

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


def nhq_server_create(ix: Index, **params) -> Server:
    return Server(ix, **params)


def nhq_gather_probe(ix: Index, waves: int, rounds: int, seed: int = 1, stream=None):
    """Random-row gather probe; returns (sink tensor, rows read)."""
    sink = torch.empty((waves, 64), dtype=torch.float32, device=ix.device)
    rows = ctypes.c_int64()
    _check(lib().nhq_gather_probe(ix.handle, int(waves), int(rounds), int(seed), sink.data_ptr(),
                                  ctypes.byref(rows), _stream(stream)), "nhq_gather_probe")
    return sink, rows.value
