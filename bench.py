"""Benchmark: hybrid QPS at Recall@10 = 0.95 on one MI355X, plain FP32 fixed
beam against BF16 storage + learned stop, and p99 latency of the serving
loop.

Default workload (the headline): 1,000,000 Gaussian-mixture vectors of
d = 960 (64 centres), 4 attributes of cardinality 2/3/5/10, 10,000 queries
with all four attributes constrained, out-degree 32, k = 10.  The composite
index is built on the GPU (not timed); the exact answers come from the GPU
brute force, checked against the CPU oracle on a sample; every Recall@10 is
computed from FP64 distances recomputed from the vectors.

One timed "step" is one full pass of the hot path over the 10,000 queries:
seed ranking of the entry sample (matrix cores), the launch order that
groups the queries by seed candidate (nhq_seed_order), and the
joint-pruning search (one wavefront per query), with the exact float32
re-score of the final candidates in the precision forms.  Three batches are kept in flight
(--in-flight): step i runs on stream i % 3 with its own candidates, outputs
and ranking scratch (nhq_seed_rank_ws), so one batch's ranking and search
use the compute units that another batch's last queries leave idle.  QPS is the
wall clock over the timed steps; the kernels' own durations (for the
roofline) come from a second pass of the same steps one after another on
one stream with HIP events around each stage.

1. FP32, fixed beam: a beam sweep; QPS at Recall@10 = 0.95 is interpolated
   (log QPS linear in recall between the bracketing beams).
2. BF16 storage + float32 re-score of the first min(4k, beam) eligible
   entries, fixed beam: the same sweep (the storage gain alone).
3. BF16 + learned stop: the stop network is trained on the GPU from traces
   of 20,000 separate training queries and runs inside the search (one
   checkpoint whose beam output sets a hop budget); the budget factor is
   swept and QPS at 0.95 interpolated the same way.
The reported ``value`` is form 3 timed over --steps steps at its first
setting that reaches Recall@10 >= 0.95; forms 1 and 2 are timed the same
way beside it.
4. Serving: the BF16 index under a Poisson stream (50,000 requests/s for
   10 s) of requests with k uniform in {1, 10, 50, 100} and 1 to 4 of the 4
   attributes constrained (the rest wildcards), the beam left to a stop
   network trained on that constraint law; p50 / p99 latency from arrival to
   result, sustained QPS, Recall@10 of the k >= 10 requests; then a
   saturation run (all requests at once) for the sustained maximum.

``--workload plain`` runs the 1M x 128 integer workload, ``ablation`` and
``build`` the parameter and builder studies.  Inputs are resident in HBM
before every timed region.  Prints ONE JSON line.  ``--gpus N`` with N > 1
exits: this build runs on one GPU.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


# seed candidates beyond n_init, as nhq_hybrid_search keeps them
SEED_MARGIN = 8
SEARCH_SOURCES = "paper_2203_13601_amd/csrc/search.hip,paper_2203_13601_amd/csrc/search_core.h"
HBM_PEAK_GBS = 8000.0


def _profiled_traffic(kernel: str, source: str, tag: str):
    """HBM bytes per launch of `kernel` from the committed rocprofv3 counter
    summary (FETCH_SIZE + WRITE_SIZE, copy-calibrated), or None when no
    summary exists or the kernel source changed since it was taken."""
    import glob
    import hashlib
    root = os.path.dirname(os.path.abspath(__file__))
    h = hashlib.sha256()
    for src in source.split(","):
        try:
            h.update(open(os.path.join(root, src), "rb").read())
        except OSError:
            return None
    h = h.hexdigest()[:16]
    for fn in sorted(glob.glob(os.path.join(root, "profiles", "%s_*%s.md" % (kernel, tag)))):
        txt = open(fn).read()
        if "source_sha256_16[%s]: %s" % (source, h) not in txt:
            continue
        for line in txt.splitlines():
            if line.startswith("traffic_bytes_per_launch[%s]:" % kernel):
                return float(line.split(":")[1])
    return None


def _copy_calibration(torch, dev):
    """Three device-to-device copies of 1 GiB, the last copies of the run: a
    counter pass divides them out of FETCH_SIZE / WRITE_SIZE to get bytes."""
    src = torch.empty(1 << 28, dtype=torch.float32, device=dev)
    dst = torch.empty_like(src)
    for _ in range(3):
        dst.copy_(src)
    torch.cuda.synchronize()
    del src, dst
    log("copy calibration: 3 copies of 1 GiB")


def _r(v, n=6):
    """floats to n significant digits (nested)"""
    if isinstance(v, float):
        return float("%.*g" % (n, v))
    if isinstance(v, dict):
        return {k: _r(x, n) for k, x in v.items()}
    if isinstance(v, list):
        return [_r(x, n) for x in v]
    return v


class Harness:
    """One workload's queries, exact answers and step / measurement
    helpers (argument marshalling and timing only)."""

    def __init__(self, w, args, dev):
        import torch
        import paper_2203_13601_amd as nhq
        self.torch, self.nhq, self.w, self.args, self.dev = torch, nhq, w, args, dev
        self.q = torch.from_numpy(w.q).to(dev)
        self.qa = torch.from_numpy(w.qattrs).to(dev)
        self.nq, self.k = w.nq, w.k
        self.n_cand = min(args.n_entry, args.n_init + SEED_MARGIN)
        self.cand = torch.empty((self.nq, self.n_cand), dtype=torch.int32, device=dev)
        self.ids = torch.empty((self.nq, self.k), dtype=torch.int32, device=dev)
        self.dists = torch.empty((self.nq, self.k), dtype=torch.float32, device=dev)
        # batches in flight (--in-flight, 3 by default): step i runs on stream
        # i % nf with its own candidates, outputs and seed-ranking scratch
        # (streams 1.. bring their own workspaces, stream 0 uses the
        # index's), so one batch's ranking and search fill the device while
        # another's last queries finish
        self.nf = max(1, getattr(args, "in_flight", 3))
        self.streams = [torch.cuda.Stream() for _ in range(self.nf)]
        self.cands = [self.cand] + [torch.empty_like(self.cand) for _ in range(self.nf - 1)]
        self.outs = [(self.ids, self.dists)] + [(torch.empty_like(self.ids), torch.empty_like(self.dists))
                                                for _ in range(self.nf - 1)]
        # launch orders (queries grouped by seed candidate, each group on one
        # XCD), one per batch in flight
        self.order = [torch.empty(self.nq, dtype=torch.int32, device=dev) for _ in range(self.nf)]
        self._ws = {}
        self.gt = None

    def _workspace(self, index, j=1):
        key = (id(index), j)
        if key not in self._ws:
            b = self.nhq.nhq_seed_rank_workspace_size(index, self.nq, self.n_cand)
            self._ws[key] = (index, self.torch.empty(b, dtype=self.torch.uint8, device=self.dev))
        return self._ws[key][1]

    def step(self, index, beam, counters=False, ev=None, j=None, **kw):
        """one batch: seed ranking, then the search; j None on the current
        stream, else on stream j of those kept in flight"""
        nhq, torch = self.nhq, self.torch
        seed_order = "order" not in kw  # else the caller's launch order
        if j is not None:
            s = self.streams[j]
            cand, out = self.cands[j], self.outs[j]
            ws = None if j == 0 else self._workspace(index, j)
            with torch.cuda.stream(s):
                nhq.nhq_seed_rank(index, self.q, self.qa, self.n_cand, out=cand, stream=s, workspace=ws)
                okw = kw
                if seed_order:
                    okw = dict(kw, order=nhq.nhq_seed_order(index, cand, stream=s, out=self.order[j],
                                                            workspace=ws))
                nhq.nhq_search_seeded(index, self.q, self.qa, cand, self.k, beam, n_init=self.args.n_init,
                                      out=out, expand=self.args.expand, stream=s, **okw)
            return None
        if ev is not None:
            ev[0].record()
        nhq.nhq_seed_rank(index, self.q, self.qa, self.n_cand, out=self.cand)
        if seed_order:
            kw = dict(kw, order=nhq.nhq_seed_order(index, self.cand, out=self.order[0]))
        if ev is not None:
            ev[1].record()
        r = nhq.nhq_search_seeded(index, self.q, self.qa, self.cand, self.k, beam, n_init=self.args.n_init,
                                  counters=counters, out=(self.ids, self.dists), expand=self.args.expand, **kw)
        if ev is not None:
            ev[2].record()
        return r

    def timed(self, index, beam, reps, **kw):
        """wall clock over `reps` steps, nf batches in flight (step i on
        stream i % nf), then the same number of steps one
        after another on one stream with HIP events around each stage, which
        give the kernels' own durations (event records are stream packets of
        their own, so they stay out of the wall-clock loop)"""
        torch = self.torch
        for j in range(1, self.nf):
            self._workspace(index, j)
        torch.cuda.synchronize()
        t = time.time()
        for i in range(reps):
            self.step(index, beam, j=i % self.nf, **kw)
        torch.cuda.synchronize()
        wall = time.time() - t
        evs = [[torch.cuda.Event(enable_timing=True) for _ in range(3)] for _ in range(reps)]
        for e in evs:
            self.step(index, beam, ev=e, **kw)
        torch.cuda.synchronize()
        return wall, [e[0].elapsed_time(e[1]) for e in evs], [e[1].elapsed_time(e[2]) for e in evs]

    def recall(self, ids):
        from paper_2203_13601_amd.metrics import recall_at_k
        w = self.w
        return recall_at_k(ids, w.x, w.q, w.attrs, w.qattrs, self.gt, self.k)

    def point(self, index, beam, **kw):
        """one setting: Recall@10 (FP64), NDC, hops, QPS over 3 steps per
        stream in flight, stage times"""
        _, _, cnt = self.step(index, beam, counters=True, **kw)
        self.torch.cuda.synchronize()
        ids = self.ids.cpu().numpy()
        rec = self.recall(ids)
        cnt = cnt.cpu().numpy().astype(np.float64)
        for j in range(self.nf):
            self.step(index, beam, j=j, **kw)
        reps = 3 * self.nf
        wall, rk, se = self.timed(index, beam, reps, **kw)
        return {"beam": beam, "recall": float(rec.mean()), "qps": self.nq * reps / wall,
                "ndc": float(cnt[:, 0].mean()), "hops": float(cnt[:, 1].mean()),
                "hops_p99": float(np.percentile(cnt[:, 1], 99)),
                "returned": float((ids >= 0).sum(axis=1).mean()),
                "rank_ms": float(np.median(rk)), "search_ms": float(np.median(se))}

    def run_form(self, index, beam, steps, warmup, **kw):
        for i in range(max(warmup, self.nf)):
            self.step(index, beam, j=i % self.nf, **kw)
        wall, rank_ms, search_ms = self.timed(index, beam, steps, **kw)
        return {"qps": self.nq * steps / wall, "ms_per_step": wall * 1000.0 / steps,
                "rank_kernels_avg_ms": float(np.mean(rank_ms)), "search_kernel_avg_ms": float(np.mean(search_ms)),
                "wall_s": wall}


def _sweep(h, index, label, beams, target, **kw):
    pts = []
    for beam in beams:
        if beam < h.k:
            continue
        p = h.point(index, beam, **kw)
        pts.append(p)
        log("%s beam %3d recall %.4f ndc %.0f hops %.1f rank %.3fms search %.3fms %.0f QPS" % (
            label, beam, p["recall"], p["ndc"], p["hops"], p["rank_ms"], p["search_ms"], p["qps"]))
        if p["recall"] >= target + 0.01 and len([x for x in pts if x["recall"] >= target]) >= 2:
            break
    return pts


def _form_errors(h, w, index, beam, storage, **kw):
    """Per returned result of the form's step: |Gamma - Gamma FP64| / Gamma FP64
    (every distance recomputed from the vectors); for bf16 / fp8 also the
    error of Gamma computed from the decoded stored row of each returned
    object (the approximation the loop orders by before the float32
    re-score), over the first 1,000 queries."""
    import paper_2203_13601_amd as nhq
    from paper_2203_13601_amd.metrics import gamma_rel_error
    h.step(index, beam, **kw)
    h.torch.cuda.synchronize()
    ids, dists = h.ids.cpu().numpy(), h.dists.cpu().numpy()
    e = gamma_rel_error(ids, dists, w.x, w.q, w.attrs, w.qattrs)
    out = {"results": int(e.size), "max": float(e.max()), "p99": float(np.percentile(e, 99)),
           "mean": float(e.mean())}
    if storage in ("bf16", "fp8"):
        ns = min(1000, h.nq)
        rows, scales = nhq.nhq_index_get_storage(index)
        sel = h.torch.from_numpy(ids[:ns].clip(min=0).astype(np.int64)).to(rows.device).reshape(-1)
        r_np = rows[sel].cpu().numpy()
        if storage == "bf16":
            dec = (r_np.view(np.uint16).astype(np.uint32) << 16).view(np.float32)
        else:
            c = r_np.astype(np.int64)
            sgn = np.where(c >> 7, -1.0, 1.0)
            ex, mn = (c >> 3) & 15, c & 7
            val = np.where(ex == 0, mn / 8.0 * 2.0 ** -6, (1.0 + mn / 8.0) * 2.0 ** (ex - 7.0))
            dec = sgn * val * scales[sel].cpu().numpy().astype(np.float64)[:, None]
        dec = dec.reshape(ns, ids.shape[1], -1)[:, :, :w.d].astype(np.float64)
        dl_dec = np.sqrt(((dec - w.q[:ns, None, :].astype(np.float64)) ** 2).sum(-1))
        from paper_2203_13601_amd.metrics import true_delta
        dl = true_delta(ids[:ns], w.x, w.q[:ns])
        ok = ids[:ns] >= 0
        es = np.abs(dl_dec - dl)[ok] / np.maximum(dl[ok], 1e-30)  # every returned object matches: Gamma = delta
        out["stored_form"] = {"results": int(es.size), "max": float(es.max()), "mean": float(es.mean())}
        del rows, scales
    return out


def _first_at(pts, target):
    ok = [p for p in pts if p["recall"] >= target]
    return ok[0] if ok else None


def _bytes_per_query(w, elem, p, rerank_rows):
    from paper_2203_13601_amd.metrics import search_bytes_per_query
    return search_bytes_per_query(d=w.d, elem_bytes=elem, R=w.degree, k=w.k, ndc=p["ndc"], hops=p["hops"],
                                  rerank_rows=rerank_rows)


def headline(args):
    import torch
    import synth
    import paper_2203_13601_amd as nhq
    from paper_2203_13601_amd.learned import train_stop_network
    from paper_2203_13601_amd.metrics import qps_at_recall

    dev = torch.device("cuda:0")
    t0 = time.time()
    w = synth.config3(n=args.n, nq=args.nq)
    tq_np, tqa_np = synth.config3_train_queries(args.train_queries)
    log("generated %s in %.1fs" % (w.name, time.time() - t0))
    x = torch.from_numpy(w.x).to(dev)
    a = torch.from_numpy(w.attrs).to(dev)
    tq, tqa = torch.from_numpy(tq_np).to(dev), torch.from_numpy(tqa_np).to(dev)
    h = Harness(w, args, dev)
    torch.cuda.synchronize()

    t0 = time.time()
    ix = nhq.nhq_build_index(x, a, degree=w.degree, cand=w.cand, storage="fp32", n_entry=args.n_entry,
                             seed=w.build_seed, builder=args.builder)
    torch.cuda.synchronize()
    build_s = time.time() - t0
    log("built the composite index (%s candidates) in %.2fs" % (args.builder, build_s))
    t0 = time.time()
    gi, _ = nhq.nhq_bruteforce_hybrid_knn(ix, h.q, h.qa, w.k)
    h.gt = gi.cpu().numpy()
    gt_s = time.time() - t0
    adj = nhq.nhq_index_get_graph(ix)
    ixb = nhq.nhq_index_create(x, a, storage="bf16", n_entry=args.n_entry, seed=w.build_seed, degree=w.degree)
    nhq.nhq_index_set_graph(ixb, adj)
    target, k, rr = args.target, w.k, args.rerank
    beams = [10, 12, 14, 16, 18, 20, 24, 28, 32, 40, 48, 64, 96, 128]

    # ---- 1 and 2: fixed-beam sweeps (fp32; bf16 and fp8 e4m3 + float32 re-score)
    s32 = _sweep(h, ix, "fp32", beams, target)
    s16 = _sweep(h, ixb, "bf16", beams, target, rerank=rr)
    ix8 = nhq.nhq_index_create(x, a, storage="fp8", n_entry=args.n_entry, seed=w.build_seed, degree=w.degree)
    nhq.nhq_index_set_graph(ix8, adj)
    s8 = _sweep(h, ix8, "fp8", beams, target, rerank=rr)
    # ---- 3: bf16 + learned stop, per training beam a sweep of the budget factor
    ce = args.check_every
    learned_runs = []
    for l_train in args.learned_beams:
        t0 = time.time()
        params, info = train_stop_network(ixb, tq, tqa, k, l_train, epochs=30, check_every=ce,
                                          n_init=args.n_init, expand=args.expand, seed=1)
        nhq.nhq_mlp_load(ixb, params)
        torch.cuda.synchronize()
        train_s = time.time() - t0
        log("stop network at beam %d: %d trace samples, trained in %.2fs (loss %.4f)" % (
            l_train, info["samples"], train_s, info["losses"][-1]))
        pts = []
        for cf in (0.75, 1.0, 1.25, 1.5, 1.75, 2.0, 2.5, 3.0):
            kw = dict(rerank=rr, learned=2, stop_threshold=0.9, check_every=ce, cap_factor=cf)
            p = h.point(ixb, l_train, **kw)
            p.update({"cap_factor": cf, "kw": kw})
            pts.append(p)
            log("bf16+learned beam %d cap %.2f recall %.4f hops %.1f (p99 %.0f) search %.3fms %.0f QPS" % (
                l_train, cf, p["recall"], p["hops"], p["hops_p99"], p["search_ms"], p["qps"]))
            if p["recall"] >= target + 0.01 and len([x for x in pts if x["recall"] >= target]) >= 2:
                break
        at = qps_at_recall([p["cap_factor"] for p in pts], [p["recall"] for p in pts],
                           [p["qps"] for p in pts], target)
        learned_runs.append({"beam": l_train, "params": params, "sweep": pts, "qps_at_target_interp": at,
                             "train_samples": info["samples"], "train_s": train_s,
                             "positive_rate": info["positive_rate"]})
    best = max((r for r in learned_runs if _first_at(r["sweep"], target) is not None),
               key=lambda r: r["qps_at_target_interp"] or 0.0, default=None)
    # ---- 3b: bf16 + the beam-width predictor (learned mode 3) at one beam
    pool_run = None
    if args.pool_beam:
        from paper_2203_13601_amd.learned import train_pool_network
        t0 = time.time()
        pparams, pinfo = train_pool_network(ixb, tq, tqa, k, args.pool_beam, epochs=60, check_every=ce,
                                            n_init=args.n_init, expand=args.expand, seed=3, rerank=rr)
        nhq.nhq_mlp_load(ixb, pparams)
        torch.cuda.synchronize()
        ptrain_s = time.time() - t0
        log("pool-size network at beam %d: %d samples in %.2fs (median target %.0f)" % (
            args.pool_beam, pinfo["samples"], ptrain_s, pinfo["pool_label_median"]))
        pts = []
        for cf in (1.0, 1.25, 1.5, 2.0, 2.5, 3.0, 4.0):
            kw = dict(rerank=rr, learned=3, check_every=ce, cap_factor=cf)
            p = h.point(ixb, args.pool_beam, **kw)
            p.update({"cap_factor": cf, "kw": kw})
            pts.append(p)
            log("bf16+pool predictor beam %d factor %.2f recall %.4f hops %.1f ndc %.0f search %.3fms %.0f QPS" % (
                args.pool_beam, cf, p["recall"], p["hops"], p["ndc"], p["search_ms"], p["qps"]))
            if p["recall"] >= target + 0.01 and len([x for x in pts if x["recall"] >= target]) >= 2:
                break
        pool_run = {"beam": args.pool_beam, "params": pparams, "sweep": pts, "train_s": ptrain_s,
                    "train_samples": pinfo["samples"], "median_pool_target": pinfo["pool_label_median"],
                    "qps_at_target_interp": qps_at_recall([p["cap_factor"] for p in pts],
                                                          [p["recall"] for p in pts], [p["qps"] for p in pts],
                                                          target)}

    # ---- timed steps at each form's first setting reaching the target
    forms = {}
    for name, index, pts, elem in (("fp32_fixed", ix, s32, 4), ("bf16_fixed", ixb, s16, 2),
                                   ("fp8_fixed", ix8, s8, 1)):
        op = _first_at(pts, target) or pts[-1]
        kw = {"rerank": rr} if name != "fp32_fixed" else {}
        run = h.run_form(index, op["beam"], args.steps, args.warmup, **kw)
        run["gamma_rel_err_vs_fp64"] = _form_errors(h, w, index, op["beam"], name.split("_")[0], **kw)
        at = qps_at_recall([p["beam"] for p in pts], [p["recall"] for p in pts], [p["qps"] for p in pts], target)
        forms[name] = {**run, "beam": op["beam"], "recall": op["recall"], "ndc": op["ndc"], "hops": op["hops"],
                       "returned": op["returned"], "qps_at_target_interp": at, "rerank": kw.get("rerank", 0),
                       "bytes_per_query": _bytes_per_query(w, elem, op, op["returned"] if elem != 4 else 0.0),
                       "sweep": [{kk: vv for kk, vv in p.items()} for p in pts]}
        log("%s: beam %d recall %.4f: %.3f ms/step, %.0f QPS (interpolated at %.2f: %s)" % (
            name, op["beam"], op["recall"], run["ms_per_step"], run["qps"], target, at))
    ix8.free()
    value_form = "bf16_fixed"
    if best is not None:
        nhq.nhq_mlp_load(ixb, best["params"])
        op = _first_at(best["sweep"], target)
        run = h.run_form(ixb, best["beam"], args.steps, args.warmup, **op["kw"])
        run["gamma_rel_err_vs_fp64"] = _form_errors(h, w, ixb, best["beam"], "bf16", **op["kw"])
        forms["bf16_learned"] = {
            **run, "beam": best["beam"], "recall": op["recall"], "ndc": op["ndc"], "hops": op["hops"],
            "returned": op["returned"], "hops_p99": op["hops_p99"], "learned_mode": 2, "check_every": ce, "cap_factor": op["cap_factor"],
            "rerank": rr, "qps_at_target_interp": best["qps_at_target_interp"],
            "train_samples": best["train_samples"], "train_s": best["train_s"],
            "bytes_per_query": _bytes_per_query(w, 2, op, op["returned"]),
            "per_training_beam": [{"beam": r["beam"], "qps_at_target_interp": r["qps_at_target_interp"],
                                   "positive_rate": r["positive_rate"],
                                   "sweep": [{kk: vv for kk, vv in p.items() if kk != "kw"} for p in r["sweep"]]}
                                  for r in learned_runs]}
        value_form = "bf16_learned"
        log("bf16+learned: beam %d cap %.2f recall %.4f: %.3f ms/step, %.0f QPS" % (
            best["beam"], op["cap_factor"], op["recall"], run["ms_per_step"], run["qps"]))
    if pool_run is not None and _first_at(pool_run["sweep"], target) is not None:
        nhq.nhq_mlp_load(ixb, pool_run["params"])
        pop = _first_at(pool_run["sweep"], target)
        prun = h.run_form(ixb, pool_run["beam"], args.steps, args.warmup, **pop["kw"])
        forms["bf16_pool_predictor"] = {
            **prun, "beam": pool_run["beam"], "recall": pop["recall"], "ndc": pop["ndc"], "hops": pop["hops"],
            "returned": pop["returned"], "learned_mode": 3, "check_every": ce, "pool_factor": pop["cap_factor"],
            "rerank": rr, "qps_at_target_interp": pool_run["qps_at_target_interp"],
            "train_samples": pool_run["train_samples"], "train_s": pool_run["train_s"],
            "median_pool_target": pool_run["median_pool_target"],
            "bytes_per_query": _bytes_per_query(w, 2, pop, pop["returned"]),
            "sweep": [{kk: vv for kk, vv in p.items() if kk != "kw"} for p in pool_run["sweep"]]}
        log("bf16_pool_predictor: beam %d factor %.2f recall %.4f: %.3f ms/step, %.0f QPS" % (
            pool_run["beam"], pop["cap_factor"], pop["recall"], prun["ms_per_step"], prun["qps"]))
        if best is not None:
            nhq.nhq_mlp_load(ixb, best["params"])
    vf = forms[value_form]
    for name in ("bf16_fixed", "fp8_fixed", "bf16_learned", "bf16_pool_predictor"):
        if name in forms:
            f = forms[name]
            f["speedup_vs_fp32_fixed"] = f["qps"] / forms["fp32_fixed"]["qps"]
            if f["qps_at_target_interp"] and forms["fp32_fixed"]["qps_at_target_interp"]:
                f["interp_speedup_vs_fp32_fixed"] = (f["qps_at_target_interp"]
                                                     / forms["fp32_fixed"]["qps_at_target_interp"])
    if "bf16_learned" in forms and forms["bf16_fixed"]["qps_at_target_interp"]:
        fl = forms["bf16_learned"]
        fl["interp_speedup_vs_bf16_fixed"] = (fl["qps_at_target_interp"] or 0.0) / forms["bf16_fixed"][
            "qps_at_target_interp"]

    # ---- roofline of the dominant kernel: the search of the reported form
    search_s = vf["search_kernel_avg_ms"] / 1000.0
    bq = vf["bytes_per_query"]
    achieved = bq * h.nq / search_s / 1e9
    kernel = "k_search_ck" if value_form == "bf16_learned" else "k_search"
    traffic = None
    if args.n == 1_000_000 and args.nq == 10_000:
        # the summary of the same launch: form and beam in its name
        traffic = _profiled_traffic(kernel, SEARCH_SOURCES, "_n1M_d960_bf16_%s_beam%d" % (
            "learned" if value_form == "bf16_learned" else "fixed", vf["beam"]))
    step_bytes = bq * h.nq + h.nq * (4.0 * w.d + 8.0 * h.n_cand)  # + the seed stage's query reads and candidates
    roof = {"bound": "hbm", "achieved": round(achieved, 2), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 5), "traffic": traffic,
            "traffic_ratio_vs_algorithmic": None if traffic is None else round(traffic / (bq * h.nq), 4),
            "kernel": kernel, "form": value_form, "bytes_per_query": round(bq, 1), "queries_per_launch": h.nq,
            "bytes_formula": "4d + H*4R + NDC*(4 + d*s_v) + rerank_rows*4d + 8k; s_v = 2 (bf16), "
                             "rerank_rows = results returned per query (a lower bound on the rows re-scored)",
            "kernel_avg_ms": round(vf["search_kernel_avg_ms"], 4),
            "rank_kernels_avg_ms": round(vf["rank_kernels_avg_ms"], 4),
            "whole_step_frac": round(step_bytes / (vf["ms_per_step"] / 1000.0) / 1e9 / HBM_PEAK_GBS, 5)}
    from paper_2203_13601_amd.metrics import search_extra_bytes_per_query
    roof["extra_bytes_per_query"] = {k2: round(v2, 1) for k2, v2 in search_extra_bytes_per_query(
        d_pad=960, elem_bytes=2, n_cand=h.n_cand, out_rows=k, rerank=True).items()}
    roof["extra_bytes_per_query"]["rerank_rows_beyond_returned_max"] = round(
        (min(rr * k, vf["beam"]) - vf.get("returned", k)) * 4.0 * w.d, 1)
    waves, rounds = 65536, 20
    nhq.nhq_gather_probe(ixb, waves, rounds)
    pe = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
    torch.cuda.synchronize()
    pe[0].record()
    for _ in range(3):
        _, rows = nhq.nhq_gather_probe(ixb, waves, rounds)
    pe[1].record()
    torch.cuda.synchronize()
    gather_gbs = rows * w.d * 2 / (pe[0].elapsed_time(pe[1]) / 3 / 1000.0) / 1e9
    roof["gather_ceiling"] = round(gather_gbs, 1)
    roof["frac_of_gather_ceiling"] = round(achieved / gather_gbs, 4)
    log("roofline: %s %.0f GB/s = %.1f%% of 8 TB/s (random %d-byte row gathers: %.0f GB/s)" % (
        kernel, achieved, 100 * achieved / HBM_PEAK_GBS, w.d * 2, gather_gbs))
    if args.copy_calibration:
        _copy_calibration(torch, dev)

    # ---- the seed set of Alg. 2 drawn at random (Sec. 3.2: n_init random
    # vertices, no ranking) against the ranked entry sample, fp32, same graph
    seed_policy = None
    if not args.no_seed_study:
        ixr = nhq.nhq_index_create(x, a, n_entry=args.n_init, seed=w.build_seed, degree=w.degree)
        nhq.nhq_index_set_graph(ixr, adj)
        hr = Harness(w, argparse.Namespace(**{**vars(args), "n_entry": args.n_init}), dev)
        hr.gt = h.gt
        rs = _sweep(hr, ixr, "fp32 random seeds", beams, target)
        seed_policy = {"random_seeds": {"n_init": args.n_init, "sweep": rs,
                                        "qps_at_target_interp": qps_at_recall(
                                            [p["beam"] for p in rs], [p["recall"] for p in rs],
                                            [p["qps"] for p in rs], target)},
                       "ranked_entry_sample": {"n_entry": args.n_entry,
                                               "qps_at_target_interp": forms["fp32_fixed"]["qps_at_target_interp"]}}
        ixr.free()
    # ---- 5. where selectivity varies: the serving stream's constraint law
    # (1 to 4 of the 4 attributes constrained) on the same query vectors; the
    # fixed beam against the learned budget at one large beam
    mixed, mixed_net, pool_net = None, None, None
    if not args.no_mixed:
        mixed, mixed_net, pool_net = mixed_selectivity(args, w, ix, ixb, tq)
    serving = None
    if not args.no_serve:
        fixed_beam = None
        if mixed is not None:
            # the fixed beams that bracket the target on the mixed batch
            sw = mixed["fixed_sweep"]
            ok = [i for i, p in enumerate(sw) if p["recall"] >= target]
            if ok:
                fixed_beam = [sw[ok[0] - 1]["beam"], sw[ok[0]]["beam"]] if ok[0] > 0 else [sw[ok[0]]["beam"]]
        serving = serve_config5(args, w, ixb, ix, h, tq, x.device, mixed_net, fixed_beam, pool_net)
    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline(args, w, ix, h, forms["fp32_fixed"]["beam"], rerank_n=0)

    out = {
        "metric": "hybrid QPS at Recall@10=0.95 on 1 GPU, plain FP32 vs BF16+learned-stop; p99 ms",
        "value": round(vf["qps"], 1),
        "unit": "queries/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(vf["ms_per_step"], 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "bf16",
        "data": "synthetic",
        "config": {"workload": w.name, "form": {"bf16_learned": "BF16 + learned stop + FP32 re-score",
                                                "bf16_fixed": "BF16 fixed beam + FP32 re-score"}[value_form],
                   "n": w.n, "d": w.d, "m": w.m, "cards": list(w.cards), "constrained": "all 4",
                   "queries_per_step": h.nq, "k": k, "beam": vf["beam"], "recall_at_setting": round(vf["recall"], 5),
                   "degree": w.degree, "cand": w.cand, "builder": args.builder, "n_entry": args.n_entry,
                   "n_init": args.n_init, "expand": args.expand, "build_s": round(build_s, 3),
                   "exact_knn_s": round(gt_s, 3), "recall": "FP64 distances recomputed from the vectors",
                   "batches_in_flight": args.in_flight, "parallelism": "single GPU"},
        "p99_ms": None if serving is None else serving["p99_ms"],
        "forms": _r({kk: {k2: v2 for k2, v2 in f.items()} for kk, f in forms.items()}),
        "mixed_selectivity": mixed,
        "seed_policy": _r(seed_policy),
        "serving": serving,
        "roofline": roof,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


def mixed_selectivity(args, w, ix, ixb, tq):
    """The learned stop where queries differ in difficulty: 10,000 queries
    with 1 to 4 of the 4 attributes constrained (|P|/|S| from 1/2 to 1/300)
    on the BF16 index.  A fixed-beam sweep against the stop network's hop
    budget at the serving beam (network trained on training queries of the
    same constraint law), each QPS at Recall@10 = 0.95 interpolated; the
    mean hops at equal recall."""
    import dataclasses
    import torch
    import synth
    import paper_2203_13601_amd as nhq
    from paper_2203_13601_amd.learned import train_pool_network, train_stop_network
    from paper_2203_13601_amd.metrics import qps_at_recall
    dev = torch.device("cuda:0")
    wm = dataclasses.replace(w, qattrs=synth.partial_constraints(w.nq, w.cards, 508))
    hm = Harness(wm, args, dev)
    gi, _ = nhq.nhq_bruteforce_hybrid_knn(ix, hm.q, hm.qa, w.k)
    hm.gt = gi.cpu().numpy()
    target, rr, ce, big = args.target, 4, args.check_every, args.serve_beam
    fixed = _sweep(hm, ixb, "mixed bf16", [16, 32, 48, 64, 96, 128, 160, 192, 256, 320, 384, 512], target, rerank=rr)
    tqa_p = torch.from_numpy(synth.partial_constraints(tq.shape[0], w.cards, 505)).to(dev)
    t0 = time.time()
    params, info = train_stop_network(ixb, tq, tqa_p, w.k, big, epochs=30, check_every=ce, n_init=args.n_init,
                                      expand=args.expand, seed=2)
    nhq.nhq_mlp_load(ixb, params)
    torch.cuda.synchronize()
    train_s = time.time() - t0
    log("mixed: stop network at beam %d: %d samples in %.2fs" % (big, info["samples"], train_s))
    learned = []
    for cf in (0.5, 0.75, 1.0, 1.25, 1.5, 2.0, 2.5, 3.0, 4.0):
        p = hm.point(ixb, big, rerank=rr, learned=2, stop_threshold=0.9, check_every=ce, cap_factor=cf)
        p["cap_factor"] = cf
        learned.append(p)
        log("mixed bf16+learned beam %d cap %.2f recall %.4f hops %.1f (p99 %.0f) %.0f QPS" % (
            big, cf, p["recall"], p["hops"], p["hops_p99"], p["qps"]))
        if p["recall"] >= target + 0.01 and len([x for x in learned if x["recall"] >= target]) >= 2:
            break
    fa = qps_at_recall([p["beam"] for p in fixed], [p["recall"] for p in fixed], [p["qps"] for p in fixed], target)
    la = qps_at_recall([p["cap_factor"] for p in learned], [p["recall"] for p in learned],
                       [p["qps"] for p in learned], target)
    # the same forms launched least selective first (nhq_query_order): the
    # queries that need the most hops start first, so the batch's tail shrinks
    order = nhq.nhq_query_order(ixb, hm.qa)
    fixed_o = _sweep(hm, ixb, "mixed bf16 ordered", [16, 32, 48, 64, 96, 128, 160, 192, 256, 320, 384, 512], target,
                     rerank=rr, order=order)
    learned_o = []
    for cf in (0.5, 0.75, 1.0, 1.25, 1.5, 2.0, 2.5, 3.0, 4.0):
        p = hm.point(ixb, big, rerank=rr, learned=2, stop_threshold=0.9, check_every=ce, cap_factor=cf, order=order)
        p["cap_factor"] = cf
        learned_o.append(p)
        log("mixed bf16+learned ordered beam %d cap %.2f recall %.4f hops %.1f %.0f QPS" % (
            big, cf, p["recall"], p["hops"], p["qps"]))
        if p["recall"] >= target + 0.01 and len([x for x in learned_o if x["recall"] >= target]) >= 2:
            break
    fao = qps_at_recall([p["beam"] for p in fixed_o], [p["recall"] for p in fixed_o], [p["qps"] for p in fixed_o],
                        target)
    lao = qps_at_recall([p["cap_factor"] for p in learned_o], [p["recall"] for p in learned_o],
                        [p["qps"] for p in learned_o], target)
    # the beam-width predictor (learned mode 3): the network trained on pool
    # size targets chooses each query's pool size at its first checkpoint
    t0 = time.time()
    pool_params, pinfo = train_pool_network(ixb, tq, tqa_p, w.k, big, epochs=60, check_every=ce,
                                            n_init=args.n_init, expand=args.expand, seed=3, rerank=rr)
    pool_s = time.time() - t0
    log("mixed: pool-size network at beam %d: %d samples in %.2fs (median target %.0f)" % (
        big, pinfo["samples"], pool_s, pinfo["pool_label_median"]))
    nhq.nhq_mlp_load(ixb, pool_params)
    pooled = []
    for cf in (0.75, 1.0, 1.25, 1.5, 2.0, 2.5, 3.0, 4.0, 6.0):
        p = hm.point(ixb, big, rerank=rr, learned=3, check_every=ce, cap_factor=cf)
        p["cap_factor"] = cf
        pooled.append(p)
        log("mixed bf16+pool predictor beam %d factor %.2f recall %.4f hops %.1f (p99 %.0f) ndc %.0f %.0f QPS" % (
            big, cf, p["recall"], p["hops"], p["hops_p99"], p["ndc"], p["qps"]))
        if p["recall"] >= target + 0.01 and len([x for x in pooled if x["recall"] >= target]) >= 2:
            break
    pa = qps_at_recall([p["cap_factor"] for p in pooled], [p["recall"] for p in pooled],
                       [p["qps"] for p in pooled], target)
    pooled_o = []
    for cf in (0.75, 1.0, 1.25, 1.5, 2.0, 2.5, 3.0, 4.0, 6.0):
        p = hm.point(ixb, big, rerank=rr, learned=3, check_every=ce, cap_factor=cf, order=order)
        p["cap_factor"] = cf
        pooled_o.append(p)
        log("mixed bf16+pool predictor ordered beam %d factor %.2f recall %.4f hops %.1f %.0f QPS" % (
            big, cf, p["recall"], p["hops"], p["qps"]))
        if p["recall"] >= target + 0.01 and len([x for x in pooled_o if x["recall"] >= target]) >= 2:
            break
    pao = qps_at_recall([p["cap_factor"] for p in pooled_o], [p["recall"] for p in pooled_o],
                        [p["qps"] for p in pooled_o], target)
    nhq.nhq_mlp_load(ixb, params)

    def hops_at(pts, key):
        prev = None
        for p in pts:
            if p["recall"] >= target:
                if prev is None or prev["recall"] >= p["recall"]:
                    return p["hops"]
                t = (target - prev["recall"]) / (p["recall"] - prev["recall"])
                return prev["hops"] + t * (p["hops"] - prev["hops"])
            prev = p
        return None
    out = {"workload": "%s queries, 1..4 of 4 attributes constrained" % w.name, "queries": w.nq,
           "fixed_qps_at_target_interp": fa, "learned_qps_at_target_interp": la,
           "learned_speedup_vs_fixed": None if not (fa and la) else la / fa,
           "fixed_hops_at_target": hops_at(fixed, "beam"), "learned_hops_at_target": hops_at(learned, "cap_factor"),
           "learned_beam": big, "learned_mode": 2, "train_samples": info["samples"], "train_s": train_s,
           "pool_predictor": {"learned_mode": 3, "qps_at_target_interp": pa,
                              "speedup_vs_fixed": None if not (fa and pa) else pa / fa,
                              "hops_at_target": hops_at(pooled, "cap_factor"), "train_samples": pinfo["samples"],
                              "train_s": pool_s, "median_pool_target": pinfo["pool_label_median"],
                              "sweep": pooled},
           "launched_least_selective_first": {
               "order": "nhq_query_order: sum of ln(count / n) over the constrained codes, largest first",
               "fixed_qps_at_target_interp": fao, "learned_qps_at_target_interp": lao,
               "pool_predictor_qps_at_target_interp": pao,
               "learned_speedup_vs_fixed": None if not (fao and lao) else lao / fao,
               "pool_predictor_speedup_vs_fixed": None if not (fao and pao) else pao / fao,
               "fixed_sweep": fixed_o, "learned_sweep": learned_o, "pool_predictor_sweep": pooled_o},
           "fixed_sweep": fixed, "learned_sweep": learned}
    log("mixed selectivity, least selective first: fixed %s QPS, learned stop %s QPS, pool predictor %s QPS" % (
        fao, lao, pao))
    log("mixed selectivity: fixed %s QPS, learned stop %s QPS, pool predictor %s QPS at Recall@10 %.2f "
        "(hops %s / %s / %s)" % (fa, la, pa, target, out["fixed_hops_at_target"], out["learned_hops_at_target"],
                                 out["pool_predictor"]["hops_at_target"]))
    return _r(out), params, pool_params


def serve_config5(args, w, ixb, ix32, h, tq, dev, params=None, fixed_beam=None, pool_params=None):
    """The serving form: Poisson stream through the continuous-batching
    server on the BF16 index (float32 re-score), then a saturation run."""
    import torch
    import synth
    import paper_2203_13601_amd as nhq
    from paper_2203_13601_amd.learned import train_stop_network
    from paper_2203_13601_amd.metrics import recall_at_k
    ns = args.serve_requests
    t0 = time.time()
    s_q, s_qa, s_k, s_arr = synth.config5_stream(ns, rate_per_s=args.serve_rate)
    log("serving stream of %d requests generated in %.1fs" % (ns, time.time() - t0))
    s_beam = np.zeros(ns, dtype=np.int32)  # the stop network chooses (automatic beam)
    # the serving network: traces of training queries with the stream's
    # constraint law (1..4 of 4 attributes constrained) at the automatic beam
    beam_auto, ce = args.serve_beam, args.check_every
    if params is None:
        tqa_p = torch.from_numpy(synth.partial_constraints(tq.shape[0], w.cards, 505)).to(dev)
        params, info = train_stop_network(ixb, tq, tqa_p, w.k, beam_auto, epochs=30, check_every=ce,
                                          n_init=args.n_init, expand=args.expand, seed=2)
    nhq.nhq_mlp_load(ixb, params)
    # exact answers of a sample of the stream (k >= 10 requests), for recall
    rng = np.random.default_rng(506)
    big = np.nonzero(s_k >= 10)[0]
    samp = np.sort(rng.choice(big, size=min(args.serve_recall_sample, big.size), replace=False))
    sq_d = torch.from_numpy(np.ascontiguousarray(s_q[samp])).to(dev)
    sqa_d = torch.from_numpy(np.ascontiguousarray(s_qa[samp])).to(dev)
    gsi, _ = nhq.nhq_bruteforce_hybrid_knn(ix32, sq_d, sqa_d, w.k)
    gsi = gsi.cpu().numpy()
    # budget factor: the smallest reaching the target on the sample (batch search)
    s_cf = None
    for cf in (0.75, 1.0, 1.25, 1.5, 2.0, 2.5, 3.0, 4.0, 6.0):
        vi, _ = nhq.nhq_hybrid_search(ixb, sq_d, sqa_d, w.k, beam_auto, n_init=args.n_init, expand=args.expand,
                                      rerank=4, learned=2, stop_threshold=0.9, check_every=ce, cap_factor=cf)
        vr = recall_at_k(vi.cpu().numpy(), w.x, s_q[samp], w.attrs, s_qa[samp], gsi, w.k).mean()
        log("serving network: cap %.1f recall %.4f on the sample" % (cf, vr))
        s_cf = cf
        if vr >= args.target + 0.005:
            break
    del sq_d, sqa_d
    torch.cuda.synchronize()
    sp = dict(n_init=args.n_init, expand=args.expand, rerank=4, auto_beam=beam_auto, beam_small=beam_auto,
              beam_large=-1, max_k=100, ring=16384, learned_mode=2, cap_factor=s_cf, stop_threshold=0.9,
              check_every=ce, lifetime_s=180.0)
    sat_n = min(ns, args.serve_saturation_requests)
    rf = rfs = None
    with nhq.Server(ixb, **sp) as srv:
        r = srv.run(s_q, s_qa, s_k, s_beam, s_arr, timeout_s=120.0)
        slots, hz = srv.slots, srv.tick_hz
        # saturation: the same requests offered all at once
        rs = srv.run(s_q[:sat_n], s_qa[:sat_n], s_k[:sat_n], s_beam[:sat_n], np.zeros(sat_n), timeout_s=120.0)
        if fixed_beam is not None:
            # the method without the network: every request at a fixed beam,
            # the two beams that bracket the target on the mixed batch (the
            # stream at the larger, saturation at both)
            fb = np.full(ns, fixed_beam[-1], dtype=np.int32)
            rf = srv.run(s_q, s_qa, s_k, fb, s_arr, timeout_s=120.0)
            rfs = [(b, srv.run(s_q[:sat_n], s_qa[:sat_n], s_k[:sat_n], np.full(sat_n, b, np.int32),
                               np.zeros(sat_n), timeout_s=120.0)) for b in fixed_beam]
    lat_ms = r["latency_s"] * 1000.0
    svc_ms = (r["ticks"][:, 1].astype(np.float64) - r["ticks"][:, 0]) / hz * 1000.0
    rec = recall_at_k(r["ids"][samp, :10], w.x, s_q[samp], w.attrs, s_qa[samp], gsi, w.k)
    out = {"offered_qps": args.serve_rate, "requests": ns, "duration_s": round(float(s_arr[-1]), 2),
           "sustained_qps": round(ns / r["elapsed_s"], 1),
           "p50_ms": round(float(np.percentile(lat_ms, 50)), 4),
           "p99_ms": round(float(np.percentile(lat_ms, 99)), 4),
           "max_ms": round(float(lat_ms.max()), 4),
           "device_service_p50_ms": round(float(np.percentile(svc_ms, 50)), 4),
           "device_service_p99_ms": round(float(np.percentile(svc_ms, 99)), 4),
           "recall_at_10_k_ge_10": round(float(rec.mean()), 5), "recall_sample": int(samp.size),
           "hops_mean": round(float(r["counters"][:, 1].mean()), 2),
           "saturation": {"requests": int(sat_n), "sustained_qps": round(sat_n / rs["elapsed_s"], 1),
                          "p50_ms": round(float(np.percentile(rs["latency_s"] * 1000.0, 50)), 4),
                          "p99_ms": round(float(np.percentile(rs["latency_s"] * 1000.0, 99)), 4)},
           "same_in_saturation_as_in_stream": bool(
               np.array_equal(rs["ids"], r["ids"][:sat_n]) and
               np.array_equal(rs["dists"].view(np.uint32), r["dists"][:sat_n].view(np.uint32))),
           "k_mix": [1, 10, 50, 100], "constrained_attrs": "1..4 of 4",
           "beam": "learned hop budget at the automatic beam %d (cap factor %.2f)" % (beam_auto, s_cf),
           "storage": "bf16 + float32 re-score of min(4k, beam) eligible entries", "slots": slots[0],
           "latency": "arrival to result seen by the host"}
    log("serving: %d requests at %.0f/s: p50 %.3f ms, p99 %.3f ms, recall@10 %.4f; saturation %.0f QPS" % (
        ns, args.serve_rate, out["p50_ms"], out["p99_ms"], out["recall_at_10_k_ge_10"],
        out["saturation"]["sustained_qps"]))
    if rf is not None:
        from paper_2203_13601_amd.metrics import qps_at_recall
        sat = samp[samp < sat_n]
        gsat = gsi[samp < sat_n]

        def srec(ids):
            return float(recall_at_k(ids[sat, :10], w.x, s_q[sat], w.attrs, s_qa[sat], gsat, w.k).mean())
        lf = rf["latency_s"] * 1000.0
        sat_pts = [{"beam": int(b), "saturation_qps": round(sat_n / x["elapsed_s"], 1),
                    "recall_at_10_k_ge_10": round(srec(x["ids"]), 5),
                    "hops_mean": round(float(x["counters"][:, 1].mean()), 2)} for b, x in rfs]
        lrec = srec(rs["ids"])
        out["saturation"]["recall_at_10_k_ge_10"] = round(lrec, 5)
        out["saturation"]["hops_mean"] = round(float(rs["counters"][:, 1].mean()), 2)
        at = qps_at_recall([p["beam"] for p in sat_pts], [p["recall_at_10_k_ge_10"] for p in sat_pts],
                           [p["saturation_qps"] for p in sat_pts], lrec)
        out["fixed_beam_form"] = {
            "beam": int(fixed_beam[-1]), "p50_ms": round(float(np.percentile(lf, 50)), 4),
            "p99_ms": round(float(np.percentile(lf, 99)), 4),
            "recall_at_10_k_ge_10": round(float(recall_at_k(rf["ids"][samp, :10], w.x, s_q[samp], w.attrs,
                                                            s_qa[samp], gsi, w.k).mean()), 5),
            "hops_mean": round(float(rf["counters"][:, 1].mean()), 2),
            "saturation": sat_pts,
            "saturation_qps_at_learned_recall_interp": None if at is None else round(at, 1)}
        if at:
            out["learned_saturation_speedup_vs_fixed_at_equal_recall"] = round(
                out["saturation"]["sustained_qps"] / at, 4)
        log("serving, fixed beam %d: p50 %.3f ms, p99 %.3f ms, recall@10 %.4f; saturation %s; at the learned "
            "form's recall %.4f: %s QPS" % (fixed_beam[-1], out["fixed_beam_form"]["p50_ms"],
                                           out["fixed_beam_form"]["p99_ms"],
                                           out["fixed_beam_form"]["recall_at_10_k_ge_10"], sat_pts, lrec, at))
    if pool_params is not None:
        # the beam-width predictor (learned mode 3): the same stream and
        # saturation run with each request's pool size chosen by the network
        nhq.nhq_mlp_load(ixb, pool_params)
        sq_d = torch.from_numpy(np.ascontiguousarray(s_q[samp])).to(dev)
        sqa_d = torch.from_numpy(np.ascontiguousarray(s_qa[samp])).to(dev)
        p_cf = None
        for cf in (0.75, 1.0, 1.25, 1.5, 2.0, 2.5, 3.0, 4.0, 6.0, 8.0):
            vi, _ = nhq.nhq_hybrid_search(ixb, sq_d, sqa_d, w.k, beam_auto, n_init=args.n_init,
                                          expand=args.expand, rerank=4, learned=3, check_every=ce, cap_factor=cf)
            vr = recall_at_k(vi.cpu().numpy(), w.x, s_q[samp], w.attrs, s_qa[samp], gsi, w.k).mean()
            log("serving pool-size network: factor %.2f recall %.4f on the sample" % (cf, vr))
            p_cf = cf
            if vr >= args.target + 0.005:
                break
        del sq_d, sqa_d
        torch.cuda.synchronize()
        with nhq.Server(ixb, **{**sp, "learned_mode": 3, "cap_factor": p_cf}) as srv:
            rp = srv.run(s_q, s_qa, s_k, s_beam, s_arr, timeout_s=120.0)
            rps = srv.run(s_q[:sat_n], s_qa[:sat_n], s_k[:sat_n], s_beam[:sat_n], np.zeros(sat_n),
                          timeout_s=120.0)
        lp = rp["latency_s"] * 1000.0
        sat = samp[samp < sat_n]
        out["pool_predictor_form"] = {
            "learned_mode": 3, "pool_factor": p_cf,
            "p50_ms": round(float(np.percentile(lp, 50)), 4), "p99_ms": round(float(np.percentile(lp, 99)), 4),
            "recall_at_10_k_ge_10": round(float(recall_at_k(rp["ids"][samp, :10], w.x, s_q[samp], w.attrs,
                                                            s_qa[samp], gsi, w.k).mean()), 5),
            "hops_mean": round(float(rp["counters"][:, 1].mean()), 2),
            "saturation_qps": round(sat_n / rps["elapsed_s"], 1),
            "saturation_recall_at_10_k_ge_10": round(float(recall_at_k(
                rps["ids"][sat, :10], w.x, s_q[sat], w.attrs, s_qa[sat], gsi[samp < sat_n], w.k).mean()), 5)}
        pf = out["pool_predictor_form"]
        log("serving, pool-size predictor (factor %.2f): p50 %.3f ms, p99 %.3f ms, recall@10 %.4f, hops %.1f; "
            "saturation %.0f QPS at recall %.4f" % (p_cf, pf["p50_ms"], pf["p99_ms"], pf["recall_at_10_k_ge_10"],
                                                    pf["hops_mean"], pf["saturation_qps"],
                                                    pf["saturation_recall_at_10_k_ge_10"]))
        nhq.nhq_mlp_load(ixb, params)
    return out


def cpu_baseline(args, w, ix, h, beam, rerank_n=0):
    """The CPU oracle on the GPU machine's host cores, on a bounded sample of the
    same workload: the reference search (same graph, entry sample, seeds and
    beam) and the brute-force exact answer (Def. 4).  Also the parity of the
    GPU's outputs on that sample: search ids against the oracle's search,
    the GPU's exact answers against the oracle's, the benchmark's recall
    against the oracle's own scoring."""
    import oracle
    import paper_2203_13601_amd as nhq
    from paper_2203_13601_amd.metrics import gamma_rel_error
    threads = os.cpu_count() or 1
    adj = nhq.nhq_index_get_graph(ix).cpu().numpy()
    entry = oracle.entry_points(w.build_seed, w.n, args.n_entry)
    kw = dict(n_init=args.n_init, key_mode=oracle.KEY32 if w.integer else oracle.KEY64, threads=threads,
              expand=args.expand)
    nsamp = 64
    t = time.time()
    oracle.search(adj, w.x, w.attrs, w.q[:nsamp], w.qattrs[:nsamp], w.k, beam, entry, **kw)
    el = time.time() - t
    if el < args.cpu_seconds:
        nsamp = int(min(w.nq, max(nsamp, nsamp * args.cpu_seconds / max(el, 1e-3))))
        t = time.time()
        o = oracle.search(adj, w.x, w.attrs, w.q[:nsamp], w.qattrs[:nsamp], w.k, beam, entry, **kw)
        el = time.time() - t
    else:
        o = oracle.search(adj, w.x, w.attrs, w.q[:nsamp], w.qattrs[:nsamp], w.k, beam, entry, **kw)
    n1 = min(w.nq, max(16, int(nsamp / threads)))
    t = time.time()
    oracle.search(adj, w.x, w.attrs, w.q[:n1], w.qattrs[:n1], w.k, beam, entry, **dict(kw, threads=1))
    el1 = time.time() - t
    # the GPU's search on the same queries
    gi_s, gd_s = nhq.nhq_search_seeded(ix, h.q[:nsamp], h.qa[:nsamp], nhq.nhq_seed_rank(
        ix, h.q[:nsamp], h.qa[:nsamp], h.n_cand), w.k, beam, n_init=args.n_init, expand=args.expand)
    gi_s, gd_s = gi_s.cpu().numpy(), gd_s.cpu().numpy()
    same = (gi_s == o[0]).all(axis=1)
    overlap = np.mean([len(set(a_[a_ >= 0]) & set(b_[b_ >= 0])) / max(1, (a_ >= 0).sum(), (b_ >= 0).sum())
                       if (a_ >= 0).any() or (b_ >= 0).any() else 1.0 for a_, b_ in zip(gi_s, o[0])])
    # brute force (C4) on the CPU: its rate, and the GPU's exact answers against it
    nb = max(4, min(nsamp, args.cpu_bf_queries))
    t = time.time()
    bi, bd, _ = oracle.bruteforce(w.x, w.attrs, w.q[:nb], w.qattrs[:nb], w.k, threads=threads)
    elb = time.time() - t
    gt_same = float((h.gt[:nb] == bi).all(axis=1).mean())
    # recall of the GPU search: the benchmark's metric against the oracle's scoring (exact answers: oracle's)
    from paper_2203_13601_amd.metrics import recall_at_k
    rb = recall_at_k(gi_s[:nb], w.x, w.q[:nb], w.attrs, w.qattrs[:nb], bi, w.k)
    ro = oracle.recall(gi_s[:nb], w.x, w.attrs, w.q[:nb], w.qattrs[:nb], bi, bd, w.k)
    err = gamma_rel_error(gi_s, gd_s, w.x, w.q[:nsamp], w.attrs, w.qattrs[:nsamp])
    out = {"value": round(nsamp / el, 1), "unit": "queries/s", "cores": threads, "kind": "oracle",
           "single_thread_value": round(n1 / el1, 1),
           "bruteforce_value": round(nb / elb, 3), "bruteforce_unit": "queries/s (C4, exact filter + FP64 top-k)",
           "sample": "%d of %d queries, beam %d, expand %d, same graph, entry sample and seeds, FP64 C oracle "
                     "(entry-sample scan + joint pruning), %d threads; brute force on the first %d" % (
                         nsamp, w.nq, beam, args.expand, threads, nb),
           "parity": {"search_ids_identical_queries": round(float(same.mean()), 5),
                      "search_result_overlap": round(float(overlap), 5),
                      "gpu_exact_answers_equal_oracle": gt_same,
                      "recall_metric_equals_oracle_recall": bool(np.allclose(rb, ro)),
                      "returned_gamma_max_rel_err_vs_fp64": float(err.max()) if err.size else 0.0}}
    log("cpu oracle: %.1f QPS on %d threads (1 thread %.1f); brute force %.2f QPS; parity %s" % (
        out["value"], threads, out["single_thread_value"], out["bruteforce_value"], out["parity"]))
    return out


def plain(args):
    """The 1M x 128 integer workload (values in [0, 255], 256 clusters, 3
    attributes of cardinality 3/4/5, full constraints): FP32 and BF16 (lossless
    here) fixed-beam sweeps, each form timed at its first beam reaching the
    target; the CPU oracle beside it."""
    import torch
    import synth
    import paper_2203_13601_amd as nhq
    from paper_2203_13601_amd.metrics import qps_at_recall
    dev = torch.device("cuda:0")
    w = synth.config2(n=args.n, nq=args.nq)
    x = torch.from_numpy(w.x).to(dev)
    a = torch.from_numpy(w.attrs).to(dev)
    h = Harness(w, args, dev)
    t0 = time.time()
    ix = nhq.nhq_build_index(x, a, degree=w.degree, cand=w.cand, n_entry=args.n_entry, seed=w.build_seed,
                             builder=args.builder)
    torch.cuda.synchronize()
    build_s = time.time() - t0
    gi, _ = nhq.nhq_bruteforce_hybrid_knn(ix, h.q, h.qa, w.k)
    h.gt = gi.cpu().numpy()
    ixb = nhq.nhq_index_create(x, a, storage="bf16", n_entry=args.n_entry, seed=w.build_seed, degree=w.degree)
    nhq.nhq_index_set_graph(ixb, nhq.nhq_index_get_graph(ix))
    beams = [args.beam] if args.beam else [10, 16, 20, 24, 28, 32, 36, 40, 48, 56, 64, 96, 128]
    forms = {}
    for name, index, elem in (("fp32_fixed", ix, 4), ("bf16_fixed", ixb, 2)):
        pts = _sweep(h, index, name, beams, args.target)
        op = _first_at(pts, args.target) or pts[-1]
        run = h.run_form(index, op["beam"], args.steps, args.warmup)
        forms[name] = {**run, "beam": op["beam"], "recall": op["recall"], "ndc": op["ndc"], "hops": op["hops"],
                       "qps_at_target_interp": qps_at_recall([p["beam"] for p in pts], [p["recall"] for p in pts],
                                                             [p["qps"] for p in pts], args.target),
                       "bytes_per_query": _bytes_per_query(w, elem, op, 0.0), "sweep": pts}
    vf = forms["fp32_fixed"]
    bq = vf["bytes_per_query"]
    achieved = bq * h.nq / (vf["search_kernel_avg_ms"] / 1000.0) / 1e9
    traffic = None
    if args.n == 1_000_000 and args.nq == 10_000:
        traffic = _profiled_traffic("k_search", SEARCH_SOURCES, "_beam%d" % vf["beam"])
    roof = {"bound": "hbm", "achieved": round(achieved, 2), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 5), "traffic": traffic, "kernel": "k_search",
            "bytes_per_query": round(bq, 1), "queries_per_launch": h.nq,
            "kernel_avg_ms": round(vf["search_kernel_avg_ms"], 4)}
    if args.copy_calibration:
        _copy_calibration(torch, dev)
    cpu = None if args.no_cpu_baseline else cpu_baseline(args, w, ix, h, vf["beam"])
    print(json.dumps({"metric": "hybrid QPS at Recall@10=0.95 on 1 GPU, 1M x 128 integer workload",
                      "value": round(vf["qps"], 1), "unit": "queries/s", "n_gpus": 1, "steps": args.steps,
                      "warmup": args.warmup, "ms_per_step": round(vf["ms_per_step"], 4), "higher_is_better": True,
                      "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
                      "config": {"workload": w.name, "n": w.n, "d": w.d, "queries_per_step": h.nq, "k": w.k,
                                 "beam": vf["beam"], "n_entry": args.n_entry, "n_init": args.n_init,
                                 "expand": args.expand, "build_s": round(build_s, 3), "batches_in_flight": args.in_flight,
                                 "parallelism": "single GPU"},
                      "forms": _r(forms), "roofline": roof, "cpu_baseline": cpu}), flush=True)


def learned10m(args):
    """The learned-stop form at full size: 10,000,000 Gaussian-mixture
    vectors of d = 96 (1,024 centres), 3 attributes of cardinality 3/4/5
    with Zipf(1.1) codes, fully constrained queries whose code tuples follow
    the data (|P|/|S| from 1/681 to 1/7.5).  The composite index (NN-descent
    candidate lists) with a stratified entry sample (--entry-per-pattern per
    attribute pattern).  The stop network is trained on the GPU from traces
    of 200,000 training queries and evaluated on 10,000 held-out queries:
    the fixed-beam sweep against the learned hop budget, QPS at
    Recall@10 = 0.95 interpolated for each, and the hops at equal recall."""
    import torch
    import synth
    import paper_2203_13601_amd as nhq
    from paper_2203_13601_amd.learned import train_stop_network
    from paper_2203_13601_amd.metrics import qps_at_recall
    dev = torch.device("cuda:0")
    t0 = time.time()
    w = synth.config4(n=args.n, nq=args.nq)
    tq_np, tqa_np = synth.config4_train_queries(args.train_queries)
    log("generated %s in %.1fs" % (w.name, time.time() - t0))
    x = torch.from_numpy(w.x).to(dev)
    a = torch.from_numpy(w.attrs).to(dev)
    tq, tqa = torch.from_numpy(tq_np).to(dev), torch.from_numpy(tqa_np).to(dev)
    h = Harness(w, args, dev)
    t0 = time.time()
    ix = nhq.nhq_build_index(x, a, degree=w.degree, cand=w.cand, n_entry=args.n_entry, seed=w.build_seed,
                             builder="nndescent", entry_per_pattern=args.entry_per_pattern)
    torch.cuda.synchronize()
    build_s = time.time() - t0
    log("built (NN-descent, %d rounds, stratified entry sample %d per pattern) in %.1fs" % (
        nhq.nhq_index_build_report(ix)["nnd_rounds_run"], args.entry_per_pattern, build_s))
    gi, _ = nhq.nhq_bruteforce_hybrid_knn(ix, h.q, h.qa, w.k)
    h.gt = gi.cpu().numpy()
    target, ce = args.target, args.check_every
    fixed = _sweep(h, ix, "fixed", [10, 12, 16, 20, 24, 32, 40, 48, 64, 96, 128], target)
    runs = []
    for l_train in args.learned_beams:
        t0 = time.time()
        params, info = train_stop_network(ix, tq, tqa, w.k, l_train, epochs=args.epochs, check_every=ce,
                                          n_init=args.n_init, expand=args.expand, seed=1)
        nhq.nhq_mlp_load(ix, params)
        torch.cuda.synchronize()
        train_s = time.time() - t0
        log("stop network at beam %d: %d samples from %d training queries, trained in %.1fs (loss %.4f)" % (
            l_train, info["samples"], tq.shape[0], train_s, info["losses"][-1]))
        pts = []
        for cf in (0.5, 0.75, 1.0, 1.25, 1.5, 2.0, 2.5, 3.0):
            p = h.point(ix, l_train, learned=2, stop_threshold=0.9, check_every=ce, cap_factor=cf)
            p["cap_factor"] = cf
            pts.append(p)
            log("learned beam %d cap %.2f recall %.4f hops %.1f (p99 %.0f) %.0f QPS" % (
                l_train, cf, p["recall"], p["hops"], p["hops_p99"], p["qps"]))
            if p["recall"] >= target + 0.01 and len([q for q in pts if q["recall"] >= target]) >= 2:
                break
        runs.append({"beam": l_train, "train_samples": info["samples"], "train_s": train_s,
                     "positive_rate": info["positive_rate"], "sweep": pts,
                     "qps_at_target_interp": qps_at_recall([p["cap_factor"] for p in pts],
                                                           [p["recall"] for p in pts], [p["qps"] for p in pts],
                                                           target),
                     "hops_at_target": _interp_at(pts, target, "hops")})
    fa = qps_at_recall([p["beam"] for p in fixed], [p["recall"] for p in fixed], [p["qps"] for p in fixed], target)
    best = max(runs, key=lambda r: r["qps_at_target_interp"] or 0.0)
    # the beam-width predictor (learned mode 3) at the largest training beam
    pool = None
    if args.pool_beam:
        from paper_2203_13601_amd.learned import train_pool_network
        pb = max(args.learned_beams)
        t0 = time.time()
        pparams, pinfo = train_pool_network(ix, tq, tqa, w.k, pb, epochs=max(args.epochs, 30), check_every=ce,
                                            n_init=args.n_init, expand=args.expand, seed=3)
        nhq.nhq_mlp_load(ix, pparams)
        torch.cuda.synchronize()
        ptrain_s = time.time() - t0
        log("pool-size network at beam %d: %d samples in %.1fs (median target %.0f)" % (
            pb, pinfo["samples"], ptrain_s, pinfo["pool_label_median"]))
        pts = []
        for cf in (0.75, 1.0, 1.25, 1.5, 2.0, 2.5, 3.0, 4.0):
            p = h.point(ix, pb, learned=3, check_every=ce, cap_factor=cf)
            p["cap_factor"] = cf
            pts.append(p)
            log("pool predictor beam %d factor %.2f recall %.4f hops %.1f ndc %.0f %.0f QPS" % (
                pb, cf, p["recall"], p["hops"], p["ndc"], p["qps"]))
            if p["recall"] >= target + 0.01 and len([q for q in pts if q["recall"] >= target]) >= 2:
                break
        pool = {"learned_mode": 3, "beam": pb, "train_samples": pinfo["samples"], "train_s": ptrain_s,
                "median_pool_target": pinfo["pool_label_median"], "sweep": pts,
                "qps_at_target_interp": qps_at_recall([p["cap_factor"] for p in pts], [p["recall"] for p in pts],
                                                      [p["qps"] for p in pts], target),
                "hops_at_target": _interp_at(pts, target, "hops"), "ndc_at_target": _interp_at(pts, target, "ndc")}
    # the forms again, launched least selective first (nhq_query_order)
    order = nhq.nhq_query_order(ix, h.qa)
    fixed_o = _sweep(h, ix, "fixed ordered", [10, 12, 16, 20, 24, 32, 40, 48, 64, 96, 128], target, order=order)
    ordered = {"fixed_qps_at_target_interp": qps_at_recall([p["beam"] for p in fixed_o], [p["recall"] for p in fixed_o],
                                                           [p["qps"] for p in fixed_o], target),
               "fixed_sweep": fixed_o}
    bl = best["beam"]
    nhq.nhq_mlp_load(ix, train_stop_network(ix, tq, tqa, w.k, bl, epochs=args.epochs, check_every=ce,
                                            n_init=args.n_init, expand=args.expand, seed=1)[0])
    pts = []
    for cf in (0.5, 0.75, 1.0, 1.25, 1.5, 2.0, 2.5, 3.0):
        p = h.point(ix, bl, learned=2, stop_threshold=0.9, check_every=ce, cap_factor=cf, order=order)
        p["cap_factor"] = cf
        pts.append(p)
        log("learned ordered beam %d cap %.2f recall %.4f hops %.1f %.0f QPS" % (bl, cf, p["recall"], p["hops"],
                                                                                 p["qps"]))
        if p["recall"] >= target + 0.01 and len([q for q in pts if q["recall"] >= target]) >= 2:
            break
    ordered["learned_qps_at_target_interp"] = qps_at_recall([p["cap_factor"] for p in pts],
                                                             [p["recall"] for p in pts], [p["qps"] for p in pts], target)
    ordered["learned_sweep"] = pts
    log("10M, least selective first: fixed %s QPS, learned stop %s QPS at Recall@10 %.2f" % (
        ordered["fixed_qps_at_target_interp"], ordered["learned_qps_at_target_interp"], target))
    out = {"metric": "hybrid QPS at Recall@10=0.95 on 1 GPU, learned stop vs fixed beam (10M x 96, Zipf)",
           "value": None if best["qps_at_target_interp"] is None else round(best["qps_at_target_interp"], 1),
           "unit": "queries/s", "n_gpus": 1, "higher_is_better": True, "vs_baseline": None, "dtype": "f32",
           "data": "synthetic",
           "config": {"workload": w.name, "n": w.n, "d": w.d, "cards": list(w.cards), "queries": w.nq,
                      "train_queries": int(tq.shape[0]), "k": w.k, "n_entry": args.n_entry,
                      "entry_per_pattern": args.entry_per_pattern, "n_init": args.n_init, "expand": args.expand,
                      "builder": "nndescent", "build_s": round(build_s, 2), "storage": "fp32",
                      "batches_in_flight": args.in_flight},
           "fixed_qps_at_target_interp": fa, "fixed_hops_at_target": _interp_at(fixed, target, "hops"),
           "learned_qps_at_target_interp": best["qps_at_target_interp"],
           "learned_hops_at_target": best["hops_at_target"],
           "learned_speedup_vs_fixed": None if not (fa and best["qps_at_target_interp"]) else
           best["qps_at_target_interp"] / fa,
           "fixed_ndc_at_target": _interp_at(fixed, target, "ndc"), "pool_predictor": pool,
           "launched_least_selective_first": ordered,
           "fixed_sweep": fixed, "learned": runs}
    print(json.dumps(_r(out)), flush=True)


def _interp_at(pts, target, key):
    """`key` interpolated linearly in recall at the target (None if never reached)"""
    prev = None
    for p in pts:
        if p["recall"] >= target:
            if prev is None or prev["recall"] >= p["recall"]:
                return p[key]
            t = (target - prev["recall"]) / (p["recall"] - prev["recall"])
            return prev[key] + t * (p[key] - prev[key])
        prev = p
    return None


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="headline",
                    choices=["headline", "plain", "learned10m", "ablation", "build", "exactbuild"],
                    help="headline: 1M x 960 FP32 / BF16 / BF16 + learned stop and serving (default); "
                         "plain: 1M x 128 integer workload; learned10m: 10M x 96 Zipf, learned stop vs fixed "
                         "beam; ablation: weight settings, selectivity and "
                         "post-filtering sweeps; build: exact vs NN-descent vs NSW candidate lists; "
                         "exactbuild: the exact 1M x 960 build and ground truth alone")
    ap.add_argument("--n", type=int, default=1_000_000)
    ap.add_argument("--nq", type=int, default=10_000)
    ap.add_argument("--target", type=float, default=0.95)
    ap.add_argument("--beam", type=int, default=0, help="plain workload: fixed beam (skip the sweep)")
    ap.add_argument("--n-entry", type=int, default=None,
                    help="entry sample size (default 1024 for the headline's 64 clusters, 4096 otherwise)")
    ap.add_argument("--n-init", type=int, default=4)
    ap.add_argument("--expand", type=int, default=None, help="vertices expanded per step (headline 2, else 6)")
    ap.add_argument("--builder", default="exact", choices=["exact", "nndescent"])
    ap.add_argument("--check-every", type=int, default=1)
    ap.add_argument("--rerank", type=int, default=4,
                    help="headline reduced forms: re-score the first min(rerank * k, beam) eligible entries in FP32")
    ap.add_argument("--learned-beams", type=int, nargs="+", default=[18, 20, 24, 32])
    ap.add_argument("--pool-beam", type=int, default=32,
                    help="headline: beam of the beam-width predictor form (learned mode 3; 0 = skip)")
    ap.add_argument("--train-queries", type=int, default=None,
                    help="training queries of the stop network (20,000; 200,000 for learned10m)")
    ap.add_argument("--epochs", type=int, default=30)
    ap.add_argument("--entry-per-pattern", type=int, default=8192)
    ap.add_argument("--in-flight", type=int, default=3,
                    help="batches kept in flight on their own streams in the timed loops (4 streams "
                         "with the default one exceed the 4 hardware queues)")
    ap.add_argument("--no-serve", action="store_true")
    ap.add_argument("--serve-rate", type=float, default=50_000.0)
    ap.add_argument("--serve-requests", type=int, default=500_000)
    ap.add_argument("--serve-saturation-requests", type=int, default=200_000)
    ap.add_argument("--serve-recall-sample", type=int, default=10_000)
    ap.add_argument("--serve-beam", type=int, default=256)
    ap.add_argument("--no-mixed", action="store_true")
    ap.add_argument("--no-seed-study", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--cpu-bf-queries", type=int, default=32)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run a plain device copy of known size (counter scaling)")
    args = ap.parse_args()
    if args.n_entry is None:
        args.n_entry = 1024 if args.workload in ("headline", "exactbuild") else 4096
    if args.train_queries is None:
        args.train_queries = 200_000 if args.workload == "learned10m" else 20_000
    if args.workload == "learned10m" and args.n == 1_000_000:
        args.n = 10_000_000
    if args.expand is None:
        args.expand = 2 if args.workload == "headline" else 6
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py: this build measures one GPU only (--gpus 1); multi-GPU runs are not "
              "part of it", file=sys.stderr)
        sys.exit(2)
    {"headline": headline, "plain": plain, "learned10m": learned10m, "ablation": ablation,
     "build": build_study, "exactbuild": exact_build}[args.workload](args)

def exact_build(args):
    """The exact composite-index build of the 1M x 960 precision-form set
    (all-pairs candidate lists on the float32 matrix cores under the fusion
    distance, Alg. 1 / Sec. 4.1 and Sec. 5.1, then edge selection) and the
    exact hybrid ground truth of its 10,000 queries (Def. 4): wall times, and
    the rate of the dense products against the fp32 matrix-core peak (the
    kernel's own duration comes from the profiler)."""
    import hashlib
    import torch
    import synth
    import paper_2203_13601_amd as nhq

    dev = torch.device("cuda:0")
    t0 = time.time()
    w = synth.config3(n=args.n, nq=args.nq)
    log("generated %s in %.1fs" % (w.name, time.time() - t0))
    x = torch.from_numpy(w.x).to(dev)
    a = torch.from_numpy(w.attrs).to(dev)
    q = torch.from_numpy(w.q).to(dev)
    qa = torch.from_numpy(w.qattrs).to(dev)
    torch.cuda.synchronize()
    t0 = time.time()
    ix = nhq.nhq_build_index(x, a, degree=w.degree, cand=w.cand, storage="fp32", n_entry=args.n_entry,
                             seed=w.build_seed, builder="exact")
    torch.cuda.synchronize()
    build_s = time.time() - t0
    log("exact build of %s in %.2fs" % (w.name, build_s))
    t0 = time.time()
    gi, _ = nhq.nhq_bruteforce_hybrid_knn(ix, q, qa, w.k)
    torch.cuda.synchronize()
    gt_s = time.time() - t0
    log("exact ground truth of %d queries in %.3fs" % (w.nq, gt_s))
    if args.copy_calibration:
        _copy_calibration(torch, dev)
    dp = min(p for p in (32, 64, 96, 128, 256, 512, 960, 1024) if p >= w.d)  # the padded row width
    adj = nhq.nhq_index_get_graph(ix).cpu().numpy()
    flop_b = 2.0 * w.n * w.n * dp
    flop_g = 2.0 * w.nq * w.n * dp
    print(json.dumps({"metric": "exact composite-index build time on 1 GPU", "value": round(build_s, 3),
                      "unit": "s", "n_gpus": 1, "higher_is_better": False, "vs_baseline": None,
                      "dtype": "f32", "data": "synthetic",
                      "config": {"workload": w.name, "n": w.n, "d": w.d, "dp": dp, "cand": w.cand,
                                 "degree": w.degree, "queries": w.nq},
                      "build_s": round(build_s, 3),
                      "build_tflops_whole": round(flop_b / build_s / 1e12, 2),
                      "ground_truth_s": round(gt_s, 4),
                      "ground_truth_tflops_whole": round(flop_g / gt_s / 1e12, 2),
                      "peak_tflops_fp32_mfma": 157.3,
                      "graph_sha256_16": hashlib.sha256(adj.tobytes()).hexdigest()[:16],
                      "ground_truth_sha256_16": hashlib.sha256(gi.cpu().numpy().tobytes()).hexdigest()[:16]}),
          flush=True)
    ix.free()


def build_study(args):
    """Composite-index builds (Alg. 1 / Sec. 4.3): the exact all-pairs
    candidate lists against NN-descent (NPG_kgraph's refinement) and
    insertion in batches of 10,000 (NPG_nsw, insertion beam 96) on the
    config-2 set (1M x 128), then NN-descent alone on the config-4 set at its
    full size (10M x 96, Zipf attributes), where all pairs would take
    minutes.  For each graph: build time, rounds, and the Recall@10 / QPS of
    the search over the beam (E = --expand)."""
    import torch
    import synth
    import paper_2203_13601_amd as nhq
    from paper_2203_13601_amd.metrics import qps_at_recall, recall_at_k

    dev = torch.device("cuda:0")
    n_cand = min(args.n_entry, args.n_init + SEED_MARGIN)
    out = {}

    def curve(ix, w, q, qa, gi, gd, beams):
        rows = []
        for beam in beams:
            def step():
                cand = nhq.nhq_seed_rank(ix, q, qa, n_cand)
                return nhq.nhq_search_seeded(ix, q, qa, cand, w.k, beam, n_init=args.n_init,
                                             expand=args.expand)
            ids, d = step()
            rec = float(recall_at_k(ids.cpu().numpy(), w.x, w.q, w.attrs, w.qattrs, gi, w.k).mean())
            torch.cuda.synchronize()
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record()
            for _ in range(3):
                step()
            e1.record()
            torch.cuda.synchronize()
            ms = e0.elapsed_time(e1) / 3
            rows.append({"beam": beam, "recall": round(rec, 5), "qps": round(w.nq / (ms / 1000.0), 1)})
            log("  beam %d recall %.4f %.0f QPS" % (beam, rec, rows[-1]["qps"]))
        at = qps_at_recall([r["beam"] for r in rows], [r["recall"] for r in rows],
                           [r["qps"] for r in rows], args.target)
        return rows, None if at is None else round(at, 1)

    for name, make, builders, beams in (
            ("config2", lambda: synth.config2(n=args.n, nq=args.nq),
             (("exact", args.n_entry), ("nndescent", args.n_entry), ("nsw", args.n_entry)),
             [16, 28, 48, 96]),
            ("config4", lambda: synth.config4(nq=args.nq),
             (("nndescent", args.n_entry), ("nndescent", 16384)), [32, 64, 128, 256])):
        t = time.time()
        w = make()
        log("generated %s in %.1fs" % (w.name, time.time() - t))
        x = torch.from_numpy(w.x).to(dev)
        a = torch.from_numpy(w.attrs).to(dev)
        q = torch.from_numpy(w.q).to(dev)
        qa = torch.from_numpy(w.qattrs).to(dev)
        gi = gd = None
        res = {}
        for b, ne in builders:
            torch.cuda.synchronize()
            t = time.time()
            ix = nhq.nhq_build_index(x, a, degree=w.degree, cand=w.cand, n_entry=ne,
                                     seed=w.build_seed, builder=b, nsw_batch=10000, nsw_beam=96)
            torch.cuda.synchronize()
            bs = time.time() - t
            rounds = nhq.nhq_index_build_report(ix)["nnd_rounds_run"]
            log("%s %s build %.2fs (%d NN-descent rounds), entry sample %d" % (name, b, bs, rounds, ne))
            if gi is None:
                gi, gd = nhq.nhq_bruteforce_hybrid_knn(ix, q, qa, w.k)
                gi, gd = gi.cpu().numpy(), gd.cpu().numpy()
            rows, at = curve(ix, w, q, qa, gi, gd, beams)
            res["%s_entry%d" % (b, ne)] = {"build_s": round(bs, 2), "nnd_rounds": rounds,
                                           "curve": rows, "qps_at_target": at}
            ix.free()
        out[name] = {"workload": w.name, "n": w.n, "d": w.d, **res}
        del x, a, q, qa, w
        torch.cuda.empty_cache()
    print(json.dumps({"metric": "composite-index build: exact vs NN-descent lists, on 1 GPU",
                      "value": out["config4"]["nndescent_entry%d" % args.n_entry]["build_s"],
                      "unit": "s",
                      "n_gpus": 1, "higher_is_better": False, "vs_baseline": None, "dtype": "f32",
                      "data": "synthetic",
                      "config": {"workload": "config2 1M x 128 and config4 10M x 96",
                                 "expand": args.expand, "n_init": args.n_init,
                                 "n_entry": args.n_entry},
                      **out}), flush=True)


def ablation(args):
    """Parameter studies of the paper's Sec. 6.5 on the config-2 shape (1M x
    128 integer clusters, 10,000 queries, k = 10), each a Recall@10 / QPS
    curve over the beam (one step = seed ranking + search, E = --expand):
      weights      the five weight settings of Gamma (Fig. 10 (i), curves
                   i-v; Eq. 8 with c = 100), each with its own index;
      selectivity  attribute cardinalities giving |P|/|S| = 1/8 ... 1/4000
                   (full constraints, default weights);
      attribute dimension  m = 6 and 9 binary attributes (|P|/|S| = 1/64
                   and 1/512) against the m = 3 set;
      post_filter  strategy B(1) on the default composite index: a search
                   by vector alone (every attribute a wildcard) whose raw
                   pool is then filtered to exact matches; the filter runs on
                   the host and is not timed, so its QPS is an upper bound.
    Recall is computed from the true vector distance of each returned
    object, since Gamma differs from delta under the other settings."""
    import torch
    import synth
    import paper_2203_13601_amd as nhq
    from paper_2203_13601_amd.metrics import qps_at_recall, recall_at_k

    dev = torch.device("cuda:0")
    w = synth.config2(n=args.n, nq=args.nq)
    log("generated %s" % w.name)
    x = torch.from_numpy(w.x).to(dev)
    q = torch.from_numpy(w.q).to(dev)
    nq, k = w.nq, w.k
    n_cand = min(args.n_entry, args.n_init + SEED_MARGIN)
    beams = [10, 16, 32, 64, 128, 256, 512]

    def curve(ix, attrs_np, qattrs_np, gi, gd, label, raw_filter=False):
        qa_dev = torch.from_numpy(qattrs_np).to(dev)
        qa_search = torch.full_like(qa_dev, 255) if raw_filter else qa_dev
        rows = []
        for beam in beams:
            kk = beam if raw_filter else k

            def step():
                cand = nhq.nhq_seed_rank(ix, q, qa_search, n_cand)
                return nhq.nhq_search_seeded(ix, q, qa_search, cand, kk, beam, n_init=args.n_init,
                                             expand=args.expand, output_mode=1 if raw_filter else 0)
            ids, _ = step()
            ids = ids.cpu().numpy()
            if raw_filter:
                keep = np.full((nq, k), -1, dtype=np.int64)
                for i in range(nq):
                    m_ = ids[i][ids[i] >= 0]
                    m_ = m_[(attrs_np[m_] == qattrs_np[i]).all(axis=1)][:k]
                    keep[i, :len(m_)] = m_
                ids = keep
            rec = float(recall_at_k(ids, w.x, w.q, attrs_np, qattrs_np, gi, k).mean())
            step()
            torch.cuda.synchronize()
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record()
            for _ in range(3):
                step()
            e1.record()
            torch.cuda.synchronize()
            ms = e0.elapsed_time(e1) / 3
            rows.append({"beam": beam, "recall": round(rec, 5), "qps": round(nq / (ms / 1000.0), 1)})
            log("%s beam %d recall %.4f %.0f QPS" % (label, beam, rec, rows[-1]["qps"]))
            if rec >= 0.999:
                break
        at = qps_at_recall([r["beam"] for r in rows], [r["recall"] for r in rows],
                           [r["qps"] for r in rows], args.target)
        return {"curve": rows, "qps_at_target": None if at is None else round(at, 1),
                "best_recall": max(r["recall"] for r in rows)}

    def index_for(attrs_np, **params):
        a_dev = torch.from_numpy(attrs_np).to(dev)
        t = time.time()
        ix = nhq.nhq_build_index(x, a_dev, degree=w.degree, cand=w.cand, n_entry=args.n_entry,
                                 seed=w.build_seed, **params)
        torch.cuda.synchronize()
        return ix, a_dev, time.time() - t

    out = {}
    # ---- weight settings
    ix0, a0, b0 = index_for(w.attrs)
    gi, gd = nhq.nhq_bruteforce_hybrid_knn(ix0, q, torch.from_numpy(w.qattrs).to(dev), k)
    gi, gd = gi.cpu().numpy(), gd.cpu().numpy()
    # delta statistics of the object set: the largest distance from 1,000
    # sampled objects to all objects (delta_max of curve iii) and the median
    # over 100,000 random pairs (the ratio of curve v, which the paper puts
    # close to the median delta)
    rng = np.random.default_rng(5)
    smp = torch.from_numpy(rng.integers(0, w.n, 1000)).to(dev)
    xs = x[smp].double()
    dmax2 = 0.0
    for c0 in range(0, w.n, 100_000):
        blk = x[c0:c0 + 100_000].double()
        d2 = (xs * xs).sum(1)[:, None] + (blk * blk).sum(1)[None, :] - 2.0 * xs @ blk.T
        dmax2 = max(dmax2, float(d2.max()))
    pa, pb = rng.integers(0, w.n, 100_000), rng.integers(0, w.n, 100_000)
    dmed = float(np.median(np.sqrt(((w.x[pa].astype(np.float64) - w.x[pb]) ** 2).sum(1))))
    dmax = float(np.sqrt(dmax2))
    log("delta_max %.1f, median delta %.1f" % (dmax, dmed))
    settings = [("iv", "default", 0.0), ("i", "harmonic", 0.0), ("ii", "harmonic_c", 100.0),
                ("iii", "normalised", dmax), ("v", "fixed", dmed)]
    wres = {}
    for curve_id, mode, p in settings:
        if mode == "default":
            ix, bs = ix0, b0
        else:
            ix, _, bs = index_for(w.attrs, weights=mode, weight_param=p)
        r = curve(ix, w.attrs, w.qattrs, gi, gd, "weights %s (%s)" % (curve_id, mode))
        r.update({"setting": mode, "param": p, "build_s": round(bs, 2)})
        wres[curve_id] = r
        if ix is not ix0:
            ix.free()
    out["weights"] = wres
    # ---- strategy B(1): vector-only search, then the attribute filter
    out["post_filter"] = curve(ix0, w.attrs, w.qattrs, gi, gd, "post-filter B(1)", raw_filter=True)
    # ---- selectivity
    sres = {}
    for cards in ((2, 2, 2), (3, 4, 5), (5, 8, 10), (10, 20, 20)):
        if cards == tuple(w.cards):
            ix, a_np, qa_np, g_i, g_d = ix0, w.attrs, w.qattrs, gi, gd
        else:
            a_np = synth.uniform_attrs(w.n, cards, 202)
            qa_np = synth.uniform_attrs(nq, cards, 204)
            ix, a_dev, _ = index_for(a_np)
            g_i, g_d = nhq.nhq_bruteforce_hybrid_knn(ix, q, torch.from_numpy(qa_np).to(dev), k)
            g_i, g_d = g_i.cpu().numpy(), g_d.cpu().numpy()
        frac = 1.0 / float(np.prod(cards))
        r = curve(ix, a_np, qa_np, g_i, g_d, "selectivity 1-1/%d" % int(np.prod(cards)))
        r.update({"cards": list(cards), "match_fraction": frac, "selectivity": 1.0 - frac})
        sres["1/%d" % int(np.prod(cards))] = r
        if ix is not ix0:
            ix.free()
    out["selectivity"] = sres
    # ---- attribute dimension (m = 6 and 9; binary attributes, so m = 6
    # matches the 1/60 selectivity of the m = 3 set closely)
    mres = {"3": {"cards": list(w.cards), "match_fraction": 1.0 / float(np.prod(w.cards)),
                  **sres["1/%d" % int(np.prod(w.cards))]}}
    for m_, cards in ((6, (2,) * 6), (9, (2,) * 9)):
        a_np = synth.uniform_attrs(w.n, cards, 202)
        qa_np = synth.uniform_attrs(nq, cards, 204)
        ix, _, _ = index_for(a_np)
        g_i, g_d = nhq.nhq_bruteforce_hybrid_knn(ix, q, torch.from_numpy(qa_np).to(dev), k)
        g_i, g_d = g_i.cpu().numpy(), g_d.cpu().numpy()
        r = curve(ix, a_np, qa_np, g_i, g_d, "m = %d" % m_)
        r.update({"cards": list(cards), "match_fraction": 1.0 / float(np.prod(cards))})
        mres[str(m_)] = r
        ix.free()
    out["attribute_dimension"] = mres
    print(json.dumps({"metric": "parameter studies (Sec. 6.5): Recall@10 / QPS curves on 1 GPU",
                      "value": wres["iv"]["qps_at_target"], "unit": "queries/s", "n_gpus": 1,
                      "higher_is_better": True, "vs_baseline": None, "dtype": "f32",
                      "data": "synthetic",
                      "config": {"workload": w.name, "n": w.n, "d": w.d, "queries_per_step": nq,
                                 "k": k, "expand": args.expand, "n_init": args.n_init,
                                 "n_entry": args.n_entry, "delta_max": dmax, "delta_median": dmed},
                      **out}), flush=True)



if __name__ == "__main__":
    main()
