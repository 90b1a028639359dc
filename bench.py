"""Benchmark: hybrid QPS at Recall@10 = 0.95 on one MI355X, plain FP32 fixed
beam against BF16 storage + learned stop, and p99 latency of the serving
loop.

Workload: the plain method at scale -- 1,000,000 integer-valued 128-d
vectors from 256 clusters, 3 uniform attributes of cardinality 3/4/5,
10,000 queries with full constraints, out-degree 32, k = 10.  The composite
index is built on the GPU (not timed); the exact answers come from the GPU
brute force (parity-tested against the CPU oracle).

1. Plain form (the reported ``value``): float32 storage, fixed beam.  A beam
   sweep finds the smallest beam reaching Recall@10 >= 0.95; one timed
   "step" is one full pass of the hot path over the 10,000 queries at that
   beam: seed ranking of the entry sample (matrix cores) plus the
   joint-pruning search (one wavefront per query).
2. BF16 + learned stop: the same graph with bf16 row storage; the stop
   network is trained on the GPU from traces of 20,000 separate training
   queries and runs inside the search (one checkpoint, whose beam output
   sets the hop budget); the budget factor is swept for Recall@10 >= 0.95
   and the same step is timed.
3. Serving: the bf16 index under a Poisson stream of requests (k uniform in
   {1, 10, 50, 100}, 1 to 3 constrained attributes, the beam left to a stop
   network trained on queries with that constraint law), through the
   continuous-batching server: p50 / p99 latency from arrival to result,
   sustained QPS, Recall@10 of the k >= 10 requests.

Inputs are resident in HBM before every timed region.  Prints ONE JSON line.
``--gpus N`` with N > 1 exits: this build runs on one GPU.
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


SEARCH_SOURCES = "paper_2203_13601_amd/csrc/search.hip,paper_2203_13601_amd/csrc/search_core.h"


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--n", type=int, default=1_000_000)
    ap.add_argument("--nq", type=int, default=10_000)
    ap.add_argument("--target", type=float, default=0.95)
    ap.add_argument("--beam", type=int, default=0, help="fixed beam (skip the choice)")
    ap.add_argument("--n-entry", type=int, default=None,
                    help="entry sample size (default 4096; 1024 for the precision workload, whose "
                         "64 clusters need fewer entries)")
    ap.add_argument("--n-init", type=int, default=4)
    ap.add_argument("--expand", type=int, default=6, help="vertices expanded per step")
    ap.add_argument("--plain-only", action="store_true", help="skip the bf16/learned and serving legs")
    ap.add_argument("--serve-rate", type=float, default=50_000.0)
    ap.add_argument("--serve-requests", type=int, default=50_000)
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run a plain device copy of known size (counter scaling)")
    ap.add_argument("--workload", default="plain",
                    choices=["plain", "precision", "ablation", "build"],
                    help="precision: the d = 960 storage forms (fp32 / bf16 / fp8 + exact rerank); "
                         "ablation: weight settings, selectivity and post-filtering sweeps; "
                         "build: exact vs NN-descent candidate lists (1M and 10M sets)")
    args = ap.parse_args()
    if args.n_entry is None:
        args.n_entry = 1024 if args.workload == "precision" else 4096

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py: this build measures one GPU only (--gpus 1); multi-GPU runs are not "
              "part of it", file=sys.stderr)
        sys.exit(2)

    import torch
    import synth
    import paper_2203_13601_amd as nhq
    from paper_2203_13601_amd.learned import train_stop_network
    from paper_2203_13601_amd.metrics import qps_at_recall, recall_at_k, search_bytes_per_query

    if args.workload == "precision":
        return precision_form(args)
    if args.workload == "ablation":
        return ablation(args)
    if args.workload == "build":
        return build_study(args)
    dev = torch.device("cuda:0")
    t_gen = time.time()
    w = synth.config2(n=args.n, nq=args.nq)
    log("generated %s in %.1fs" % (w.name, time.time() - t_gen))
    x = torch.from_numpy(w.x).to(dev)
    a = torch.from_numpy(w.attrs).to(dev)
    q = torch.from_numpy(w.q).to(dev)
    qa = torch.from_numpy(w.qattrs).to(dev)
    torch.cuda.synchronize()

    t0 = time.time()
    ix = nhq.nhq_build_index(x, a, degree=w.degree, cand=w.cand, storage="fp32",
                             n_entry=args.n_entry, seed=w.build_seed)
    torch.cuda.synchronize()
    build_s = time.time() - t0
    log("built the composite index in %.2fs" % build_s)

    t0 = time.time()
    gi, gd = nhq.nhq_bruteforce_hybrid_knn(ix, q, qa, w.k)
    torch.cuda.synchronize()
    gt_s = time.time() - t0
    gi, gd = gi.cpu().numpy(), gd.cpu().numpy()
    log("exact answers in %.2fs" % gt_s)

    nq, k = w.nq, w.k
    n_cand = min(args.n_entry, args.n_init + SEED_MARGIN)
    cand = torch.empty((nq, n_cand), dtype=torch.int32, device=dev)
    ids = torch.empty((nq, k), dtype=torch.int32, device=dev)
    dists = torch.empty((nq, k), dtype=torch.float32, device=dev)

    def step(index, beam, counters=False, ev=None, **kw):
        if ev is not None:
            ev[0].record()
        nhq.nhq_seed_rank(index, q, qa, n_cand, out=cand)
        if ev is not None:
            ev[1].record()
        r = nhq.nhq_search_seeded(index, q, qa, cand, k, beam, n_init=args.n_init, counters=counters,
                                  out=(ids, dists), expand=args.expand, **kw)
        if ev is not None:
            ev[2].record()
        return r

    def timed(index, beam, reps, **kw):
        # wall clock over `reps` steps with nothing else on the stream; then
        # the same number of steps with HIP events around each stage (event
        # records are stream packets of their own, so they stay out of the
        # wall-clock loop)
        torch.cuda.synchronize()
        t = time.time()
        for _ in range(reps):
            step(index, beam, **kw)
        torch.cuda.synchronize()
        wall = time.time() - t
        evs = [[torch.cuda.Event(enable_timing=True) for _ in range(3)] for _ in range(reps)]
        for e in evs:
            step(index, beam, ev=e, **kw)
        torch.cuda.synchronize()
        rank_ms = [e[0].elapsed_time(e[1]) for e in evs]
        search_ms = [e[1].elapsed_time(e[2]) for e in evs]
        return wall, rank_ms, search_ms

    def point(index, beam, elem=4, **kw):
        _, _, cnt = step(index, beam, counters=True, **kw)
        torch.cuda.synchronize()
        rec = recall_at_k(ids.cpu().numpy(), dists.cpu().numpy(), gi, gd, w.attrs, w.qattrs, k)
        cnt = cnt.cpu().numpy().astype(np.float64)
        step(index, beam, **kw)
        wall, rk, se = timed(index, beam, 3, **kw)
        bq_p = search_bytes_per_query(d_pad=128, elem_bytes=elem, R=w.degree, k=k, n_cand=n_cand,
                                      ndc=float(cnt[:, 0].mean()), hops=float(cnt[:, 1].mean()), d=w.d, m=w.m)
        return {"beam": beam, "recall": float(rec.mean()), "qps": nq * 3 / wall,
                "ndc": float(cnt[:, 0].mean()), "hops": float(cnt[:, 1].mean()),
                "hops_p99": float(np.percentile(cnt[:, 1], 99)),
                "rank_ms": float(np.median(rk)), "search_ms": float(np.median(se)),
                "search_hbm_frac": bq_p * nq / (float(np.median(se)) / 1000.0) / 8.0e12}

    # ---- 1. plain form: float32 storage, fixed beam
    sweep = []
    beams = [args.beam] if args.beam else [10, 16, 20, 24, 28, 32, 36, 40, 48, 56, 64, 96, 128, 256, 512]
    for beam in beams:
        if beam < k:
            continue
        p = point(ix, beam)
        sweep.append(p)
        log("fp32 beam %4d recall %.4f ndc %.0f hops %.0f rank %.3fms search %.3fms" % (
            beam, p["recall"], p["ndc"], p["hops"], p["rank_ms"], p["search_ms"]))
        if not args.beam and p["recall"] >= args.target and beam >= 64:
            break
    ok = [s for s in sweep if s["recall"] >= args.target]
    op = ok[0] if ok else sweep[-1]
    beam = op["beam"]
    q_at = qps_at_recall([s["beam"] for s in sweep], [s["recall"] for s in sweep],
                         [s["qps"] for s in sweep], args.target)
    for _ in range(args.warmup):
        step(ix, beam)
    wall, rank_ms, search_ms = timed(ix, beam, args.steps)
    value = nq * args.steps / wall
    ms_per_step = wall * 1000.0 / args.steps
    log("plain fp32: %d steps at beam %d: %.3f ms/step, %.0f QPS" % (args.steps, beam, ms_per_step, value))

    # ---- roofline of the dominant kernel (the search)
    bq = search_bytes_per_query(d_pad=128, elem_bytes=4, R=w.degree, k=k, n_cand=n_cand,
                                ndc=op["ndc"], hops=op["hops"], d=w.d, m=w.m)
    search_avg_s = float(np.mean(search_ms)) / 1000.0
    traffic = None
    if args.n == 1_000_000 and args.nq == 10_000:
        traffic = _profiled_traffic("k_search", SEARCH_SOURCES, "_beam%d" % beam)
    achieved = bq * nq / search_avg_s / 1e9
    roof = {"bound": "hbm", "achieved": round(achieved, 2), "peak": 8000.0, "unit": "GB/s",
            "frac": round(achieved / 8000.0, 5), "traffic": traffic,
            "kernel": "k_search", "bytes_per_query": round(bq, 1), "queries_per_launch": nq,
            "kernel_avg_ms": round(search_avg_s * 1000.0, 4),
            "rank_kernels_avg_ms": round(float(np.mean(rank_ms)), 4)}

    # random-row gather ceiling at the same row size and lane layout
    waves, rounds = 65536, 20
    nhq.nhq_gather_probe(ix, waves, rounds)
    pe = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
    torch.cuda.synchronize()
    pe[0].record()
    for _ in range(3):
        _, rows = nhq.nhq_gather_probe(ix, waves, rounds)
    pe[1].record()
    torch.cuda.synchronize()
    gather_gbs = rows * 128 * 4 / (pe[0].elapsed_time(pe[1]) / 3 / 1000.0) / 1e9
    roof["gather_ceiling"] = round(gather_gbs, 1)
    roof["frac_of_gather_ceiling"] = round(achieved / gather_gbs, 4)
    log("random 512-byte row gathers: %.0f GB/s; the search reaches %.1f%% of that" % (
        gather_gbs, 100.0 * achieved / gather_gbs))

    if args.copy_calibration:
        src = torch.empty(1 << 28, dtype=torch.float32, device=dev)  # 1 GiB
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
        log("copy calibration: 3 copies of 1 GiB")

    forms = {"fp32_fixed": {"qps": round(value, 1), "recall": round(op["recall"], 5), "beam": beam,
                            "ms_per_step": round(ms_per_step, 4),
                            "qps_at_target_interp": None if q_at is None else round(q_at, 1)}}
    serving = None
    if not args.plain_only:
        # ---- 2. bf16 storage + learned stop (same graph and entry sample)
        ixb = nhq.nhq_index_create(x, a, storage="bf16", n_entry=args.n_entry, seed=w.build_seed,
                                   degree=w.degree)
        nhq.nhq_index_set_graph(ixb, nhq.nhq_index_get_graph(ix))
        tq_np, tqa_np = synth.config2_train_queries(20_000)
        tq, tqa = torch.from_numpy(tq_np).to(dev), torch.from_numpy(tqa_np).to(dev)
        ce = 8
        # bf16 with a fixed beam first (same beam as the plain form): the
        # reference the learned stop has to beat at equal storage
        bp = point(ixb, beam, elem=2)
        for _ in range(args.warmup):
            step(ixb, beam)
        bwall, _, bsearch = timed(ixb, beam, args.steps)
        forms["bf16_fixed"] = {"qps": round(nq * args.steps / bwall, 1), "recall": round(bp["recall"], 5),
                               "beam": beam, "ms_per_step": round(bwall * 1000.0 / args.steps, 4),
                               "search_kernel_avg_ms": round(float(np.mean(bsearch)), 4)}
        log("bf16 fixed beam %d: recall %.4f, %.0f QPS" % (beam, bp["recall"], forms["bf16_fixed"]["qps"]))
        # the stop network per training beam; each beam's cap sweep stops at
        # the first factor that reaches the target; the fastest beam is kept
        best = None
        for l_train in (40, 64):
            t0 = time.time()
            params, info = train_stop_network(ixb, tq, tqa, k, l_train, epochs=30, check_every=ce,
                                              n_init=args.n_init, expand=args.expand, seed=1)
            nhq.nhq_mlp_load(ixb, params)
            torch.cuda.synchronize()
            train_s = time.time() - t0
            log("stop network at beam %d: %d trace samples, trained in %.2fs (loss %.4f)" % (
                l_train, info["samples"], train_s, info["losses"][-1]))
            lsweep = []
            lkw = None
            for cf in (1.0, 1.125, 1.25, 1.5, 1.75, 2.0, 2.5, 3.0):
                kw = dict(learned=2, stop_threshold=0.9, check_every=ce, cap_factor=cf)
                p = point(ixb, l_train, elem=2, **kw)
                p["cap_factor"] = cf
                lsweep.append(p)
                log("bf16+learned beam %d cap %.2f recall %.4f hops %.1f (p99 %.0f) search %.3fms" % (
                    l_train, cf, p["recall"], p["hops"], p["hops_p99"], p["search_ms"]))
                if p["recall"] >= args.target:
                    lkw = kw
                    break
            if lkw is None:
                continue
            lop = lsweep[-1]
            for _ in range(args.warmup):
                step(ixb, l_train, **lkw)
            lwall, lrank, lsearch = timed(ixb, l_train, args.steps, **lkw)
            lvalue = nq * args.steps / lwall
            log("bf16+learned beam %d: %d steps: %.3f ms/step, %.0f QPS" % (
                l_train, args.steps, lwall * 1000 / args.steps, lvalue))
            cand_form = {
                "qps": round(lvalue, 1), "recall": round(lop["recall"], 5), "beam": l_train,
                "learned_mode": 2, "check_every": ce, "cap_factor": lkw["cap_factor"],
                "hops_mean": round(lop["hops"], 2), "hops_p99": lop["hops_p99"],
                "ms_per_step": round(lwall * 1000.0 / args.steps, 4),
                "search_kernel_avg_ms": round(float(np.mean(lsearch)), 4),
                "train_samples": info["samples"], "train_s": round(train_s, 2),
                "speedup_vs_fp32_fixed": round(lvalue / value, 4),
                "sweep": [{kk: (round(vv, 5) if isinstance(vv, float) else vv) for kk, vv in sp.items()}
                          for sp in lsweep]}
            if best is None or cand_form["qps"] > best["qps"]:
                best = cand_form
        if best is not None:
            forms["bf16_learned"] = best

        # ---- 3. serving: Poisson stream through the continuous-batching server
        ns = args.serve_requests
        rng = np.random.default_rng(502)
        s_q = np.ascontiguousarray(w.q[rng.integers(0, nq, size=ns)])
        s_qa = synth.partial_constraints(ns, w.cards, 504)
        s_k = rng.choice(np.array([1, 10, 50, 100], dtype=np.int32), size=ns)
        s_arr = synth.poisson_arrivals(ns, args.serve_rate, 501)
        s_beam = np.zeros(ns, dtype=np.int32)  # the stop network chooses (automatic beam)
        sq_d, sqa_d = torch.from_numpy(s_q).to(dev), torch.from_numpy(s_qa).to(dev)
        gsi, gsd = nhq.nhq_bruteforce_hybrid_knn(ix, sq_d, sqa_d, k)
        gsi, gsd = gsi.cpu().numpy(), gsd.cpu().numpy()
        # the serving network: traces of training queries with the stream's
        # constraint law (1..3 constrained attributes) at the automatic beam
        s_beam_auto, s_ce = 256, 8
        tqa_p = torch.from_numpy(synth.partial_constraints(tq.shape[0], w.cards, 505)).to(dev)
        sparams, sinfo = train_stop_network(ixb, tq, tqa_p, k, s_beam_auto, epochs=30, check_every=s_ce,
                                            n_init=args.n_init, expand=args.expand, seed=2)
        nhq.nhq_mlp_load(ixb, sparams)
        # budget factor: the smallest reaching the target on a validation slice (batch search)
        nv = min(5000, ns)
        s_cf = None
        for cf in (1.5, 2.0, 2.5, 3.0, 4.0, 6.0):
            vi, vd = nhq.nhq_hybrid_search(ixb, sq_d[:nv], sqa_d[:nv], k, s_beam_auto, n_init=args.n_init,
                                           expand=args.expand, learned=2, stop_threshold=0.9,
                                           check_every=s_ce, cap_factor=cf)
            vr = recall_at_k(vi.cpu().numpy(), vd.cpu().numpy(), gsi[:nv], gsd[:nv], w.attrs, s_qa[:nv], k)
            log("serving network: cap %.1f validation recall %.4f" % (cf, vr.mean()))
            s_cf = cf
            if vr.mean() >= args.target + 0.005:
                break
        torch.cuda.synchronize()
        with nhq.Server(ixb, n_init=args.n_init, expand=args.expand, auto_beam=s_beam_auto,
                        beam_small=s_beam_auto, beam_large=-1, max_k=100, ring=8192, learned_mode=2,
                        cap_factor=s_cf, stop_threshold=0.9, check_every=s_ce, lifetime_s=120.0) as srv:
            r = srv.run(s_q, s_qa, s_k, s_beam, s_arr, timeout_s=60.0)
            slots = srv.slots
            hz = srv.tick_hz
        lat_ms = r["latency_s"] * 1000.0
        svc_ms = (r["ticks"][:, 1].astype(np.float64) - r["ticks"][:, 0]) / hz * 1000.0
        big = s_k >= 10
        srec = recall_at_k(r["ids"][big, :10], r["dists"][big, :10], gsi[big], gsd[big], w.attrs,
                           s_qa[big], k)
        serving = {"offered_qps": args.serve_rate, "requests": ns,
                   "sustained_qps": round(ns / r["elapsed_s"], 1),
                   "p50_ms": round(float(np.percentile(lat_ms, 50)), 4),
                   "p99_ms": round(float(np.percentile(lat_ms, 99)), 4),
                   "max_ms": round(float(lat_ms.max()), 4),
                   "device_service_p50_ms": round(float(np.percentile(svc_ms, 50)), 4),
                   "device_service_p99_ms": round(float(np.percentile(svc_ms, 99)), 4),
                   "recall_at_10_k_ge_10": round(float(srec.mean()), 5),
                   "hops_mean": round(float(r["counters"][:, 1].mean()), 2),
                   "k_mix": [1, 10, 50, 100], "constrained_attrs": "1..3 of 3",
                   "beam": "learned budget at automatic beam %d (cap factor %.1f)" % (s_beam_auto, s_cf),
                   "storage": "bf16", "slots": slots[0], "latency": "arrival to result seen by the host"}
        log("serving: %d requests at %.0f/s offered: p50 %.3f ms, p99 %.3f ms, recall@10 %.4f" % (
            ns, args.serve_rate, serving["p50_ms"], serving["p99_ms"], serving["recall_at_10_k_ge_10"]))

    # ---- CPU oracle on a bounded sample (same graph, entry sample, beam)
    cpu = None
    if not args.no_cpu_baseline:
        import oracle
        adj = nhq.nhq_index_get_graph(ix).cpu().numpy()
        entry = oracle.entry_points(w.build_seed, w.n, args.n_entry)
        threads = os.cpu_count() or 1
        nsamp = 64
        kw = dict(n_init=args.n_init, key_mode=oracle.KEY32, threads=threads, expand=args.expand)
        t = time.time()
        oracle.search(adj, w.x, w.attrs, w.q[:nsamp], w.qattrs[:nsamp], k, beam, entry, **kw)
        el = time.time() - t
        if el < args.cpu_seconds:
            nsamp = int(min(nq, max(nsamp, nsamp * args.cpu_seconds / max(el, 1e-3))))
            t = time.time()
            oracle.search(adj, w.x, w.attrs, w.q[:nsamp], w.qattrs[:nsamp], k, beam, entry, **kw)
            el = time.time() - t
        n1 = min(nq, max(16, int(nsamp / threads)))
        t = time.time()
        oracle.search(adj, w.x, w.attrs, w.q[:n1], w.qattrs[:n1], k, beam, entry, **dict(kw, threads=1))
        el1 = time.time() - t
        cpu = {"value": round(nsamp / el, 1), "unit": "queries/s", "cores": threads, "kind": "oracle",
               "single_thread_value": round(n1 / el1, 1),
               "sample": "%d of %d queries, beam %d, expand %d, same graph and entry sample, FP64 C "
                         "oracle (entry-sample scan + joint pruning), %d threads" % (
                             nsamp, nq, beam, args.expand, threads)}
        log("cpu oracle: %.1f QPS on %d threads" % (nsamp / el, threads))

    out = {
        "metric": "hybrid QPS at Recall@10=0.95 on 1 GPU, plain FP32 vs BF16+learned-stop; p99 ms",
        "value": round(value, 1),
        "unit": "queries/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": w.name, "form": "plain FP32 fixed beam", "n": w.n, "d": w.d, "m": w.m,
                   "cards": list(w.cards), "queries_per_step": nq, "k": k, "beam": beam,
                   "degree": w.degree, "cand": w.cand, "n_entry": args.n_entry, "n_init": args.n_init,
                   "expand": args.expand, "recall_at_beam": round(op["recall"], 5),
                   "build_s": round(build_s, 3), "exact_knn_s": round(gt_s, 3),
                   "parallelism": "single GPU"},
        "p99_ms": None if serving is None else serving["p99_ms"],
        "forms": forms,
        "serving": serving,
        "sweep": sweep,
        "roofline": roof,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


def precision_form(args):
    """The storage forms on the precision-form shape: d = 960 Gaussian mixture
    (64 centres), 4 attributes of cardinality 2/3/5/10, all constrained.  One
    graph (built from the float32 rows) serves float32, bf16 and fp8 e4m3
    (per-row scale) storage; bf16 and fp8 re-score the first 4k eligible
    entries from the float32 copy.  For each form: the smallest beam reaching
    Recall@10 >= target, its timed step, the search kernel's HBM fraction and
    the relative error of every returned distance against FP64."""
    import torch
    import synth
    import paper_2203_13601_amd as nhq
    from paper_2203_13601_amd.metrics import recall_at_k, search_bytes_per_query
    dev = torch.device("cuda:0")
    w = synth.config3(n=args.n, nq=args.nq)

    # FP64 references of the measurement (plain numpy): Gamma = delta (1 + chi / m_q)
    def gamma_fp64(qv, qattr, xv, xattr):
        cons = qattr != 0xFF
        mq = int(cons.sum())
        chi = int((cons & (qattr != xattr)).sum())
        dl = float(np.sqrt(((qv.astype(np.float64) - xv.astype(np.float64)) ** 2).sum()))
        return dl if mq == 0 else dl * (1.0 + chi / mq)

    def decode_bf16(bits):
        return (bits.astype(np.uint32) << 16).view(np.float32).astype(np.float64)

    def decode_e4m3(codes, scales):
        c = codes.astype(np.int64)
        sgn = np.where(c >> 7, -1.0, 1.0)
        e, mnt = (c >> 3) & 15, c & 7
        val = np.where(e == 0, mnt / 8.0 * 2.0 ** -6, (1.0 + mnt / 8.0) * 2.0 ** (e - 7.0))
        return sgn * val * scales[:, None]
    x = torch.from_numpy(w.x).to(dev)
    a = torch.from_numpy(w.attrs).to(dev)
    q = torch.from_numpy(w.q).to(dev)
    qa = torch.from_numpy(w.qattrs).to(dev)
    t0 = time.time()
    ix = nhq.nhq_build_index(x, a, degree=w.degree, cand=w.cand, n_entry=args.n_entry, seed=w.build_seed)
    torch.cuda.synchronize()
    build_s = time.time() - t0
    log("built %s in %.1fs" % (w.name, build_s))
    gi, gd = nhq.nhq_bruteforce_hybrid_knn(ix, q, qa, w.k)
    gi, gd = gi.cpu().numpy(), gd.cpu().numpy()
    adj = nhq.nhq_index_get_graph(ix)
    k, nq = w.k, w.nq
    n_cand = min(args.n_entry, args.n_init + SEED_MARGIN)
    cand = torch.empty((nq, n_cand), dtype=torch.int32, device=dev)
    nsamp = min(nq, 1000)

    def gamma64(ids, dist):
        """|Gamma returned - Gamma FP64| / Gamma FP64 for every returned result of the sample"""
        errs = []
        for i in range(nsamp):
            for v, g in zip(ids[i], dist[i]):
                if v < 0:
                    continue
                ex = gamma_fp64(w.q[i], w.qattrs[i], w.x[v], w.attrs[v])
                errs.append(abs(float(g) - ex) / max(ex, 1e-30))
        e = np.asarray(errs)
        return {"results": int(e.size), "max": float(e.max()), "p99": float(np.percentile(e, 99)),
                "mean": float(e.mean())}

    forms = {}
    for storage, elem, scale_b, rr in (("fp32", 4, 0, 0), ("bf16", 2, 0, 4), ("fp8", 1, 4, 4)):
        index = ix if storage == "fp32" else nhq.nhq_index_create(x, a, storage=storage, n_entry=args.n_entry,
                                                                   seed=w.build_seed, degree=w.degree)
        if index is not ix:
            nhq.nhq_index_set_graph(index, adj)
        kw = dict(n_init=args.n_init, expand=args.expand, rerank=rr)

        def step(beam, counters=False):
            nhq.nhq_seed_rank(index, q, qa, n_cand, out=cand)
            return nhq.nhq_search_seeded(index, q, qa, cand, k, beam, counters=counters, **kw)

        chosen = None
        sweep = []
        beams = (10, 16, 24, 32, 40, 48, 64, 96, 128, 192, 256, 384, 512)
        for beam in beams:
            if beam < rr * k:
                continue
            ids, dist, cnt = step(beam, counters=True)
            torch.cuda.synchronize()
            ids_np, dist_np = ids.cpu().numpy(), dist.cpu().numpy()
            rec = float(recall_at_k(ids_np, dist_np, gi, gd, w.attrs, w.qattrs, k).mean())
            c = cnt.cpu().numpy().astype(np.float64)
            sweep.append({"beam": beam, "recall": round(rec, 5), "ndc": round(c[:, 0].mean(), 1),
                          "hops": round(c[:, 1].mean(), 1)})
            log("%s beam %d recall %.4f" % (storage, beam, rec))
            if rec >= args.target:
                chosen = (beam, rec, c, ids_np, dist_np)
                break
        if chosen is None:
            chosen = (beam, rec, c, ids_np, dist_np)
        beam, rec, c, ids_np, dist_np = chosen
        for _ in range(args.warmup):
            step(beam)
        evs = [[torch.cuda.Event(enable_timing=True) for _ in range(3)] for _ in range(args.steps)]
        torch.cuda.synchronize()
        t = time.time()
        for e in evs:
            e[0].record()
            nhq.nhq_seed_rank(index, q, qa, n_cand, out=cand)
            e[1].record()
            nhq.nhq_search_seeded(index, q, qa, cand, k, beam, **kw)
            e[2].record()
        torch.cuda.synchronize()
        wall = time.time() - t
        search_ms = float(np.mean([e[1].elapsed_time(e[2]) for e in evs]))
        bq = search_bytes_per_query(d_pad=960, elem_bytes=elem, R=w.degree, k=k, n_cand=n_cand,
                                    ndc=c[:, 0].mean(), hops=c[:, 1].mean(), d=w.d, m=w.m,
                                    scale_bytes=scale_b, out_rows=(rr * k if rr else k))
        err = gamma64(ids_np, dist_np)
        form = {"beam": beam, "recall": round(rec, 5), "qps": round(nq * args.steps / wall, 1),
                "ms_per_step": round(wall * 1000 / args.steps, 4), "search_kernel_ms": round(search_ms, 4),
                "bytes_per_query": round(bq, 1),
                "search_hbm_frac": round(bq * nq / (search_ms / 1000.0) / 8.0e12, 4),
                "rerank": rr, "gamma_rel_err_vs_fp64": err, "sweep": sweep}
        if storage != "fp32":
            # Gamma from the stored (decoded) rows of the returned objects: the
            # approximation the loop orders by before the float32 re-score
            rows, scales = nhq.nhq_index_get_storage(index)
            sel = torch.from_numpy(ids_np[:nsamp].clip(min=0).astype(np.int64)).to(dev)
            r_np = rows[sel.reshape(-1)].cpu().numpy()
            if storage == "bf16":
                dec = decode_bf16(r_np.view(np.uint16))
            else:
                dec = decode_e4m3(r_np, scales[sel.reshape(-1)].cpu().numpy().astype(np.float64))
            dec = dec.reshape(nsamp, k, -1)[:, :, : w.d]
            errs = []
            for i in range(nsamp):
                for j in range(k):
                    v = ids_np[i, j]
                    if v < 0:
                        continue
                    ex = gamma_fp64(w.q[i], w.qattrs[i], w.x[v], w.attrs[v])
                    ap = gamma_fp64(w.q[i], w.qattrs[i], dec[i, j], w.attrs[v])
                    errs.append(abs(ap - ex) / max(ex, 1e-30))
            e = np.asarray(errs)
            form["stored_form_gamma_rel_err"] = {"results": int(e.size), "max": float(e.max()),
                                                 "p99": float(np.percentile(e, 99)), "mean": float(e.mean())}
            del rows
        forms[storage] = form
        log("%s: beam %d recall %.4f %.0f QPS, search %.3f ms (%.1f%% of HBM), max rel err %.2e" % (
            storage, beam, rec, form["qps"], search_ms, 100 * form["search_hbm_frac"], err["max"]))
        if index is not ix:
            index.free()
    out = {"metric": "hybrid QPS at Recall@10=0.95 on 1 GPU, storage forms (precision form)",
           "value": forms["bf16"]["qps"], "unit": "queries/s", "n_gpus": 1, "steps": args.steps,
           "warmup": args.warmup, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
           "dtype": "bf16", "data": "synthetic",
           "config": {"workload": w.name, "n": w.n, "d": w.d, "m": w.m, "cards": list(w.cards),
                      "queries_per_step": nq, "k": k, "expand": args.expand, "n_entry": args.n_entry,
                      "build_s": round(build_s, 2)},
           "forms": forms}
    print(json.dumps(out), flush=True)


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
            rec = float(recall_at_k(ids.cpu().numpy(), d.cpu().numpy(), gi, gd, w.attrs, w.qattrs,
                                    w.k).mean())
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

    def true_delta(ids):
        v = np.where(ids >= 0, ids, 0)
        dd = np.sqrt(((w.x[v].astype(np.float64) - w.q[:, None, :]) ** 2).sum(-1))
        return np.where(ids >= 0, dd, np.inf)

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
            rec = float(recall_at_k(ids, true_delta(ids), gi, gd, attrs_np, qattrs_np, k).mean())
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
