"""Benchmark: exact kNN (k=16) + FoF (b = 0.2 x mean spacing) at N = 2^24 on one GPU.

One step = jz_build (z-order sort + tree planes) + jz_knn_fof(k, b) (kNN and
FoF on the same tree, run concurrently on two streams; --serial: jz_knn then
jz_fof) + jz_tree_free on a clustered synthetic point set already resident in HBM
(60% of points in 4096 Gaussian clumps, 40% uniform background; the stand-in
for the paper's cosmological snapshots). The tree grows nodes 16-fold per plane
in the concurrent schedule (the library's default of 8 with --serial). Prints
one JSON line.

value = N * steps / (wall time of the timed steps)  [points/s]

The line also carries:
  roofline     the dominant kernel (leaf-stage kNN), timed with HIP events on
               the stream it runs on, against the FP32 VALU rate for plain
               (non-fused, non-packed) add/mul: 256 CU * 64 lanes * 2.4 GHz
  cpu_baseline the CPU oracle (exact kd-tree kNN + FoF) on the host cores,
               and the last step's GPU result compared with it
  fp64_report  binary64 cross-check of that result (sampled kNN rows, every
               FoF pair): decisions that flip at float32 near-ties
  breakdown    device times (build, kNN + FoF, and each half's own) and walk
               statistics
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

FLOPS_PER_EVAL = 8            # 3 sub + 3 mul + 2 add per squared distance
VALU_PEAK_TFLOPS = 256 * 64 * 2.4e9 / 1e12  # plain fp32 add/mul, no FMA, no packed ops
HBM_PEAK_GBS = 8000.0


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--n", type=int, default=2 ** 24)
    ap.add_argument("--clumps", type=int, default=4096)
    ap.add_argument("--k", type=int, default=16)
    ap.add_argument("--alpha", type=float, default=0.2)
    ap.add_argument("--seed", type=int, default=2)
    ap.add_argument("--period", type=float, default=0.0,
                    help="step mode: > 0 runs in the periodic cube [0, period)^3 (minimum image)")
    ap.add_argument("--leaf-max", type=int, default=0,
                    help="step mode: most points per leaf (0: the library default)")
    ap.add_argument("--coarsen", type=int, default=0,
                    help="step mode: node growth per plane (0: 16 with kNN and FoF concurrent, "
                         "the library default with --serial)")
    ap.add_argument("--n-target", type=int, default=0,
                    help="step mode: plane stop rule's node count (0: the library default)")
    ap.add_argument("--ngr", type=int, default=0,
                    help="step mode: top nodes per super node (0: the library default)")
    ap.add_argument("--key-bits", type=int, default=0,
                    help="step mode: Morton key bits per dimension (0: the library default)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--serial", action="store_true",
                    help="step mode: jz_knn then jz_fof instead of jz_knn_fof (the two concurrent)")
    ap.add_argument("--cpu-threads", type=int, default=0)
    ap.add_argument("--traffic-json", default=os.path.join(ROOT, "profiles", "leaf_knn_traffic.json"),
                    help="HBM bytes per launch of the dominant kernel from rocprofv3 counters")
    ap.add_argument("--mode", choices=["step", "batched", "served", "copycal"], default="step",
                    help="step: N=2^24 kNN+FoF (default); batched: many sets in one forest vs "
                         "per-set launches; served: Poisson request stream")
    ap.add_argument("--sets", type=int, default=4096, help="batched: number of sets")
    ap.add_argument("--rate", type=float, default=2000.0, help="served: requests per second")
    ap.add_argument("--duration", type=float, default=30.0,
                    help="served: measured seconds of arrivals (after the warm-up)")
    ap.add_argument("--measure-after", type=float, default=5.0,
                    help="served: seconds of warm-up arrivals before the measured ones")
    ap.add_argument("--streams", type=int, default=4, help="served: server worker streams")
    return ap.parse_args()


def main():
    args = parse()
    if args.gpus != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path "
              "(run with --gpus 1)", file=sys.stderr)
        sys.exit(2)
    if args.mode == "batched":
        return batched(args)
    if args.mode == "served":
        return served(args)
    if args.mode == "copycal":
        return copycal(args)
    import numpy as np
    import torch

    from paper_2604_05885_amd import api, inputs

    torch.cuda.set_device(0)
    n, k = args.n, args.k
    t0 = time.time()
    pts, info = inputs.clustered(n, args.clumps, args.seed, return_info=True)
    b = inputs.linking_length(n, args.alpha)
    print("# generated n=%d in %.1fs (max clump %d)" % (n, time.time() - t0, info["max_clump"]),
          file=sys.stderr, flush=True)
    dev = torch.from_numpy(pts).cuda()
    idx = torch.empty((n, k), dtype=torch.int32, device="cuda")
    d2 = torch.empty((n, k), dtype=torch.float32, device="cuda")
    lab = torch.empty(n, dtype=torch.int32, device="cuda")
    stream = torch.cuda.current_stream()
    kw = {}
    if args.period > 0:
        kw["period"] = args.period
    if args.key_bits > 0:
        kw["key_bits"] = args.key_bits
    if args.leaf_max > 0:
        kw["leaf_max"] = args.leaf_max
    if args.coarsen > 0:
        kw["coarsen"] = args.coarsen
    elif not args.serial:
        # node growth 16 per plane (three planes at 2^24 instead of four):
        # with the two halves concurrent, the shorter kNN walk leaves the FoF
        # half's tail to overlap the leaf kNN; one after the other, the
        # library's default of 8 is the faster
        kw["coarsen"] = 16
    if args.n_target > 0:
        kw["n_target"] = args.n_target
    if args.ngr > 0:
        kw["ngr"] = args.ngr
    opts = api.default_opts(**kw) if kw else None

    def step(ev=None):
        if ev is not None:
            ev[0].record(stream)
        t = api.jz_build(dev, opts, stream=stream)
        if ev is not None:
            ev[1].record(stream)
        if args.serial:
            t.knn(k, idx, d2, stream=stream)
            sk = t.stats()
            if ev is not None:
                ev[2].record(stream)
            t.fof(b, lab, stream=stream)
            sf = t.stats()
        else:
            # the two halves run concurrently (FoF on the library's second stream)
            t.knn_fof(k, b, idx, d2, lab, stream=stream)
            sk, sf = t.last_stats
            if ev is not None:
                ev[2].record(stream)
        if ev is not None:
            ev[3].record(stream)
        t.free()
        return sk, sf

    for i in range(args.warmup):
        step()
        print("# warmup %d done" % i, file=sys.stderr, flush=True)
    api.jz_set_profiling(True)
    evs = [[torch.cuda.Event(enable_timing=True) for _ in range(4)] for _ in range(args.steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    per = []
    for i in range(args.steps):
        per.append(step(evs[i]))
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    api.jz_set_profiling(False)

    build_ms = [e[0].elapsed_time(e[1]) for e in evs]
    knn_fof_ms = [e[1].elapsed_time(e[3]) for e in evs]
    # each half's own device time (in the concurrent schedule the two overlap)
    knn_ms = [sk["total_ms"] for sk, _ in per]
    fof_ms = [sf["total_ms"] for _, sf in per]
    leaf_ms = [sk["leaf_ms"] for sk, _ in per]
    sk, sf = per[-1]
    evals = sk["evaluations"]
    leaf_avg = float(np.mean(leaf_ms))
    achieved = evals * FLOPS_PER_EVAL / (leaf_avg * 1e-3) / 1e12
    traffic = None
    if os.path.exists(args.traffic_json):
        with open(args.traffic_json) as f:
            tj = json.load(f)
        # counters count only while the kernel source they were taken on is unchanged
        if tj.get("workload") == "clustered-2^24-k16" and tj.get("kernel_hash") == kernel_hash():
            traffic = tj.get("bytes_per_launch")

    value = n * args.steps / elapsed
    out = {
        "metric": "kNN(k=16)+FoF points/s at N=2^24 on 1 GPU",
        "value": value,
        "unit": "points/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": elapsed / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "clustered N=2^24 f32 in [0,1)^3, 60%% in %d Gaussian clumps "
                               "(sigma 0.002-0.02, counts ~ w^-1.9) + 40%% uniform; "
                               "kNN k=%d + FoF b=%.4g (alpha=%g)" % (args.clumps, k, b, args.alpha),
                   "n": n, "k": k, "b": b, "seed": args.seed, "max_clump": info["max_clump"],
                   "period": args.period},
        "roofline": {"bound": "alu", "kernel": "k_leaf_knn<16>", "achieved": achieved,
                     "peak": VALU_PEAK_TFLOPS, "unit": "TFLOP/s", "frac": achieved / VALU_PEAK_TFLOPS,
                     "traffic": traffic, "evaluations": evals, "flops_per_eval": FLOPS_PER_EVAL,
                     "leaf_ms": leaf_avg},
        "breakdown": {"schedule": "serial" if args.serial else "kNN and FoF concurrent",
                      "tree_opts": {f: getattr(opts if opts is not None else api.default_opts(), f)
                                    for f in ("leaf_max", "coarsen", "n_target", "ngr", "key_bits")},
                      "build_ms": float(np.median(build_ms)),
                      "knn_fof_ms": float(np.median(knn_fof_ms)), "knn_ms": float(np.median(knn_ms)),
                      "fof_ms": float(np.median(fof_ms)), "knn_leaf_ms": leaf_avg,
                      "fof_leaf_ms": float(np.mean([s["leaf_ms"] for _, s in per])),
                      "knn_stats": sk, "fof_stats": sf},
    }
    if args.period > 0:
        out["config"]["workload"] += "; periodic cube of side %g (minimum image)" % args.period
    if not args.no_cpu_baseline and args.period == 0:
        import oracle
        threads = args.cpu_threads or oracle.default_threads()
        t0 = time.perf_counter()
        oi, od = oracle.knn_kd(pts, k, threads=threads)
        t1 = time.perf_counter()
        ol = oracle.fof_kd(pts, b, threads=threads)
        t2 = time.perf_counter()
        # the timed GPU result of the last step against the oracle: every kNN
        # row and every label
        gi, gd, gl = idx.cpu().numpy(), d2.cpu().numpy(), lab.cpu().numpy()
        ok = bool(np.array_equal(gi, oi) and np.array_equal(gd.view(np.uint32), od.view(np.uint32))
                  and np.array_equal(gl, ol))
        out["cpu_baseline"] = {"value": n / (t2 - t0), "unit": "points/s", "cores": threads,
                               "kind": "oracle",
                               "sample": "the full benchmark set (N=2^24): exact kd-tree kNN k=%d "
                                         "(%.1fs) + FoF (%.1fs)" % (k, t1 - t0, t2 - t1),
                               "gpu_matches_oracle": ok}
        # binary64 cross-check of the same result (a report, not a gate):
        # sampled kNN rows re-ranked in binary64, every FoF pair's decision
        rows = np.random.default_rng(0).choice(n, 4096, replace=False)
        flips = oracle.knn_f64_report(pts, gi[rows], rows=rows, threads=threads)
        rep = oracle.fof_f64_report(pts, b, labels=gl, threads=threads)
        out["fp64_report"] = {"knn_rows_checked": int(rows.size),
                              "knn_rows_flipped": int(flips.size),
                              "fof_pairs_f32_only": rep["pairs_f32_only"],
                              "fof_pairs_f64_only": rep["pairs_f64_only"],
                              "fof_partition_differs": rep["partition_differs"],
                              "fof_points_relabelled": rep["points_relabelled"]}
    print(json.dumps(out), flush=True)


KERNEL_SOURCES = ("knn.hip", "jz_device.h")  # the leaf-kNN kernel and the device helpers it inlines


def kernel_hash() -> str:
    """sha256 over the leaf-kNN kernel's source files (ties traffic counters to
    a kernel version)."""
    import hashlib
    h = hashlib.sha256()
    for name in KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_2604_05885_amd", "csrc", name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def copycal(args):
    """Plain device copy of a known size, for scaling rocprofv3 FETCH_SIZE /
    WRITE_SIZE readings to bytes (run under rocprofv3 --pmc)."""
    import torch
    nbytes = 1 << 30
    src = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(3):
        dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"mode": "copycal", "bytes_read_per_copy": nbytes,
                      "bytes_written_per_copy": nbytes, "copies": 3}), flush=True)


def batched(args):
    """Many independent clustered sets (N per set log-uniform in [2^10, 2^18]),
    kNN k=16 + FoF with each set's own b: one forest (one sort and one launch
    per stage for all sets) against per-set jz_build + jz_knn + jz_fof."""
    import numpy as np
    import torch

    from paper_2604_05885_amd import api, inputs

    torch.cuda.set_device(0)
    t0 = time.time()
    pts, off, b = inputs.batched_sets(args.sets, seed=4)
    n = int(off[-1])
    print("# generated %d sets, %d points in %.1fs" % (args.sets, n, time.time() - t0),
          file=sys.stderr, flush=True)
    dev = torch.from_numpy(pts).cuda()
    k = args.k
    idx = torch.empty((n, k), dtype=torch.int32, device="cuda")
    d2 = torch.empty((n, k), dtype=torch.float32, device="cuda")
    lab = torch.empty(n, dtype=torch.int32, device="cuda")
    stream = torch.cuda.current_stream()

    t0 = time.time()
    opts, tuned_ms = api.jz_autotune(dev, off, k=k, b=b, stream=stream)
    print("# autotuned leaf_max=%d coarsen=%d (%.1f ms) in %.1fs" % (
        opts.leaf_max, opts.coarsen, tuned_ms, time.time() - t0), file=sys.stderr, flush=True)

    def forest():
        f = api.jz_forest_build(dev, off, opts, stream=stream)
        f.knn(k, idx, d2, stream=stream)
        f.fof(b, lab, stream=stream)
        st = f.stats()
        f.free()
        return st

    for _ in range(args.warmup):
        forest()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        st = forest()
    torch.cuda.synchronize()
    t_batched = (time.perf_counter() - t0) / args.steps
    bi, bd, bl = idx.clone(), d2.clone(), lab.clone()

    def plain(limit=None):
        for s in range(args.sets if limit is None else limit):
            a, e = int(off[s]), int(off[s + 1])
            if e == a:
                continue
            t = api.jz_build(dev[a:e], stream=stream)
            t.knn(k, idx[a:e], d2[a:e], stream=stream)
            t.fof(float(b[s]), lab[a:e], stream=stream)
            t.free()

    plain(min(args.sets, 64))  # warm-up
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    plain()
    torch.cuda.synchronize()
    t_plain = time.perf_counter() - t0
    same = bool(torch.equal(bi, idx) and torch.equal(bd.view(torch.int32), d2.view(torch.int32))
                and torch.equal(bl, lab))
    out = {
        "metric": "batched kNN(k=16)+FoF solves/s (sets solved per second)",
        "value": args.sets / t_batched,
        "unit": "solves/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": t_batched * 1e3, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": "%d clustered sets, N per set log-uniform in [2^10, 2^18] "
                               "(total %d points), kNN k=%d + FoF b=fl32(0.2 N_s^-1/3) per set"
                               % (args.sets, n, k), "sets": args.sets, "points": n},
        "plain_solves_per_s": args.sets / t_plain,
        "speedup_vs_plain": t_plain / t_batched,
        "points_per_s": n / t_batched,
        "identical_to_plain": same,
        "forest_stats": {kk: v for kk, v in st.items() if kk in ("planes", "nodes", "super_nodes")},
        "autotuned": {"leaf_max": opts.leaf_max, "coarsen": opts.coarsen,
                      "n_target": opts.n_target, "ngr": opts.ngr},
    }
    print(json.dumps(out), flush=True)


def served(args):
    """Open-loop Poisson stream of kNN / FoF requests (k in {8,16,32}, alpha in
    {0.1,0.2}, N log-uniform in [2^12, 2^22]) through the continuous-batching
    server. Every request gets a fresh clustered set drawn on the GPU from its
    own seed (on the client's stream, right before submission: the server
    orders the request after it). Latency = completion - scheduled arrival, so
    queueing and any client delay count. Reported beside it: the same stream
    at 60% of the rate, and per-request plain launches (FIFO, one at a time)
    run back to back on the same request mix."""
    import threading

    import numpy as np
    import torch

    from paper_2604_05885_amd import api, inputs

    torch.cuda.set_device(0)
    client = torch.cuda.Stream()

    def params(reqs):
        """Per-request clump parameters, drawn on the host and uploaded once,
        before the clock starts."""
        cs, ss, ns, spans = [], [], [], []
        c0 = 0
        for r in reqs:
            n_cl, cen, sig, cnt = inputs.clump_params(r["n"], r["clumps"], r["seed"])
            cs.append(cen)
            ss.append(sig)
            ns.append(cnt)
            spans.append((c0, c0 + len(sig), n_cl))
            c0 += len(sig)
        dev = lambda a, t: torch.from_numpy(np.concatenate(a)).to("cuda", t)
        return dev(cs, torch.float64), dev(ss, torch.float64), dev(ns, torch.int64), spans

    def make(r, prm, i):
        cen, sig, cnt, spans = prm
        a, b, n_cl = spans[i]
        with torch.cuda.stream(client):
            p = inputs.clustered_device(r["n"], r["seed"], n_cl, cen[a:b], sig[a:b], cnt[a:b])
            if r["op"] == "knn":
                out = (torch.empty((r["n"], r["k"]), dtype=torch.int32, device="cuda"),
                       torch.empty((r["n"], r["k"]), dtype=torch.float32, device="cuda"))
            else:
                out = (torch.empty(r["n"], dtype=torch.int32, device="cuda"),)
        return p, out

    def submit(S, r, p, out):
        with torch.cuda.stream(client):
            if r["op"] == "knn":
                return S.submit_knn(p, r["k"], *out)
            return S.submit_fof(p, inputs.linking_length(r["n"], r["alpha"]), *out)

    def run_open(rate, warm, measure, seed):
        reqs = inputs.served_requests(int(rate * (warm + measure)), seed=seed, rate_hz=rate)
        prm = params(reqs)
        S = api.Server(streams=args.streams, max_batch_sets=4096, hbm_budget=int(200e9))
        for i, r in enumerate(reqs[:16]):  # warm the library (kernels, pool, list sizes)
            p, out = make(r, prm, i)
            S.wait(submit(S, r, p, out))
        torch.cuda.synchronize()
        done = []          # (ticket, due_ns, request)
        results = {}
        lock = threading.Condition()
        state = {"n_sub": 0, "stop": False, "collected": 0}
        aborted = False

        def collector():
            i = 0
            while True:
                state["collected"] = i
                with lock:
                    while i >= state["n_sub"] and not state["stop"]:
                        lock.wait()
                    if i >= state["n_sub"]:
                        return
                    tk, due, r = done[i]
                try:
                    _, t_done = S.wait(tk)
                    results[i] = (t_done, None)
                except api.JzError as e:
                    results[i] = (None, str(e))
                S.release(tk)
                i += 1

        th = threading.Thread(target=collector)
        th.start()
        t0 = api.now_ns() + int(0.05e9)
        late_max = 0.0
        backlog = []
        for i, r in enumerate(reqs):
            due = t0 + int(r["t"] * 1e9)
            while api.now_ns() < due:
                pass
            late_max = max(late_max, (api.now_ns() - due) / 1e6)
            if state["n_sub"] - state["collected"] > 2000:
                # more than a second of arrivals outstanding: the device does
                # not keep up; stop before their buffers exhaust memory
                aborted = True
                break
            p, out = make(r, prm, i)
            tk = submit(S, r, p, out)
            with lock:
                done.append((tk, due, r))
                state["n_sub"] += 1
                lock.notify()
            if len(done) % 500 == 0:
                backlog.append((r["t"], S.stats()["pending"]))
        with lock:
            state["stop"] = True
            lock.notify()
        th.join()
        st = S.stats()
        S.close()
        lat, npts, first_due, last_done, failed, err = [], 0, None, 0, 0, None
        for i, (tk, due, r) in enumerate(done):
            t_done, e = results[i]
            if e is not None:
                failed += 1
                err = err or e
                continue
            if r["t"] >= warm:
                lat.append((t_done - due) / 1e6)
                npts += r["n"]
                first_due = due if first_due is None else min(first_due, due)
                last_done = max(last_done, t_done)
        lat = np.array(lat)
        span = (last_done - first_due) / 1e9
        half = [b for t, b in backlog if t >= warm]
        return {"offered_req_per_s": rate, "solves_per_s": len(lat) / span,
                "points_per_s": npts / span, "p50_ms": float(np.percentile(lat, 50)),
                "p99_ms": float(np.percentile(lat, 99)), "requests": int(len(lat)),
                "batches": st["batches"], "max_batch": st["max_batch_sets_seen"],
                "failed": failed, "first_error": err, "client_late_max_ms": late_max,
                "pending_first_half_max": int(max(half[:len(half) // 2] or [0])),
                "pending_second_half_max": int(max(half[len(half) // 2:] or [0])),
                "aborted_backlog": aborted,
                "sustained": bool(not aborted and len(lat) / span >= 0.97 * rate)}

    def run_fifo(count, seed):
        """Per-request plain launches (build + kNN / FoF), one at a time on
        one stream, back to back: the device time of the same mix without
        batching or overlap."""
        reqs = inputs.served_requests(count, seed=seed, rate_hz=2000.0)
        prm = params(reqs)
        stream = torch.cuda.current_stream()
        total_t, npts = 0.0, 0
        for i, r in enumerate(reqs):
            p, out = make(r, prm, i)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            t = api.jz_build(p, stream=stream)
            if r["op"] == "knn":
                t.knn(r["k"], *out, stream=stream)
            else:
                t.fof(inputs.linking_length(r["n"], r["alpha"]), *out, stream=stream)
            t.free()
            total_t += time.perf_counter() - t0
            npts += r["n"]
        return {"solves_per_s": count / total_t, "points_per_s": npts / total_t,
                "requests": count}

    cont = run_open(args.rate, args.measure_after, args.duration, seed=5)
    print("# continuous batching done", file=sys.stderr, flush=True)
    light = run_open(0.6 * args.rate, 2.0, 10.0, seed=7)
    print("# 60%% load done", file=sys.stderr, flush=True)
    fifo = run_fifo(1000, seed=9)
    out = {
        "metric": "served kNN/FoF solves/s with p50/p99 latency (open-loop Poisson arrivals)",
        "value": cont["solves_per_s"], "unit": "solves/s", "n_gpus": 1,
        "steps": cont["requests"], "warmup": 0, "ms_per_step": None, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": "Poisson %g req/s for %gs after %gs warm-up; each request kNN "
                               "(k in {8,16,32}) or FoF (alpha in {0.1,0.2}) on a fresh clustered "
                               "set drawn on the GPU from its own seed, N log-uniform in "
                               "[2^12, 2^22]; HBM budget 200 GB"
                               % (args.rate, args.duration, args.measure_after)},
        "continuous_batching": cont,
        "continuous_batching_at_60pct": light,
        "per_request_fifo_back_to_back": fifo,
        "speedup_vs_fifo": cont["solves_per_s"] / fifo["solves_per_s"],
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
