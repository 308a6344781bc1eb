"""Benchmark: exact kNN (k=16) + FoF (b = 0.2 x mean spacing) at N = 2^24 on one GPU.

One step = jz_build (z-order sort + tree planes) + jz_knn(k) + jz_fof(b) +
jz_tree_free on a clustered synthetic point set already resident in HBM
(60% of points in 4096 Gaussian clumps, 40% uniform background; the stand-in
for the paper's cosmological snapshots). Prints one JSON line.

value = N * steps / (wall time of the timed steps)  [points/s]

The line also carries:
  roofline     the dominant kernel (leaf-stage kNN), timed with HIP events on
               the stream it runs on, against the FP32 VALU rate for plain
               (non-fused, non-packed) add/mul: 256 CU * 64 lanes * 2.4 GHz
  cpu_baseline the CPU oracle (exact kd-tree kNN + FoF) on the host cores
  breakdown    per-call device times (build / knn / fof) and walk statistics
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
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-threads", type=int, default=0)
    ap.add_argument("--traffic-json", default=os.path.join(ROOT, "profiles", "leaf_knn_traffic.json"),
                    help="HBM bytes per launch of the dominant kernel from rocprofv3 counters")
    ap.add_argument("--mode", choices=["step", "batched", "served", "copycal"], default="step",
                    help="step: N=2^24 kNN+FoF (default); batched: many sets in one forest vs "
                         "per-set launches; served: Poisson request stream")
    ap.add_argument("--sets", type=int, default=4096, help="batched: number of sets")
    ap.add_argument("--rate", type=float, default=2000.0, help="served: requests per second")
    ap.add_argument("--duration", type=float, default=10.0, help="served: seconds of arrivals")
    ap.add_argument("--measure-after", type=float, default=2.0,
                    help="served: arrivals before this time (s) are warm-up")
    ap.add_argument("--pool", type=int, default=64, help="served: distinct point sets")
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

    def step(ev=None):
        if ev is not None:
            ev[0].record(stream)
        t = api.jz_build(dev, stream=stream)
        if ev is not None:
            ev[1].record(stream)
        t.knn(k, idx, d2, stream=stream)
        sk = t.stats()
        if ev is not None:
            ev[2].record(stream)
        t.fof(b, lab, stream=stream)
        sf = t.stats()
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
    knn_ms = [e[1].elapsed_time(e[2]) for e in evs]
    fof_ms = [e[2].elapsed_time(e[3]) for e in evs]
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
                   "n": n, "k": k, "b": b, "seed": args.seed, "max_clump": info["max_clump"]},
        "roofline": {"bound": "alu", "kernel": "k_leaf_knn<16>", "achieved": achieved,
                     "peak": VALU_PEAK_TFLOPS, "unit": "TFLOP/s", "frac": achieved / VALU_PEAK_TFLOPS,
                     "traffic": traffic, "evaluations": evals, "flops_per_eval": FLOPS_PER_EVAL,
                     "leaf_ms": leaf_avg},
        "breakdown": {"build_ms": float(np.median(build_ms)), "knn_ms": float(np.median(knn_ms)),
                      "fof_ms": float(np.median(fof_ms)), "knn_leaf_ms": leaf_avg,
                      "fof_leaf_ms": float(np.mean([s["leaf_ms"] for _, s in per])),
                      "knn_stats": sk, "fof_stats": sf},
    }
    if not args.no_cpu_baseline:
        import oracle
        threads = args.cpu_threads or oracle.default_threads()
        t0 = time.perf_counter()
        oi, od = oracle.knn_kd(pts, k, threads=threads)
        t1 = time.perf_counter()
        ol = oracle.fof_kd(pts, b, threads=threads)
        t2 = time.perf_counter()
        # the timed GPU result of the last step, checked on a sample of rows
        gi = idx.cpu().numpy()
        rows = np.random.default_rng(0).choice(n, 4096, replace=False)
        ok = bool(np.array_equal(gi[rows], oi[rows]) and
                  np.array_equal(lab.cpu().numpy(), ol))
        out["cpu_baseline"] = {"value": n / (t2 - t0), "unit": "points/s", "cores": threads,
                               "kind": "oracle",
                               "sample": "the full benchmark set (N=2^24): exact kd-tree kNN k=%d "
                                         "(%.1fs) + FoF (%.1fs)" % (k, t1 - t0, t2 - t1),
                               "gpu_matches_oracle": ok}
    print(json.dumps(out), flush=True)


def kernel_hash() -> str:
    """sha256 of the leaf-kNN source file (ties traffic counters to a kernel version)."""
    import hashlib
    with open(os.path.join(ROOT, "paper_2604_05885_amd", "csrc", "knn.hip"), "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()[:16]


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
        "autotuned": {"leaf_max": opts.leaf_max, "coarsen": opts.coarsen},
    }
    print(json.dumps(out), flush=True)


def served(args):
    """Open-loop Poisson stream of kNN / FoF requests (k in {8,16,32}, alpha in
    {0.1,0.2}, N log-uniform in [2^12, 2^22]) through the continuous-batching
    server, against the same stream through per-request launches (one request
    per batch, one worker). Latency = completion - scheduled arrival."""
    import numpy as np
    import torch

    from paper_2604_05885_amd import api, inputs

    torch.cuda.set_device(0)
    rng = np.random.default_rng(5)
    t0 = time.time()
    pool = []
    for i in range(args.pool):
        nn = int(np.floor(2.0 ** rng.uniform(12, 22)))
        p = inputs.clustered(nn, max(1, int(round(4096 * nn / 2.0 ** 24))), seed=5_000_000 + i)
        pool.append(torch.from_numpy(p).cuda())
    outs = [{kk: (torch.empty((q.shape[0], kk), dtype=torch.int32, device="cuda"),
                  torch.empty((q.shape[0], kk), dtype=torch.float32, device="cuda"))
             for kk in (8, 16, 32)} for q in pool]
    labs = [torch.empty(q.shape[0], dtype=torch.int32, device="cuda") for q in pool]
    torch.cuda.synchronize()
    print("# pool of %d sets (%d points) in %.1fs" % (args.pool, sum(q.shape[0] for q in pool),
                                                      time.time() - t0), file=sys.stderr, flush=True)
    def schedule(rate, duration, seed):
        rs = inputs.served_requests(int(rate * duration), seed=seed, rate_hz=rate)
        pick = np.random.default_rng(seed + 1)
        for r in rs:
            r["set"] = int(pick.integers(args.pool))
        return rs

    reqs = schedule(args.rate, args.duration, 5)

    def run(streams, max_sets, reqs=reqs, measure_after=args.measure_after):
        S = api.Server(streams=streams, max_batch_sets=max_sets, hbm_budget=int(200e9))
        # warm the library (kernels, pool, learned list sizes)
        for q, o, l in zip(pool[:8], outs[:8], labs[:8]):
            S.wait(S.submit_knn(q, 16, *o[16]))
            S.wait(S.submit_fof(q, inputs.linking_length(q.shape[0]), l))
        t_start = api.now_ns() + int(0.05e9)
        tickets = []
        for r in reqs:
            due = t_start + int(r["t"] * 1e9)
            while api.now_ns() < due:
                pass
            q = pool[r["set"]]
            if r["op"] == "knn":
                tk = S.submit_knn(q, r["k"], *outs[r["set"]][r["k"]])
            else:
                tk = S.submit_fof(q, inputs.linking_length(q.shape[0], r["alpha"]),
                                  labs[r["set"]])
            tickets.append((tk, due, r))
        lat, last_done, first_due, npts = [], 0, None, 0
        failed, first_error = 0, None
        for tk, due, r in tickets:
            try:
                _, done_ns = S.wait(tk)
            except api.JzError as e:  # reported, not hidden: a failed request is a bug
                failed += 1
                first_error = first_error or str(e)
                S.release(tk)
                continue
            S.release(tk)
            if r["t"] >= measure_after:
                lat.append((done_ns - due) / 1e6)
                last_done = max(last_done, done_ns)
                first_due = due if first_due is None else min(first_due, due)
                npts += pool[r["set"]].shape[0]
        st = S.stats()
        S.close()
        lat = np.array(lat)
        span = (last_done - first_due) / 1e9
        return {"solves_per_s": len(lat) / span, "points_per_s": npts / span,
                "p50_ms": float(np.percentile(lat, 50)), "p99_ms": float(np.percentile(lat, 99)),
                "requests": len(lat), "batches": st["batches"],
                "max_batch": st["max_batch_sets_seen"], "failed": failed,
                "first_error": first_error}

    cont = run(args.streams, 4096)
    fifo = run(1, 1)
    # When the offered rate exceeds what the device sustains, the queue grows
    # for the whole run and p50/p99 measure that backlog; so the server is
    # also run at 60% of the solves/s it sustained, where latency is service
    # time plus batching delay.
    light_rate = 0.6 * cont["solves_per_s"]
    light = run(args.streams, 4096, reqs=schedule(light_rate, 6.0, 7), measure_after=1.0)
    light["offered_req_per_s"] = light_rate
    out = {
        "metric": "served kNN/FoF solves/s with p50/p99 latency (open-loop Poisson arrivals)",
        "value": cont["solves_per_s"], "unit": "solves/s", "n_gpus": 1,
        "steps": len(reqs), "warmup": 0, "ms_per_step": None, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": "Poisson %g req/s for %gs (first %gs warm-up); each request kNN "
                               "(k in {8,16,32}) or FoF (alpha in {0.1,0.2}) on one of %d clustered "
                               "sets with N log-uniform in [2^12, 2^22]; HBM budget 200 GB"
                               % (args.rate, args.duration, args.measure_after, args.pool)},
        "continuous_batching": cont,
        "per_request_fifo": fifo,
        "continuous_batching_at_60pct_of_sustained": light,
        "speedup_vs_fifo": cont["solves_per_s"] / fifo["solves_per_s"],
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
