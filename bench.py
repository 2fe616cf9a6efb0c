#!/usr/bin/env python3
"""Benchmark of the DFacTo hot path on one MI355X.

Workload (default, ``paper1200m``): the paper-shape tensor, 6,500,000 x
2,500,000 x 1,500,000 with 1.2B distinct coordinates, Zipf(1.2) per mode over
seeded permutations (drawn and deduplicated on the device), |N(0,1)| FP32
values; rank R = 32 with FP32 factors initialized U(0,1).  The same run
measures R = 32 with BF16-stored factors and R = 10 (FP32 and BF16) beside
it.  ``--workload zipf50m`` runs the 1M x 500K x 200K, 50M-nonzero Zipf(1.1)
tensor instead.

One step = --als-per-step CP-ALS iterations (each three MTTKRPs with the
FP64 Gram / solve / normalize epilogue and the fit; default 1 for the paper
shape, 10 for zipf50m) followed by one GD gradient at the resulting point
(three more MTTKRPs, gradients and the objective).  ``value`` is the step's
MTTKRP throughput, MTTKRPs per step * nnz * R / step time, in nnz*R/s, with
the tensor resident in HBM.  The flattenings are built once, before the
timed region (as the paper's per-iteration times also exclude it); the build
time is reported separately.

Prints ONE JSON line (see --help for options).
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "MTTKRP nnz·R/s + % HBM peak; CP-ALS iter time; served solves/s, p50/p99"
HBM_PEAK_GBS = 8000.0
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "mttkrp_{}_traffic.json")
KERNEL_SRC = os.path.join(ROOT, "paper_1406_4519_amd", "csrc", "mttkrp.hip")


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def kernel_hash() -> str:
    with open(KERNEL_SRC, "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()[:16]


def load_traffic(workload: str):
    """HBM bytes per launch from the committed rocprofv3 counter summary of
    the workload, or None when there is none or the kernel source changed
    since the counters were taken."""
    try:
        with open(TRAFFIC_FILE.format(workload)) as f:
            d = json.load(f)
    except (OSError, ValueError):
        return None
    if d.get("kernel_sha256_16") != kernel_hash():
        return None
    return d.get("traffic_bytes_per_launch")


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(sample, dims, R, F0, target_s: float, threads: int):
    """Time the FP64 oracle's MTTKRP (its loop as it stands, over `threads`
    row-partitioned workers whose results are bitwise those of one) for the
    three modes on the first S of the sampled nonzeros, with the full-size
    factors; S grows until the run takes about target_s.  Returns the
    line's cpu_baseline dict (unit nnz*R/s, the metric's)."""
    import numpy as np
    import oracle
    oracle.build()
    i_all, j_all, k_all, v_all = sample
    oracle.config(threads, assume_distinct=True)
    try:
        S = min(len(v_all), 1_000_000)
        while True:
            i, j, k = i_all[:S], j_all[:S], k_all[:S]
            v = v_all[:S].astype(np.float64)
            t0 = time.perf_counter()
            for m in range(3):
                oracle.mttkrp(i, j, k, v, dims, F0, m)
            dt = time.perf_counter() - t0
            if dt >= target_s * 0.5 or S >= len(v_all):
                break
            S = min(len(v_all), int(S * min(8.0, target_s / max(dt, 1e-3))))
    finally:
        oracle.config(1, False)
    return {"value": 3.0 * S * R / dt, "unit": "nnz·R/s", "cores": threads, "kind": "oracle",
            "seconds": round(dt, 3), "cpu_model": cpu_model(),
            "sample": f"oracle MTTKRP, all three modes (FP64, {threads} "
                      f"thread{'s' if threads > 1 else ''}, output rows split by nonzero count), "
                      f"on {S:,} seeded random nonzeros of the tensor with its full-size "
                      f"factors, R={R}"}


def run_batched(args):
    """Batched CP-ALS: args.batch independent Zipf(1.1) tensors (dims
    log-uniform in [1e3, 1e5] per mode, nnz log-uniform in [1e4, 5e6], R from
    {8, 16, 32}), args.iters ALS iterations each, run as one group (grouped
    launches, tuned MTTKRP grids) and, for comparison, one tensor at a time
    through dfacto_als_iter.  value = grouped throughput, sum over tensors of
    3 nnz R per iteration, per second."""
    import numpy as np
    import torch
    from paper_1406_4519_amd import dfacto, gen

    dev = torch.device("cuda:0")
    ctx = dfacto.Context(0)
    t0 = time.perf_counter()
    staged = []
    for t in range(args.batch):
        coo, R, F0 = gen.batched_tensor(t)
        d = [torch.from_numpy(a.view(np.int32)).to(dev) for a in (coo.i, coo.j, coo.k)]
        staged.append((coo.dims, d + [torch.from_numpy(coo.val).to(dev)], R, F0, coo.nnz))
    torch.cuda.synchronize()
    log(f"generated {args.batch} tensors in {time.perf_counter() - t0:.1f}s")
    # the builds from device-resident COO, timed on their own: build_threads
    # host threads, each with a context on a stream of its own (a build
    # waits for its stream at the end; the library call releases the GIL)
    from concurrent.futures import ThreadPoolExecutor
    nth = max(1, args.build_threads)
    bctx = [dfacto.Context(0, stream=torch.cuda.Stream()) for _ in range(nth)]
    torch.cuda.synchronize()
    tb = time.perf_counter()

    def build_slice(w):
        return [(q, dfacto.build_flattenings(bctx[w], staged[q][0], *staged[q][1]))
                for q in range(w, len(staged), nth)]

    with ThreadPoolExecutor(nth) as ex:
        built = dict(kv for part in ex.map(build_slice, range(nth)) for kv in part)
    torch.cuda.synchronize()
    build_s = time.perf_counter() - tb
    members = [(built[q], R, F0, nnz, dims) for q, (dims, d, R, F0, nnz) in enumerate(staged)]
    del staged
    log(f"built {args.batch} tensors in {build_s:.3f}s")
    work = sum(3.0 * nnz * R for _, R, _, nnz, _ in members) * args.iters
    total_nnz = sum(nnz for _, _, _, nnz, _ in members)

    def fresh(dtype_name):
        tdt = torch.float32 if dtype_name == "f32" else torch.bfloat16
        Fs = [[torch.from_numpy(np.ascontiguousarray(f, dtype=np.float32)).to(dev).to(tdt)
               for f in F0] for _, _, F0, _, _ in members]
        lams = [torch.zeros(R, dtype=torch.float64, device=dev) for _, R, _, _, _ in members]
        return Fs, lams, torch.zeros(len(members), dtype=torch.float64, device=dev)

    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    res = {}
    for dt in ("f32", "bf16"):
        Fs, lams, fits = fresh(dt)
        start = [[f.clone() for f in F] for F in Fs]
        tc = time.perf_counter()
        g = dfacto.Group(ctx, [m[0] for m in members], Fs, lams, fits, tune=True, graph=True)
        create_s = time.perf_counter() - tc
        info = g.info()

        def timed():
            torch.cuda.synchronize()
            ts = time.perf_counter()
            e0.record()
            g.als(args.iters)
            e1.record()
            torch.cuda.synchronize()
            return e0.elapsed_time(e1), time.perf_counter() - ts

        # the first call captures the iteration graphs (end to end counts
        # it); the same iterations from the same start are then timed as
        # graph replays, and must give the same factors bit for bit
        first_ms, wall = timed()
        first = [[f.clone() for f in F] for F in Fs]
        for F, S in zip(Fs, start):
            for f, s0 in zip(F, S):
                f.copy_(s0)
        ms, _ = timed()
        same = all(torch.equal(a, b) for F, S in zip(Fs, first) for a, b in zip(F, S))
        res[dt] = dict(ms=ms, first_ms=first_ms, wall_s=wall, create_s=create_s, info=info,
                       replay_equals_first=same, mean_fit=float(fits.mean().item()))
        g.close()
        del Fs, lams, fits, start, first
    # one tensor at a time (FP32), same iterations
    Fs, lams, fits = fresh("f32")
    fit1 = torch.zeros(1, dtype=torch.float64, device=dev)
    torch.cuda.synchronize()
    ts = time.perf_counter()
    e0.record()
    for (T, R, _, _, _), F, lam in zip(members, Fs, lams):
        for _ in range(args.iters):
            dfacto.als_iter(ctx, T, F, lam, fit1)
    e1.record()
    torch.cuda.synchronize()
    seq_ms = e0.elapsed_time(e1)
    seq_wall = time.perf_counter() - ts
    g32 = res["f32"]
    line = {"metric": "grouped CP-ALS nnz·R/s (batched solves)",
            "value": work / (g32["ms"] * 1e-3), "unit": "nnz·R/s", "n_gpus": 1,
            "steps": args.iters, "warmup": args.iters, "ms_per_step": round(g32["ms"] / args.iters, 4),
            "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
            "data": "synthetic",
            "config": {"workload": f"batched: {args.batch} tensors, dims log-uniform [1e3,1e5], "
                                   f"nnz log-uniform [1e4,5e6], Zipf(1.1), R in {{8,16,32}}, "
                                   f"{args.iters} ALS iterations each",
                       "total_nnz": total_nnz, "parallelism": "single GPU"},
            "extra": {"solves_per_s_grouped_f32": args.batch / (g32["ms"] * 1e-3),
                      "build_s": round(build_s, 3), "build_threads": nth,
                      "solves_per_s_end_to_end_f32": args.batch / (build_s + g32["create_s"] +
                                                                   g32["wall_s"]),
                      "solves_per_s_grouped_bf16": args.batch / (res["bf16"]["ms"] * 1e-3),
                      "solves_per_s_one_at_a_time_f32": args.batch / (seq_ms * 1e-3),
                      "grouped_ms": {k: round(v["ms"], 3) for k, v in res.items()},
                      "grouped_first_call_ms": {k: round(v["first_ms"], 3) for k, v in res.items()},
                      "replay_equals_first": {k: v["replay_equals_first"] for k, v in res.items()},
                      "one_at_a_time_ms": round(seq_ms, 3),
                      "one_at_a_time_wall_s": round(seq_wall, 3),
                      "grouped_speedup_f32": round(seq_ms / g32["ms"], 3),
                      "bf16_value": work / (res["bf16"]["ms"] * 1e-3),
                      "group_create_s": {k: round(v["create_s"], 3) for k, v in res.items()},
                      "launches_per_iter": g32["info"]["launches_per_iter"],
                      "tuned_mttkrp_forms": {
                          k: [dict(cpl=c, lanes=l, chunks_per_group=q, grid=gr, of=nf)
                              for c, l, q, gr, nf in zip(v["info"]["mttkrp_cpl"],
                                                         v["info"]["mttkrp_lanes"],
                                                         v["info"]["mttkrp_chunks_per_group"],
                                                         v["info"]["mttkrp_grid"],
                                                         v["info"]["mttkrp_forms"])]
                          for k, v in res.items()},
                      "group_bytes": g32["info"]["bytes"],
                      "mean_fit": {k: v["mean_fit"] for k, v in res.items()}}}
    print(json.dumps(line), flush=True)
    for m in members:
        m[0].close()
    for c in bctx:
        c.close()
    ctx.close()


def _served_run(dfacto, np, pool, big, rate, n_warm, n_meas, dt, seed, large_frac):
    """One sustained-load run: n_warm + n_meas Poisson arrivals at `rate`
    per second (requests drawn from `pool`, a fraction large_frac of them
    `big`), submitted in real time; a collector thread waits for results in
    submission order and keeps only their timings (the factors are dropped
    as they arrive).  Latency = submission to factors in host memory."""
    import queue
    import threading
    rng = np.random.default_rng(seed)
    n = n_warm + n_meas
    arrivals = np.cumsum(rng.exponential(1.0 / rate, n))
    picks = [big if (big is not None and rng.random() < large_frac)
             else pool[int(rng.integers(len(pool)))] for _ in range(n)]
    srv = dfacto.Server(0, max_slots=64)
    q = queue.Queue()
    recs = [None] * n

    def collect():
        while True:
            item = q.get()
            if item is None:
                return
            idx, rid = item
            r = srv.wait(rid)
            recs[idx] = (r["status"], r["iters"], r["t_submit"], r["t_admit"], r["t_done"])

    th = threading.Thread(target=collect, daemon=True)
    th.start()
    start = time.perf_counter()
    for idx, (a, (coo, R, F0)) in enumerate(zip(arrivals, picks)):
        now = time.perf_counter() - start
        if a > now:
            time.sleep(a - now)
        q.put((idx, srv.submit(coo.dims, coo.i, coo.j, coo.k, coo.val, R, F0, dtype=dt,
                               tol=1e-4, max_iters=50)))
        if idx == n_warm - 1:
            log(f"    {dt} {rate:g}/s: warm-up submitted at {time.perf_counter() - start:.1f}s")
    submit_s = time.perf_counter() - start
    q.put(None)
    th.join()
    st = srv.stats()
    srv.close()
    meas = recs[n_warm:]
    lat = np.array([r[4] - r[2] for r in meas])
    t_first = min(r[2] for r in meas)
    t_last = max(r[4] for r in meas)
    served = n_meas / (t_last - t_first)
    offered = n_meas / (arrivals[-1] - arrivals[n_warm])
    qn = max(1, n_meas // 4)
    p50_first = float(np.median(lat[:qn]))
    p50_last = float(np.median(lat[-qn:]))
    # sustained: the device keeps up (served >= 95% of offered) and the
    # queue does not grow (the last quarter's median latency at most twice
    # the first quarter's, plus 50 ms)
    sustained = bool(served >= 0.95 * offered and p50_last <= 2.0 * p50_first + 0.05)
    big_lat = [r[4] - r[2] for r, p in zip(meas, picks[n_warm:]) if p is big]
    out = dict(offered_per_s=round(offered, 2), solves_per_s=round(served, 2),
               p50_ms=round(float(np.percentile(lat, 50)) * 1e3, 2),
               p99_ms=round(float(np.percentile(lat, 99)) * 1e3, 2),
               p50_first_quarter_ms=round(p50_first * 1e3, 2),
               p50_last_quarter_ms=round(p50_last * 1e3, 2), sustained=sustained,
               warmup_requests=n_warm, measured_requests=n_meas,
               mean_iters=round(float(np.mean([r[1] for r in meas])), 2),
               failed=int(sum(r[0] != dfacto.OK for r in recs)),
               peak_active=st["peak_active"], boundaries=st["iterations"],
               large_requests=len(big_lat),
               large_p50_ms=round(float(np.percentile(big_lat, 50)) * 1e3, 1) if big_lat else None,
               submit_span_s=round(submit_s, 2), span_s=round(t_last - t_first, 2),
               budget_gb=round(st["budget"] / 1e9, 1),
               worker_s={k: round(st[k], 3) for k in
                         ("t_admit", "t_build", "t_groups", "t_iterate", "t_deliver")})
    log(f"    {dt} {rate:g}/s: {out}")
    return out


def run_served(args):
    """Served CP-ALS under sustained load: Poisson arrivals at args.rate per
    second of solves drawn from the batched distribution plus args.large_frac
    of 50M-nonzero 1M x 500K x 200K requests, each run to a fit change below
    1e-4 or 50 iterations, admitted by device footprint and batched
    continuously.  args.served_warmup requests warm the server up, then
    args.served_requests are measured: completed solves per second over the
    measured requests' span, p50 / p99 latency (submission to factors in
    host memory) and whether the load was sustained.  With --rate-search,
    also the highest offered rate that is sustained (steps of 25/s, then
    two halvings of the interval), per storage dtype, on shorter runs."""
    import numpy as np
    from paper_1406_4519_amd import dfacto, gen

    if args.served_one is None:
        return _served_parent(args)
    t0 = time.perf_counter()
    pool = []
    for t in range(args.pool):
        coo, R, F0 = gen.batched_tensor(t)
        pool.append((coo, R, [f.astype(np.float32) for f in F0]))
    big = None
    if args.large_frac > 0:
        coo = gen.zipf_distinct((1_000_000, 500_000, 200_000), 50_000_000, 1.1, seed=7)
        Rb = 32
        big = (coo, Rb, [f.astype(np.float32) for f in gen.init_factors(coo.dims, Rb, seed=1007)])
    log(f"generated the request pool in {time.perf_counter() - t0:.1f}s")
    dt, rate, n_warm, n_meas, seed = args.served_one.split(",")
    out = _served_run(dfacto, np, pool, big, float(rate), int(n_warm), int(n_meas), dt, int(seed),
                      args.large_frac)
    print("SERVED_RUN " + json.dumps(out), flush=True)


def _served_child(args, dt, rate, n_warm, n_meas, seed):
    """One served run in a process of its own.  A server started in a
    process where another server has already run serves about 20-35% fewer
    solves per second (measured; reusing the first server's streams or its
    memory pool does not remove it), so every run starts from a fresh
    process and the runs compare on equal terms."""
    import subprocess
    cmd = [sys.executable, "-u", os.path.abspath(__file__), "--workload", "served",
           "--served-one", f"{dt},{rate},{n_warm},{n_meas},{seed}",
           "--large-frac", str(args.large_frac), "--pool", str(args.pool)]
    r = subprocess.run(cmd, stdout=subprocess.PIPE, text=True)
    lines = [ln for ln in r.stdout.splitlines() if ln.startswith("SERVED_RUN ")]
    if r.returncode != 0 or not lines:
        raise RuntimeError(f"served run {dt} at {rate:g}/s failed (exit {r.returncode})")
    return json.loads(lines[-1][len("SERVED_RUN "):])


def _served_parent(args):
    out = {}
    for dt in args.served_dtypes.split(","):
        log(f"  {dt}: {args.served_warmup} + {args.served_requests} requests at {args.rate:g}/s")
        out[dt] = _served_child(args, dt, args.rate, args.served_warmup, args.served_requests,
                                12345)
    search = {}
    if args.rate_search:
        for dt in args.served_dtypes.split(","):
            best, tried = None, []

            def probe(rate):
                r = _served_child(args, dt, rate, 100, args.search_requests, 777)
                tried.append(dict(rate=rate, solves_per_s=r["solves_per_s"],
                                  p50_ms=r["p50_ms"], p99_ms=r["p99_ms"],
                                  sustained=r["sustained"]))
                return r

            # steps of 25/s up to the first rate not sustained, then halving
            # the interval twice (6.25/s resolution)
            lo, hi, rate = None, None, 50.0
            while rate <= args.rate:
                r = probe(rate)
                if not r["sustained"]:
                    hi = rate
                    break
                lo = rate
                best = dict(rate=rate, **{k: r[k] for k in ("solves_per_s", "p50_ms", "p99_ms")})
                rate += 25.0
            for _ in range(2 if lo is not None and hi is not None else 0):
                mid = (lo + hi) / 2
                r = probe(mid)
                if r["sustained"]:
                    lo = mid
                    best = dict(rate=mid,
                                **{k: r[k] for k in ("solves_per_s", "p50_ms", "p99_ms")})
                else:
                    hi = mid
            search[dt] = dict(highest_sustained=best, tried=tried)
    served_line(args, out, search)


def served_line(args, out, search):
    f = out["f32"] if "f32" in out else next(iter(out.values()))
    n = f["measured_requests"]
    line = {"metric": "served CP-ALS solves/s, p50/p99 latency",
            "value": f["solves_per_s"], "unit": "solves/s", "n_gpus": 1, "steps": n,
            "warmup": f["warmup_requests"], "ms_per_step": round(f["span_s"] * 1e3 / n, 4),
            "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
            "dtype": "f32" if "f32" in out else next(iter(out)), "data": "synthetic",
            "config": {"workload": f"served: Poisson {args.rate:g}/s, {args.served_warmup} warm-up "
                                   f"+ {args.served_requests} measured requests, batched-"
                                   f"distribution solves + {args.large_frac:g} 50M-nonzero "
                                   f"1M x 500K x 200K requests, fit change < 1e-4 or 50 "
                                   f"iterations, continuous batching",
                       "requests": n, "parallelism": "single GPU"},
            "extra": dict(out, rate_search=search or None)}
    print(json.dumps(line), flush=True)


# DFacTo's own seconds per iteration on its synthetic tensors (Section 5,
# the two synthetic tables), for context: {I: (ALS, GD)}
PAPER_T4 = {10_000: (1.14, 2.32), 100_000: (2.72, 5.87), 1_000_000: (7.26, 16.51),
            10_000_000: (41.64, 121.30)}
PAPER_T5 = {10_000: (0.05, 0.09), 100_000: (0.92, 1.81), 1_000_000: (12.06, 21.74),
            10_000_000: (144.48, 275.19)}


def run_synthetic(args):
    """The paper's synthetic sweeps (Section 5) on preferential-attachment
    tensors, I = J = K in {1e4, 1e5, 1e6, 1e7}: nnz = 1e6 (first table) and
    nnz = 2 I (second table); R = 10, FP32 factors.  Per case: one CP-ALS
    iteration (average of 3 after a warm-up) and one full GD iteration
    (gradient + Armijo line search + update; the average of iterations 2-3,
    each starting from twice the previous step)."""
    import numpy as np
    import torch
    from paper_1406_4519_amd import dfacto, gen

    dev = torch.device("cuda:0")
    ctx = dfacto.Context(0)
    R = 10
    cases = []
    for table, nnz_of in (("nnz=1e6", lambda I: 1_000_000), ("nnz=2I", lambda I: 2 * I)):
        for I in (10_000, 100_000, 1_000_000, 10_000_000):
            t0 = time.perf_counter()
            coo = gen.preferential_distinct((I, I, I), nnz_of(I), seed=500 + len(cases))
            gen_s = time.perf_counter() - t0
            arrs = [torch.from_numpy(x.view(np.int32)).to(dev) for x in (coo.i, coo.j, coo.k)]
            v = torch.from_numpy(coo.val).to(dev)
            torch.cuda.synchronize()
            tb = time.perf_counter()
            T = dfacto.build_flattenings(ctx, coo.dims, *arrs, v)
            torch.cuda.synchronize()
            build_ms = (time.perf_counter() - tb) * 1e3
            del arrs, v
            info = T.info()
            F0 = gen.init_factors(coo.dims, R, seed=600 + len(cases))
            F = [torch.from_numpy(np.ascontiguousarray(f, dtype=np.float32)).to(dev) for f in F0]
            G = [torch.empty((d, R), dtype=torch.float32, device=dev) for d in coo.dims]
            lam = torch.zeros(R, dtype=torch.float64, device=dev)
            fit = torch.zeros(1, dtype=torch.float64, device=dev)
            dfacto.als_iter(ctx, T, F, lam, fit)
            torch.cuda.synchronize()
            ts = time.perf_counter()
            for _ in range(3):
                dfacto.als_iter(ctx, T, F, lam, fit)
            torch.cuda.synchronize()
            als_ms = (time.perf_counter() - ts) * 1e3 / 3
            for m, f0 in enumerate(F0):
                F[m].copy_(torch.from_numpy(np.ascontiguousarray(f0, dtype=np.float32)).to(dev))
            gd, a0 = [], 1.0
            for _ in range(3):
                torch.cuda.synchronize()
                tg = time.perf_counter()
                r = dfacto.gd_step(ctx, T, F, G, alpha0=a0, shrink=0.5, c=1e-4, max_trials=60)
                gd.append(((time.perf_counter() - tg) * 1e3, r["trials"]))
                a0 = 2.0 * r["alpha"] if r["accepted"] else a0
            paper = (PAPER_T4 if table == "nnz=1e6" else PAPER_T5)[I]
            c = dict(table=table, I=I, nnz=info["nnz"], nfib=list(info["nfib"]),
                     generate_s=round(gen_s, 2), build_ms=round(build_ms, 2),
                     als_iter_ms=round(als_ms, 3), fit=float(fit.item()),
                     gd_iter_ms=round((gd[1][0] + gd[2][0]) / 2, 3),
                     gd_trials=[x[1] for x in gd], gd_first_iter_ms=round(gd[0][0], 3),
                     paper_s={"als": paper[0], "gd": paper[1]})
            log(f"{table} I={I:,}: {c}")
            cases.append(c)
            T.close()
            del F, G
            torch.cuda.empty_cache()
    big = [c for c in cases if c["table"] == "nnz=2I" and c["I"] == 10_000_000][0]
    line = {"metric": "synthetic preferential-attachment tensors: ms per CP-ALS iteration",
            "value": big["als_iter_ms"], "unit": "ms", "n_gpus": 1, "steps": 3, "warmup": 1,
            "ms_per_step": big["als_iter_ms"], "higher_is_better": False, "scaling": "weak",
            "vs_baseline": None, "dtype": "f32", "data": "synthetic",
            "config": {"workload": "the paper's synthetic sweeps: I = J = K in {1e4, 1e5, 1e6, 1e7}, "
                                   "nnz = 1e6 and nnz = 2I, preferential attachment, R = 10; value = "
                                   "CP-ALS iteration at I = 1e7, nnz = 2e7",
                       "parallelism": "single GPU"},
            "extra": {"cases": cases}}
    print(json.dumps(line), flush=True)
    ctx.close()


def run_joint(args):
    """Joint matrix completion + tensor factorization at the zipf50m shape:
    X = the 1M x 500K x 200K, 50M-nonzero Zipf(1.1) tensor (users x items x
    words) and Y = 10M distinct Zipf(1.1) ratings over the same users and
    items (|N(0,1)| values), R = 32, FP32 factors, mu = 1, lam = 0.1: time
    of one joint gradient (+ objective) and one joint ALS iteration."""
    import numpy as np
    import torch
    from paper_1406_4519_amd import dfacto, gen

    dev = torch.device("cuda:0")
    coo, R, F0 = gen.zipf_50m()
    yc = gen.zipf_distinct((coo.dims[0], coo.dims[1], 1), 10_000_000, 1.1, seed=31)
    log("generated X and Y")
    ctx = dfacto.Context(0)
    X = dfacto.build_flattenings(ctx, coo.dims,
                                 *[torch.from_numpy(a.view(np.int32)).to(dev)
                                   for a in (coo.i, coo.j, coo.k)],
                                 torch.from_numpy(coo.val).to(dev))
    tb = time.perf_counter()
    Y = dfacto.build_ratings(ctx, (coo.dims[0], coo.dims[1]),
                             torch.from_numpy(yc.i.view(np.int32)).to(dev),
                             torch.from_numpy(yc.j.view(np.int32)).to(dev),
                             torch.from_numpy(yc.val).to(dev))
    torch.cuda.synchronize()
    yb_ms = (time.perf_counter() - tb) * 1e3
    F = [torch.from_numpy(np.ascontiguousarray(f, dtype=np.float32)).to(dev) for f in F0]
    G = [torch.empty((d, R), dtype=torch.float32, device=dev) for d in coo.dims]
    f = torch.zeros(1, dtype=torch.float64, device=dev)
    mu, lam = 1.0, 0.1
    dfacto.joint_grad(ctx, X, Y, F, G, f, mu, lam)
    dfacto.joint_als_iter(ctx, X, Y, F, mu, lam)
    torch.cuda.synchronize()
    reps = 5
    ts = time.perf_counter()
    for _ in range(reps):
        dfacto.joint_grad(ctx, X, Y, F, G, f, mu, lam)
    torch.cuda.synchronize()
    grad_ms = (time.perf_counter() - ts) * 1e3 / reps
    fs = []
    ts = time.perf_counter()
    for _ in range(3):
        dfacto.joint_als_iter(ctx, X, Y, F, mu, lam)
    torch.cuda.synchronize()
    als_ms = (time.perf_counter() - ts) * 1e3 / 3
    dfacto.joint_grad(ctx, X, Y, F, G, f, mu, lam)
    torch.cuda.synchronize()
    res = dict(ratings=yc.nnz, ratings_build_ms=round(yb_ms, 1), joint_grad_ms=round(grad_ms, 3),
               joint_als_iter_ms=round(als_ms, 3), f_after=float(f.item()))
    log(f"joint: {res}")
    line = {"metric": "joint matrix completion + tensor factorization: ms per ALS iteration",
            "value": res["joint_als_iter_ms"], "unit": "ms", "n_gpus": 1, "steps": 3, "warmup": 1,
            "ms_per_step": res["joint_als_iter_ms"], "higher_is_better": False, "scaling": "weak",
            "vs_baseline": None, "dtype": "f32", "data": "synthetic",
            "config": {"workload": "joint model: X = zipf50m (1M x 500K x 200K, 50M nonzeros), "
                                   "Y = 10M Zipf(1.1) ratings over its users x items, R = 32, "
                                   "mu = 1, lam = 0.1", "parallelism": "single GPU"},
            "extra": res}
    print(json.dumps(line), flush=True)
    X.close()
    Y.close()
    ctx.close()



def _dev_sample(i, j, k, v, n, seed=11):
    """n seeded random nonzeros of a device COO, copied to host (uint32 /
    float32 numpy), for the CPU baseline."""
    import numpy as np
    import torch
    g = torch.Generator(device=i.device)
    g.manual_seed(seed)
    n = min(n, i.numel())
    pick = torch.randperm(i.numel(), generator=g, device=i.device)[:n].sort().values
    out = [a[pick].cpu().numpy() for a in (i, j, k)]
    out = [np.ascontiguousarray(a).view(np.uint32) for a in out]
    return out[0], out[1], out[2], v[pick].cpu().numpy()


def _stream_bw(dev, gib=4):
    """Achievable device bandwidth: a plain device-to-device copy of `gib`
    GiB (read + write), best of 5."""
    import torch
    n = gib * (1 << 30) // 4
    a = torch.ones(n, dtype=torch.float32, device=dev)
    b = torch.empty_like(a)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    best = 1e30
    for _ in range(6):
        e0.record()
        b.copy_(a)
        e1.record()
        torch.cuda.synchronize()
        best = min(best, e0.elapsed_time(e1))
    del a, b
    torch.cuda.empty_cache()
    return 2.0 * 4 * n / (best * 1e-3) / 1e9


def run_tensor(args):
    """The default workload (paper1200m) and zipf50m / small: timed steps of
    CP-ALS iterations + one GD gradient for each (R, factor dtype)."""
    import numpy as np
    import torch
    from paper_1406_4519_amd import dfacto, gen

    dev = torch.device("cuda:0")
    t0 = time.perf_counter()
    if args.workload == "paper1200m":
        dims = (6_500_000, 2_500_000, 1_500_000)
        i, j, k, v = gen.zipf_distinct_torch(
            dims, args.paper_nnz, 1.2, seed=3, device=dev, batch=1 << 28,
            progress=lambda m: log(f"  [{time.perf_counter() - t0:.0f}s] {m}"))
        ranks, init_seed = tuple(int(x) for x in args.ranks.split(",")), 1003
        aps = args.als_per_step or 1
        wl = (f"paper1200m: 6,500,000 x 2,500,000 x 1,500,000, {args.paper_nnz:,} distinct "
              f"Zipf(1.2) coordinates (seeded permutation per mode), |N(0,1)| FP32 values, R=32, "
              f"U(0,1) FP32 factors; step = {aps} CP-ALS iteration{'s' if aps > 1 else ''} + 1 GD "
              f"gradient ({3 * aps + 3} MTTKRPs); R=32 BF16 and R=10 FP32/BF16 in extra.runs")
    else:
        coo, R0, _ = gen.zipf_50m() if args.workload == "zipf50m" else gen.small_uniform()
        dims = coo.dims
        i, j, k = (torch.from_numpy(a.view(np.int32)).to(dev) for a in (coo.i, coo.j, coo.k))
        v = torch.from_numpy(coo.val).to(dev)
        ranks, init_seed = (R0,), (1002 if args.workload == "zipf50m" else 1001)
        aps = args.als_per_step or (10 if args.workload == "zipf50m" else 5)
        wl = (f"{args.workload}: {' x '.join(f'{d:,}' for d in dims)}, {coo.nnz:,} distinct "
              f"coordinates, R={R0}; step = {aps} CP-ALS iterations + 1 GD gradient "
              f"({3 * aps + 3} MTTKRPs)")
        del coo
    torch.cuda.synchronize()
    log(f"generated in {time.perf_counter() - t0:.1f}s")
    sample = None if args.no_cpu_baseline else _dev_sample(i, j, k, v, args.cpu_sample)
    # the library allocates through torch's caching allocator: the build
    # reuses device memory the input generator has already mapped (fresh
    # device memory is mapped and cleared by the kernel driver at a few tens of
    # GB/s, which would dominate the build's time)
    ctx = dfacto.Context(0, allocator="torch")
    torch.cuda.synchronize()
    tb = time.perf_counter()
    relabel = {"auto": None, "on": True, "off": False}[args.relabel]
    T = dfacto.build_flattenings(ctx, dims, i, j, k, v, relabel=relabel)
    torch.cuda.synchronize()
    build_ms = (time.perf_counter() - tb) * 1e3
    del i, j, k, v
    torch.cuda.empty_cache()
    info = T.info()
    nnz = info["nnz"]
    log(f"built in {build_ms:.0f} ms: {nnz:,} nonzeros nfib={info['nfib']} nroot={info['nroot']} "
        f"bytes={info['bytes'] / 1e9:.2f} GB")
    per_step = 3.0 * aps + 3.0

    def make(R, dt, F0):
        tdt = torch.float32 if dt == "f32" else torch.bfloat16
        F = [torch.from_numpy(np.ascontiguousarray(f, dtype=np.float32)).to(dev).to(tdt)
             for f in F0]
        G = [torch.empty((d, R), dtype=torch.float32, device=dev) for d in dims]
        z = lambda n: torch.zeros(n, dtype=torch.float64, device=dev)
        return F, G, z(R), z(1), z(1)

    def variant(R, dt, F0, headline):
        F, G, lam, fit, fval = make(R, dt, F0)

        def step():
            for _ in range(aps):
                dfacto.als_iter(ctx, T, F, lam, fit)
            dfacto.gd_grad(ctx, T, F, G, fval)

        for _ in range(args.warmup):
            step()
        torch.cuda.synchronize()
        dfacto.profile_enable(ctx, True)
        torch.cuda.synchronize()
        ts = time.perf_counter()
        for _ in range(args.steps):
            step()
        torch.cuda.synchronize()
        el = time.perf_counter() - ts
        prof = dfacto.profile_read(ctx)
        dfacto.profile_enable(ctx, False)
        el_eager, graph_ok = el, None
        if not args.no_graph:
            # the same step captured once as a HIP graph and replayed; its
            # first replay must equal an eager step from the same state
            state = [x.clone() for x in (*F, lam, fit)]
            step()
            torch.cuda.synchronize()
            eager = [x.clone() for x in (*F, lam, fit, *G, fval)]
            for x, y in zip((*F, lam, fit), state):
                x.copy_(y)
            del state
            torch.cuda.synchronize()
            g = torch.cuda.CUDAGraph()
            side = torch.cuda.Stream()
            side.wait_stream(torch.cuda.current_stream())
            main = torch.cuda.current_stream()
            try:
                with torch.cuda.graph(g, stream=side):
                    ctx.set_stream(side)
                    step()
            finally:
                ctx.set_stream(main)
            g.replay()
            torch.cuda.synchronize()
            as_bits = lambda a: a.view(torch.int16) if a.dtype == torch.bfloat16 else a
            graph_ok = all(torch.equal(as_bits(a), as_bits(b))
                           for a, b in zip((*F, lam, fit, *G, fval), eager))
            del eager
            if graph_ok:
                for _ in range(2):
                    g.replay()
                torch.cuda.synchronize()
                ts = time.perf_counter()
                for _ in range(args.steps):
                    g.replay()
                torch.cuda.synchronize()
                el = time.perf_counter() - ts
            else:
                log("graph replay differs from the eager step: timing the eager steps")
            del g
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        reps = 3
        e0.record()
        for _ in range(reps):
            dfacto.als_iter(ctx, T, F, lam, fit)
        e1.record()
        torch.cuda.synchronize()
        als_ms = e0.elapsed_time(e1) / reps
        e0.record()
        for _ in range(reps):
            dfacto.gd_grad(ctx, T, F, G, fval)
        e1.record()
        torch.cuda.synchronize()
        gd_ms = e0.elapsed_time(e1) / reps
        # per mode: the main kernel alone (library events) and the whole call
        modes = []
        for m in range(3):
            dfacto.profile_enable(ctx, True)
            e0.record()
            for _ in range(reps):
                dfacto.mttkrp(ctx, T, m, F, G[m])
            e1.record()
            pm = dfacto.profile_read(ctx)
            dfacto.profile_enable(ctx, False)
            kms = pm["ms"] / pm["launches"]
            kb = pm["bytes"] / pm["launches"]
            modes.append(dict(call_ms=round(e0.elapsed_time(e1) / reps, 4),
                              kernel_ms=round(kms, 4), alg_bytes=round(kb),
                              frac=round(kb / (kms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
                              nnzR_per_s=round(nnz * R / (kms * 1e-3))))
        avg = prof["ms"] / max(prof["launches"], 1)
        bpl = prof["bytes"] / max(prof["launches"], 1)
        out = dict(ms_per_step=round(el * 1e3 / args.steps, 4),
                   ms_per_step_eager=round(el_eager * 1e3 / args.steps, 4),
                   graph_replay_equals_eager=graph_ok,
                   value=per_step * nnz * R * args.steps / el,
                   als_iter_ms=round(als_ms, 3), gd_grad_ms=round(gd_ms, 3),
                   main_kernel_ms=round(avg, 4), launches=prof["launches"],
                   alg_bytes_per_launch=round(bpl),
                   achieved_GBs=round(bpl / (avg * 1e-3) / 1e9, 1) if avg > 0 else 0.0,
                   modes=modes, fit=float(fit.item()), f=float(fval.item()))
        out["frac"] = round(out["achieved_GBs"] / HBM_PEAK_GBS, 4)
        if headline:
            out["_state"] = (F, G)
        else:
            del F, G
            torch.cuda.empty_cache()
        log(f"R={R} {dt}: {json.dumps({k2: v2 for k2, v2 in out.items() if k2 != '_state'})}")
        return out

    runs = {}
    R = ranks[0]
    F0 = gen.init_factors(dims, R, seed=init_seed)
    head = variant(R, "f32", F0, True)
    F, G = head.pop("_state")
    # the main kernel's request ceiling (same requests without arithmetic)
    # and cold repetitions (a 2 GiB write-read first evicts the 256 MB
    # Infinity Cache), per mode, headline configuration
    ceiling, cold = [], []
    evict = torch.empty((2 << 30) // 4, dtype=torch.float32, device=dev)
    sink = None
    for m in range(0 if args.no_ceiling else 3):
        row = {}
        for pat, name in ((0, "own_rows"), (1, "uniform_rows"), (2, "l2_rows"), (3, "no_gathers")):
            sink = dfacto.gather_probe(ctx, T, m, F, pat, sink)
            torch.cuda.synchronize()
            dfacto.profile_enable(ctx, True)
            for _ in range(3):
                dfacto.gather_probe(ctx, T, m, F, pat, sink)
            pp = dfacto.profile_read(ctx)
            dfacto.profile_enable(ctx, False)
            row[name + "_ms"] = round(pp["ms"] / pp["launches"], 4)
        row["mttkrp_frac_of_own_ceiling"] = round(row["own_rows_ms"] /
                                                  head["modes"][m]["kernel_ms"], 4)
        ceiling.append(row)
        ks = []
        for _ in range(5):
            evict.fill_(float(len(ks)))
            dfacto.profile_enable(ctx, True)
            dfacto.mttkrp(ctx, T, m, F, G[m])
            pp = dfacto.profile_read(ctx)
            dfacto.profile_enable(ctx, False)
            ks.append(pp["ms"])
        kb = head["modes"][m]["alg_bytes"]
        cms = float(np.median(ks))
        cold.append(dict(kernel_ms=round(cms, 4),
                         frac=round(kb / (cms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)))
    del evict, sink
    gd_iters = []
    if args.gd_iters > 0:
        for m, f0 in enumerate(F0):
            F[m].copy_(torch.from_numpy(np.ascontiguousarray(f0, dtype=np.float32)).to(dev))
        a0 = 1.0
        for _ in range(args.gd_iters):
            torch.cuda.synchronize()
            tg = time.perf_counter()
            inf = dfacto.gd_step(ctx, T, F, G, alpha0=a0, shrink=0.5, c=1e-4, max_trials=60)
            gd_iters.append(dict(ms=round((time.perf_counter() - tg) * 1e3, 3),
                                 trials=inf["trials"], alpha=inf["alpha"], f=inf["f"]))
            a0 = 2.0 * inf["alpha"] if inf["accepted"] else a0
    del F, G
    torch.cuda.empty_cache()
    runs[f"R{R}_f32"] = head
    if not args.no_bf16:
        runs[f"R{R}_bf16"] = variant(R, "bf16", F0, False)
    for R2 in ranks[1:]:
        F02 = gen.init_factors(dims, R2, seed=init_seed)
        runs[f"R{R2}_f32"] = variant(R2, "f32", F02, False)
        if not args.no_bf16:
            runs[f"R{R2}_bf16"] = variant(R2, "bf16", F02, False)
    stream_gbs = _stream_bw(dev)
    if args.copy_mib > 0:
        n = args.copy_mib * (1 << 20) // 4
        src = torch.ones(n, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    T.close()
    ctx.close()
    cpu = None
    if sample is not None:
        threads = oracle_threads()
        log(f"timing the CPU oracle on a bounded sample ({threads} threads) ...")
        cpu = cpu_baseline(sample, dims, R, F0, args.cpu_seconds, threads)
        if threads > 1:
            one = cpu_baseline(sample, dims, R, F0, args.cpu_seconds / 2, 1)
            cpu["one_thread"] = {k2: one[k2] for k2 in ("value", "seconds", "sample")}
    traffic = load_traffic(args.workload)
    roofline = {"bound": "hbm", "achieved": head["achieved_GBs"], "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": head["frac"], "traffic": traffic,
                "kernel": "k_mttkrp (main MTTKRP kernel, all 3 modes)",
                "launches": head["launches"], "avg_launch_ms": head["main_kernel_ms"],
                "alg_bytes_per_launch": head["alg_bytes_per_launch"],
                "frac_cold": round(sum(c["frac"] for c in cold) / 3, 4) if cold else None,
                "achievable_stream_GBs": round(stream_gbs, 1),
                "frac_of_achievable": round(head["achieved_GBs"] / stream_gbs, 4)}
    line = {"metric": METRIC, "value": head["value"], "unit": "nnz·R/s", "n_gpus": 1,
            "steps": args.steps, "warmup": args.warmup, "ms_per_step": head["ms_per_step"],
            "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
            "data": "synthetic",
            "config": {"workload": wl, "nnz": nnz, "R": R, "dims": list(dims),
                       "als_per_step": aps, "parallelism": "single GPU"},
            "roofline": roofline, "cpu_baseline": cpu,
            "extra": {"timed_as": "HIP graph replay of the step" if head["graph_replay_equals_eager"]
                      else "eager launches",
                      "build_ms": round(build_ms, 1),
                      "build_memory": "torch caching allocator (memory the generator mapped)",
                      "relabeled": info["relabeled"], "nfib": list(info["nfib"]),
                      "nroot": list(info["nroot"]), "nentry": list(info["nentry"]),
                      "runs": runs, "gather_ceiling": ceiling, "cold_mttkrp": cold,
                      "gd_iterations": gd_iters,
                      "paper_context_s": {"als_iter_4_machines": 480, "gd_iter_4_machines": 1143}}}
    print(json.dumps(line), flush=True)


def oracle_threads() -> int:
    """Host cores this process may use, capped at the 16 a one-GPU share of
    the host offers."""
    try:
        n = len(os.sched_getaffinity(0))
    except (AttributeError, OSError):
        n = os.cpu_count() or 1
    return max(1, min(n, 16))


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawTextHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="paper1200m",
                    choices=["paper1200m", "zipf50m", "small", "batched", "served", "synthetic",
                             "joint"])
    ap.add_argument("--batch", type=int, default=256, help="batched workload: number of tensors")
    ap.add_argument("--iters", type=int, default=20, help="batched workload: ALS iterations")
    ap.add_argument("--build-threads", type=int, default=2,
                    help="batched workload: host threads building the tensors")
    ap.add_argument("--rate", type=float, default=200.0, help="served workload: arrivals per second")
    ap.add_argument("--served-warmup", type=int, default=200,
                    help="served workload: warm-up requests (not measured)")
    ap.add_argument("--served-requests", type=int, default=4000,
                    help="served workload: measured requests")
    ap.add_argument("--rate-search", action="store_true",
                    help="served workload: also find the highest sustained rate")
    ap.add_argument("--search-requests", type=int, default=600,
                    help="served workload: measured requests per rate-search run")
    ap.add_argument("--large-frac", type=float, default=0.05,
                    help="served workload: fraction of 50M-nonzero requests")
    ap.add_argument("--pool", type=int, default=48, help="served workload: distinct small tensors")
    ap.add_argument("--paper-nnz", type=int, default=1_200_000_000,
                    help="paper1200m workload: distinct nonzeros")
    ap.add_argument("--served-dtypes", default="f32,bf16",
                    help="served workload: factor storage dtypes, run in this order")
    ap.add_argument("--served-one", default=None,
                    help="served workload: one run 'dtype,rate,warm-up,measured,seed' in this "
                         "process (each served run is started this way in a process of its own)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-sample", type=int, default=400_000_000,
                    help="nonzeros copied to the host for the CPU baseline (at most)")
    ap.add_argument("--no-bf16", action="store_true", help="skip the BF16-factor runs")
    ap.add_argument("--relabel", choices=("auto", "on", "off"), default="auto",
                    help="relabeled gathers: by size (the library's default), always or never")
    ap.add_argument("--als-per-step", type=int, default=0,
                    help="CP-ALS iterations in a step, then one GD gradient "
                         "(default: 1 for paper1200m, 10 for zipf50m)")
    ap.add_argument("--ranks", default="32,10",
                    help="paper1200m workload: ranks, the first is the headline")
    ap.add_argument("--no-ceiling", action="store_true",
                    help="skip the request-ceiling probes and cold repetitions (profiling runs)")
    ap.add_argument("--gd-iters", type=int, default=3,
                    help="full GD iterations (line search) timed after the steps")
    ap.add_argument("--no-graph", action="store_true",
                    help="time eager launches instead of a HIP graph replay of the step")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--copy-mib", type=int, default=0,
                    help="after the timed region, run one plain device copy of this many MiB "
                         "(a known-size kernel for calibrating hardware byte counters)")
    args = ap.parse_args()

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path "
              "(how it would shard is a design note). Run with --gpus 1.", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_1406_4519_amd import dfacto

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    dfacto.load()  # fail loudly if the HIP library is missing
    if args.workload == "batched":
        return run_batched(args)
    if args.workload == "served":
        return run_served(args)
    if args.workload == "synthetic":
        return run_synthetic(args)
    if args.workload == "joint":
        return run_joint(args)
    return run_tensor(args)


if __name__ == "__main__":
    main()
