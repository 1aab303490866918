#!/usr/bin/env python3
"""Throughput of cascaded bilateral sampling (CABS) sketches on one MI355X.

One step = one complete CABS sketch (pilot sampling and evaluation, pilot
sketch with FP64 SVD and orthogonalisation, weighted k-means with snapping on
both sides, follow-up evaluation and sketch) plus the relative Frobenius error
of the result from i.i.d. sampled entries, on a synthetic low-rank-plus-noise
matrix that is never materialised (1e5 x 2e4, rank 200, s_i = 1/i, noise
N(0, 1e-3^2); k1 = k2 = 200, c = 5, FP32; error from 1e7 sampled entries).
Every step draws a fresh pilot sample (seed = step index), like the paper's
repeated runs.  Inputs (generator tables) are resident in HBM before timing.

Two timed phases over the same workload:
  * sequential: K sketches one after another on one stream, with per-kernel
    family timing (HIP events on the launch stream) for the roofline figure of
    the k-means distance GEMM + argmin kernel;
  * served: K sketch requests (sketch + error) through the continuous-batching
    server, closed loop with --slots requests in flight; `value` is this
    whole-job throughput and p50/p99 are its submit-to-completion latencies.
Also prints the FP64 CPU oracle timed on a bounded sample of the same workload.

`--stream` replaces all of this with the serving stream of uneven requests
(closed-loop maximum, then Poisson arrivals at fractions of it, p50/p99 from
arrival to completion); `--config NAME` times another workload.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "rank-k sketches/s at fixed rel-Frobenius error; p50/p99 sketch latency"
PEAK_TFLOPS = {"f64": 78.6, "f32": 157.3, "bf16": 2500.0, "f16": 2500.0}
PEAK_HBM_GBS = 8000.0


def parse():
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--config", default="lowrank1e5", help="workload name from workloads.CONFIGS")
    ap.add_argument("--compute", default=None, help="f64 | f32 | bf16 | f16 (default: the workload's)")
    ap.add_argument("--err-samples", type=int, default=None)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--slots", type=int, default=8, help="server slots (requests in flight) in the served phase")
    ap.add_argument("--no-served", action="store_true", help="skip the served phases (profiling runs)")
    ap.add_argument("--no-variants", action="store_true",
                    help="skip the BF16 served form and the scaled-signal workload")
    ap.add_argument("--copy-probe-mb", type=int, default=0,
                    help="before timing, copy a buffer of this many MiB device-to-device once (a kernel of known "
                         "traffic for calibrating rocprofv3 FETCH_SIZE / WRITE_SIZE)")
    ap.add_argument("--cpu-scale", type=float, default=0.5,
                    help="row/column scale of the workload the CPU oracle is timed on")
    ap.add_argument("--stream", action="store_true",
                    help="instead of the headline workload: the serving stream of uneven requests (Poisson "
                         "arrivals at fractions of the closed-loop maximum, p50/p99 per point)")
    ap.add_argument("--stream-requests", type=int, default=2000, help="requests per stream phase")
    ap.add_argument("--stream-pool", type=int, default=16, help="distinct request matrices built and uploaded")
    ap.add_argument("--stream-fracs", default="0.25,0.5,0.75,0.9",
                    help="offered load points as fractions of the measured closed-loop maximum")
    ap.add_argument("--stream-compute", default="bf16")
    return ap.parse_args()


def pmc_traffic(kernel: str):
    """HBM bytes per launch of `kernel` from the committed rocprofv3 counter summary
    (profiles/pmc_traffic.json), or None when the kernel's source has changed
    since the counters were taken."""
    import hashlib
    try:
        with open(os.path.join(ROOT, "profiles", "pmc_traffic.json")) as f:
            rec = json.load(f)[kernel]
        with open(os.path.join(ROOT, rec["source"]), "rb") as f:
            if hashlib.sha256(f.read()).hexdigest() != rec["source_sha256"]:
                return None
        return float(rec["bytes_per_launch"])
    except (OSError, KeyError, ValueError):
        return None


def cpu_baseline(config: str, scale: float, err_samples: int) -> dict:
    """The FP64 oracle on the same workload with m and n scaled by `scale`
    (k, c unchanged; error from err_samples * scale samples), one sketch.
    The oracle's cost is linear in m + n (Section 4), so the measured rate is
    scaled by (m_s + n_s) / (m + n) to sketches/s of the full workload."""
    import numpy as np

    import workloads
    from oracle import cabs as oc
    from oracle.matrices import Matrix

    full, cfg = workloads.config(config)
    spec, _ = workloads.config(config, scale)
    k = min(cfg["k"], spec.m, spec.n)
    ns = max(1, int(err_samples * scale))
    t0 = time.perf_counter()
    res = oc.cabs(spec, oc.Params.square(k, kmeans_iters=cfg["iters"], seed=0))
    if ns > 0:
        oc.rel_error_sampled(Matrix(spec), res.C, res.Umid, res.Rt, ns, 0)
    dt = time.perf_counter() - t0
    threads = None
    try:
        from threadpoolctl import threadpool_info
        threads = max((i.get("num_threads", 0) for i in threadpool_info()), default=None)
    except Exception:
        pass
    ratio = (spec.m + spec.n) / (full.m + full.n)
    return {"value": ratio / dt, "unit": "sketches/s", "cores": threads or os.cpu_count(), "kind": "oracle",
            "sample": f"FP64 NumPy oracle, one sketch of the same workload at m={spec.m}, n={spec.n} "
                      f"(scale {scale}), k={k}, c={cfg['iters']}, error from {ns} samples: {dt:.2f} s; "
                      f"rate scaled by (m_s+n_s)/(m+n)={ratio:.3g} (cost linear in m+n)",
            "seconds": dt}


def run_stream(args):
    """The serving stream: requests of uneven shape (m, n log-uniform in [1e3, 5e5], low-rank + noise or RBF,
    k in {16, ..., 256}, pilot size k, seed 1000 + id), sketches only.  The closed-loop maximum is measured
    first (--slots requests in flight); then the same requests arrive as a Poisson process at each fraction
    of that rate, and latency runs from arrival to completion (the server's submit-to-completion time plus
    any delay of the host loop in submitting).  Host generation of a 5e5-row orthonormal basis takes
    seconds, so the first --stream-pool recipes are built and uploaded once and request i runs on matrix
    i mod pool with its own k and seed."""
    import numpy as np
    import torch

    import workloads
    from paper_1607_07395_amd import api

    torch.cuda.set_device(0)
    n_req = args.stream_requests
    recs = workloads.request_stream(n_requests=n_req, qps=1.0, seed=0)
    P = max(1, min(args.stream_pool, n_req))
    t_b = time.perf_counter()
    pool = []
    for i in range(P):
        pool.append(api.DeviceMatrix(workloads.request_matrix(recs[i]), storage="f32"))
        print(f"stream: matrix {i + 1}/{P} {recs[i]['kind']} {recs[i]['m']}x{recs[i]['n']}", file=sys.stderr,
              flush=True)
    build_s = time.perf_counter() - t_b
    comp, iters, S = args.stream_compute, 5, max(1, args.slots)

    def params(i):
        mat = pool[i % P]
        k = min(recs[i]["k"], mat.spec.m, mat.spec.n)
        return mat, api.make_params(k, k, k, k, kmeans_iters=iters, compute=comp, seed=recs[i]["seed"])

    need = 0
    for mat in pool:
        kk = min(256, mat.spec.m, mat.spec.n)
        need = max(need, api.workspace_bytes(mat, api.make_params(kk, kk, kk, kk, kmeans_iters=iters, compute=comp)))
    srv = api.Server(0, hbm_budget_bytes=S * (need + (1 << 20)), max_slots=S)

    def drive(ids, arrivals):
        """Submit ids (closed loop when arrivals is None); returns latencies (ms) and the span (s)."""
        live, lat, last = {}, [], 0.0
        nxt, n = 0, len(ids)
        t0 = time.perf_counter()
        while nxt < n or live:
            now = time.perf_counter() - t0
            while nxt < n and ((arrivals is None and len(live) < S) or (arrivals is not None and arrivals[nxt] <= now)):
                mat, prm = params(ids[nxt])
                out = api.alloc_result(mat, prm)
                lag = 0.0 if arrivals is None else (time.perf_counter() - t0) - arrivals[nxt]
                live[srv.submit(mat, prm, out)] = (out, lag)
                nxt += 1
            for t in list(live):
                r = srv.poll(t)
                if r is not None:
                    _, lag = live.pop(t)
                    lat.append((r + lag) * 1e3)
                    last = time.perf_counter() - t0
            time.sleep(0.0002)
        return np.array(lat), last

    try:
        drive(list(range(min(n_req, 2 * S))), None)  # warm-up
        torch.cuda.synchronize()
        lat, span = drive(list(range(n_req)), None)
        lam = n_req / span
        closed = {"sketches_per_s": lam, "p50_ms": float(np.percentile(lat, 50)),
                  "p99_ms": float(np.percentile(lat, 99))}
        print(f"stream: closed loop {lam:.1f} sketches/s", file=sys.stderr, flush=True)
        points = []
        for f in [float(x) for x in args.stream_fracs.split(",") if x]:
            rng = np.random.default_rng(1)
            arr = np.cumsum(rng.exponential(1.0 / (f * lam), size=n_req))
            arr -= arr[0]
            lat, span = drive(list(range(n_req)), arr)
            points.append({"load_frac": f, "offered_per_s": f * lam, "sketches_per_s": n_req / span,
                           "p50_ms": float(np.percentile(lat, 50)), "p99_ms": float(np.percentile(lat, 99))})
            print(f"stream: load {f:g} -> p50 {points[-1]['p50_ms']:.1f} ms, p99 {points[-1]['p99_ms']:.1f} ms",
                  file=sys.stderr, flush=True)
    finally:
        srv.close()
    kinds = [pool[i % P].spec.kind for i in range(n_req)]
    print(json.dumps({
        "metric": "serving stream: sketches/s and p50/p99 latency under Poisson arrivals",
        "unit": "sketches/s", "n_gpus": 1, "dtype": comp, "data": "synthetic",
        "config": {"workload": "uneven requests: m, n log-uniform in [1e3, 5e5], low-rank + noise (rank 16-256) "
                               "or RBF (d = 32, 10-100 clusters), k in {16, 32, 64, 128, 256}, c = 5, sketch only",
                   "requests": n_req, "matrix_pool": P, "slots": S,
                   "pool_shapes": [[int(m.spec.m), int(m.spec.n), m.spec.kind] for m in pool],
                   "lowrank_share": kinds.count("lowrank") / n_req, "pool_build_s": build_s},
        "closed_loop": closed, "poisson": points}), flush=True)


def main():
    args = parse()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(json.dumps({"error": "this build runs on one GPU only; use --gpus 1"}))
        sys.exit(2)
    if args.stream:
        run_stream(args)
        return

    import numpy as np
    import torch

    import workloads
    from paper_1607_07395_amd import api

    torch.cuda.set_device(0)
    spec, cfg = workloads.config(args.config)
    compute = args.compute or cfg["precision"]
    storage = "f64" if compute == "f64" else "f32"
    ns = cfg["err_samples"] if args.err_samples is None else args.err_samples
    k, iters = cfg["k"], cfg["iters"]

    if args.copy_probe_mb > 0:
        src = torch.ones(args.copy_probe_mb << 18, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    mat = api.DeviceMatrix(spec, storage=storage)
    prm = api.make_params(k, k, k, k, kmeans_iters=iters, compute=compute, seed=0)
    ws = api._dev_alloc(api.workspace_bytes(mat, prm), mat.device)
    out = api.alloc_result(mat, prm)
    ews = None

    def step(i):
        nonlocal ews
        prm.seed = i
        api.sketch(mat, prm, ws=ws, out=out)
        e3 = api.error(mat, prm, out, ns, seed=1000 + i, ws=ews)
        ews = e3._ws
        return e3

    for i in range(args.warmup):
        step(10_000 + i)
    torch.cuda.synchronize()

    api.timing_reset()
    api.timing_enable(True)
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(args.steps)]
    errs = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        evs[i][0].record()
        errs.append(step(i))
        evs[i][1].record()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    api.timing_enable(False)

    seq_elapsed = t1 - t0
    lat = np.array([a.elapsed_time(b) for a, b in evs])
    rel_seq = np.array([float(e[2].item()) for e in errs])
    diag = out.diagnostics()

    # dominant throughput kernel: fused distance GEMM + argmin; (c + 1) assignments per side per sketch
    flops = args.steps * (iters + 1) * 2.0 * (spec.m + spec.n) * k * k
    a_ms, a_n = api.timing_read("assign")
    achieved = flops / (a_ms * 1e-3) / 1e12 if a_ms > 0 else 0.0
    peak = PEAK_TFLOPS[compute]
    fam = {f: api.timing_read(f) for f in ("assign", "eval", "tsgemm", "gram", "svd", "snap", "centroid", "error")}
    api.timing_reset()

    # ---- served phase: closed loop, `slots` requests in flight ----
    S = max(1, args.slots)

    def served(mat_, comp, n_req, seed0):
        p0 = api.make_params(k, k, k, k, kmeans_iters=iters, compute=comp, seed=0)
        req_bytes = max(api.workspace_bytes(mat_, p0), api.error_workspace_bytes(mat_, p0, ns))
        srv = api.Server(0, hbm_budget_bytes=S * (req_bytes + (1 << 20)), max_slots=S)
        sets = [(api.alloc_result(mat_, p0), torch.zeros(3, dtype=torch.float64, device="cuda")) for _ in range(S)]

        def run(n, s0):
            free = list(range(S))
            live = {}
            lats, rels = [], []
            nxt = 0
            while nxt < n or live:
                while free and nxt < n:
                    j = free.pop()
                    p = api.make_params(k, k, k, k, kmeans_iters=iters, compute=comp, seed=s0 + nxt)
                    t = srv.submit(mat_, p, sets[j][0], err_samples=ns, err_seed=1000 + s0 + nxt, err_out=sets[j][1])
                    live[t] = j
                    nxt += 1
                for t in list(live):
                    r = srv.poll(t)
                    if r is not None:
                        j = live.pop(t)
                        lats.append(r * 1e3)
                        rels.append(float(sets[j][1][2].item()))
                        free.append(j)
                time.sleep(0.0002)
            return np.array(lats), np.array(rels)

        try:
            run(min(S, max(1, args.warmup)), 20_000)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            lat_, rel_ = run(n_req, seed0)
            torch.cuda.synchronize()
            return time.perf_counter() - t0, lat_, rel_
        finally:
            srv.close()

    if args.no_served:
        elapsed, s_lat, s_rel = seq_elapsed, lat, rel_seq
        mode = "sequential (served phase skipped)"
    else:
        elapsed, s_lat, s_rel = served(mat, compute, args.steps, 0)
        mode = f"served: continuous-batching server, {S} requests in flight (closed loop), sketch + error each"
    variants = {}
    if not args.no_served and not args.no_variants and compute == "f32":
        # the mixed-precision served form on the same workload and seeds
        e_b, l_b, r_b = served(mat, "bf16", args.steps, 0)
        variants["bf16_served"] = {
            "sketches_per_s": args.steps / e_b, "p50_ms": float(np.percentile(l_b, 50)),
            "p99_ms": float(np.percentile(l_b, 99)), "rel_frobenius_error_mean": float(r_b.mean()),
            "error_ratio_to_f32_served": float(r_b.mean() / s_rel.mean())}
    if not args.no_variants and args.config == "lowrank1e5":
        # the same shape with s_i = sqrt(mn)/i, so that the signal dominates the noise
        spec_s, _ = workloads.config("lowrank1e5s")
        mat_s = api.DeviceMatrix(spec_s, storage=storage)
        out_s = api.alloc_result(mat_s, prm)
        def timed_sketches(**kw):
            errs, times = [], []
            for i in range(3):
                p = api.make_params(k, k, k, k, kmeans_iters=iters, compute=compute, seed=i, **kw)
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                api.sketch(mat_s, p, out=out_s)
                torch.cuda.synchronize()
                times.append(time.perf_counter() - t0)
                errs.append(float(api.error(mat_s, p, out_s, ns, seed=1000 + i)[2].item()))
            return float(np.mean(errs)), 1e3 * float(np.median(times))

        e_km, t_km = timed_sketches()
        variants["scaled_signal_f32"] = {"workload": "as above with s_i = sqrt(mn)/i", "rel_frobenius_error_mean": e_km,
                                         "sketch_ms_median": t_km, "sketches": 3}
        # the hard-threshold follow-up of Section 5 (the k rows and columns of largest |P_l|^2)
        e_h, t_h = timed_sketches(weight="pow", weight_param=2.0, follow_up="hard")
        variants["scaled_signal_hard_threshold_f32"] = {
            "workload": "as above with s_i = sqrt(mn)/i; follow-up: the k rows and columns of largest |P_l|^2",
            "rel_frobenius_error_mean": e_h, "sketch_ms_median": t_h, "sketches": 3}
        del mat_s, out_s

    result = {
        "metric": METRIC,
        "value": args.steps / elapsed,
        "unit": "sketches/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * elapsed / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": compute,
        "data": "synthetic",
        "config": {
            "workload": (f"{spec.kind} {spec.m}x{spec.n}" + (f" r={spec.r} noise={spec.noise_std:g}" if spec.kind == "lowrank"
                         else f" d={spec.d}") + f", k1=k2={k}, c={iters}, error from {ns} sampled entries"),
            "m": spec.m, "n": spec.n, "k": k, "kmeans_iters": iters, "err_samples": ns,
            "mode": mode,
            "rel_frobenius_error_mean": float(s_rel.mean()), "rel_frobenius_error_max": float(s_rel.max()),
            "p50_ms": float(np.percentile(s_lat, 50)), "p99_ms": float(np.percentile(s_lat, 99)),
            "sequential": {"sketches_per_s": args.steps / seq_elapsed, "ms_per_step": 1e3 * seq_elapsed / args.steps,
                           "p50_ms": float(np.percentile(lat, 50)), "p99_ms": float(np.percentile(lat, 99)),
                           "rel_frobenius_error_mean": float(rel_seq.mean())},
            "rank_final": diag["rank_final"], "entries_touched": diag["entries"],
            "snap_full_scans": [diag["snap_scans_r"], diag["snap_scans_c"]],
            **variants,
        },
        "roofline": {
            "kernel": "assign_fast_kernel (k-means distance GEMM + argmin), sequential phase",
            "bound": "mfma", "achieved": achieved, "peak": peak, "unit": "TFLOP/s",
            "frac": achieved / peak if peak else None,
            "traffic": pmc_traffic("assign_fast_kernel") if compute == "f32" and args.config == "lowrank1e5" else None,
            "traffic_unit": "bytes per launch (rocprofv3 FETCH_SIZE x2 + WRITE_SIZE, calibrated on a device copy; "
                            "profiles/lowrank1e5_f32_pmc_traffic.md)",
            "launches": a_n, "avg_launch_ms": a_ms / max(a_n, 1),
        },
        "kernel_ms_per_step": {f: v[0] / args.steps for f, v in fam.items()},
    }
    if not args.no_cpu_baseline:
        result["cpu_baseline"] = cpu_baseline(args.config, args.cpu_scale, ns)
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
