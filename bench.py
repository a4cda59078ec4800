#!/usr/bin/env python3
"""Throughput of the sliced fast kernel summation on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload negdist]

A step is one complete ksum_execute (projection, per-slice set-up, 1-D sums,
slice average) over the workload's inputs, which are resident in HBM before the
timed region starts.  The metric is target points x slices per second,
M * P / t_step.  Prints one JSON line on stdout (logs go to stderr).

Besides the headline number the line carries
  * p50 / p99 step latency,
  * "roofline": the kernel with the largest share of the step, timed with HIP
    events on the library's stream during a second timed region, its
    algorithmic work per launch over its average launch duration, against the
    MI355X peak of the resource that bounds it,
  * "cpu_baseline": the FP64 CPU oracle timed on this host on a bounded sample
    of the same workload (the first Q slices), plus the GPU result's error
    against the oracle on those slices and against the exact direct sum on a
    subsample of targets.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import workloads as wlm  # noqa: E402

METRIC = "target-pts x slices/s at <=1e-3 rel err vs direct, mixed vs FP32; p50/p99 latency"
UNIT = "target-pts x slices/s"

# MI355X published peaks
PEAK_HBM_GBS = 8000.0
PEAK_FP32_MFMA_TFLOPS = 157.3
PEAK_FP32_VALU_TFLOPS = 157.3


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def plan_kwargs(wl, sigma, precision="fp32"):
    kw = dict(seed=wl.dir_seed, precision=precision)
    if wl.kernel != "negdist":
        kw.update(sigma=sigma, n_coeff=wl.n_coeff, T=wl.T, method=wl.method)
        if wl.method == "nfft":
            kw.update(oversample=wl.oversample, window_m=wl.window_m)
    if wl.kernel == "laplacian":
        kw["method"] = "nfft"
    return kw


def kernel_work(stage, wl, P):
    """Algorithmic work of one launch of a stage: (bound, amount, unit, peak).

    Per-unit figures (per slice unless noted; L = N + M):
      project       2 d flops per point-slice            -> 2 (N+M) d P flops   (FP32 MFMA)
      sort_group    8 B (key, index) per entry + 4 B weight per source + 4 B t per target
      sort_hist     4 B projection per entry + 4 B weight per source
      sort_scatter  4 B projection read + 8 B (key, index) write per entry
      nfft_spread   4 B projection + 4 B weight per source
      nfft_interp   4 B projection read + 4 B t write per target
      accumulate    4 B t per target-slice read
      backproject   2 P flops per output coordinate     -> 2 R P d flops per launch, R = M (grad_y)
                    or N (grad_x); counted as (N + M) P d, the mean of the two launches (MFMA FP32)
    """
    N, M, d = wl.N, wl.M, wl.d
    L = N + M
    if stage == "project":
        return "mfma", 2.0 * L * d * P / 1e12, "TFLOP/s", PEAK_FP32_MFMA_TFLOPS
    if stage == "backproject":
        return "mfma", 1.0 * L * d * P / 1e12, "TFLOP/s", PEAK_FP32_MFMA_TFLOPS
    gb = {
        "sort_group": (8.0 * L + 4.0 * N + 4.0 * M) * P,
        "sort_hist": (4.0 * L + 4.0 * N) * P,
        "sort_scatter": 12.0 * L * P,
        "nfft_spread": 8.0 * N * P,
        "nfft_interp": 8.0 * M * P,
        "ndft_adjoint": 8.0 * N * P,
        "ndft_forward": 8.0 * M * P,
        "accumulate": 4.0 * M * P,
    }.get(stage)
    if gb is None:
        return None
    return "hbm", gb / 1e9, "GB/s", PEAK_HBM_GBS


# stage -> (kernel name prefix in the rocprofv3 summaries, source file of the kernel)
STAGE_KERNEL = {
    "project": ("proj_gemm_kernel", "k_project.hip"),
    "sort_group": ("sort_fast_kernel", "k_sort.hip"),
    "sort_scatter": ("sort_scatter_kernel", "k_sort.hip"),
    "sort_hist": ("sort_hist_kernel", "k_sort.hip"),
    "nfft_spread": ("nfft_spread_kernel", "k_fourier.hip"),
    "nfft_interp": ("nfft_interp_accum_kernel", "k_fourier.hip"),
    "ndft_adjoint": ("ndft_adjoint_kernel", "k_fourier.hip"),
    "ndft_forward": ("ndft_forward_kernel", "k_fourier.hip"),
    "accumulate": ("accumulate_kernel", "k_reduce.hip"),
}
WORKLOAD_TAG = {"negdist": "negdist_N1e5_d784_P256", "laplace": "laplace_N2e5_d3072_P512",
                "gauss_nfft": "gauss_nfft_N1e6_d50_P256", "gauss_ndft": "gauss_ndft_N1e3_d10_P64"}


def measure_stream_peak(dev, nbytes=1 << 30, reps=5):
    """Copy bandwidth of this GPU: best of `reps` device-to-device copies of `nbytes`
    (read + write counted), timed with events.  The reference that the HBM-bound
    stages are measured against next to the nominal peak."""
    import torch
    src = torch.empty(nbytes // 4, dtype=torch.float32, device=dev)
    dst = torch.empty_like(src)
    src.fill_(1.0)
    dst.copy_(src)
    best = None
    for _ in range(reps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        dst.copy_(src)
        e1.record()
        torch.cuda.synchronize()
        t = e0.elapsed_time(e1) * 1e-3
        best = t if best is None else min(best, t)
    del src, dst
    torch.cuda.empty_cache()
    return {"GBps": 2 * nbytes / best / 1e9, "bytes": nbytes, "reps": reps, "kind": "device-to-device copy"}


def source_digest(fname):
    import hashlib
    h = hashlib.sha256()
    for g in (fname, "device_common.h", "internal.h"):
        with open(os.path.join(ROOT, "paper_2401_08260_amd", "csrc", g), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def measured_traffic(workload, stage):
    """HBM bytes per launch of a stage's kernel from the committed FETCH_SIZE / WRITE_SIZE
    summary (already scaled by the copy-kernel calibration), or None when there is no
    summary or the kernel's source differs from the one the counters were taken with."""
    if stage not in STAGE_KERNEL or workload not in WORKLOAD_TAG:
        return None
    kname, src = STAGE_KERNEL[stage]
    path = os.path.join(ROOT, "profiles", f"hbm_traffic_{WORKLOAD_TAG[workload]}.md")
    if not os.path.exists(path):
        return None
    rd = wr = None
    digest = None
    with open(path) as f:
        for line in f:
            if line.startswith("| `" + kname):
                cols = [c.strip() for c in line.strip().strip("|").split("|")]
                rd, wr = float(cols[3]), float(cols[4])
            elif line.startswith("- source-digest " + src + " "):
                digest = line.split()[-1]
    if rd is None or digest != source_digest(src):
        return None
    return {"read_GB": rd, "write_GB": wr, "total_GB": rd + wr,
            "source": os.path.relpath(path, ROOT)}


def cpu_baseline(wl, x, y, w, sigma, xi, s_gpu, t_gpu, budget_s, exact_targets, s_mixed=None):
    """Oracle timing on a bounded sample + errors of the GPU result (oracle leg)."""
    from oracle import direct, sliced

    try:
        from threadpoolctl import threadpool_info
        blas_threads = max([i.get("num_threads", 1) for i in threadpool_info()] or [1])
    except Exception:  # pragma: no cover
        blas_threads = os.cpu_count() or 1
    method = "sort" if wl.kernel == "negdist" else wl.method
    # size the sample from the marginal cost of a slice (the first call also pays for
    # converting the points), then take as many slices as the budget allows
    def run(q):
        t0 = time.perf_counter()
        sliced.sliced_sum(wl.kernel, x, y, w, xi[:q], sigma, method, wl.n_coeff, wl.T, return_slices=True)
        return time.perf_counter() - t0
    q1 = min(wl.P, 4)
    t1 = run(1)
    tq = run(q1) if q1 > 1 else t1
    per = max((tq - t1) / max(q1 - 1, 1), tq / q1 * 0.25, 1e-4)
    Q = int(max(1, min(wl.P, (budget_s - t1) / per)))
    t0 = time.perf_counter()
    _, ts = sliced.sliced_sum(wl.kernel, x, y, w, xi[:Q], sigma, method, wl.n_coeff, wl.T, return_slices=True)
    dt = time.perf_counter() - t0
    out = {"value": wl.M * Q / dt, "unit": UNIT, "cores": int(blas_threads), "kind": "oracle",
           "sample": f"first {Q} of {wl.P} slices at full N={wl.N}, M={wl.M}, d={wl.d} "
                     f"({dt:.1f} s; FP64 projection + per-slice 1-D fast sum)"}
    # parity of the GPU per-slice sums on the sampled slices
    if t_gpu is not None:
        par = sliced.rel_l2(t_gpu[:Q].astype(np.float64), ts)
    elif Q == wl.P:   # every slice was sampled: compare the averages
        par = sliced.rel_l2(s_gpu.astype(np.float64), ts.mean(axis=0))
    else:
        par = None
    # error of the GPU result against the exact sum on a subsample of targets (also timed)
    k = min(exact_targets, wl.M)
    t0 = time.perf_counter()
    ex = direct.direct_sum(wl.kernel, x, y[:k], w, sigma if sigma > 0 else 1.0)
    dte = time.perf_counter() - t0
    s_sub = s_gpu[:k].astype(np.float64)
    errs = {"parity_rel_l2_vs_oracle": par, "parity_slices": Q,
            "exact_rel_l2": sliced.rel_l2(s_sub, ex),
            "exact_per_summand": sliced.per_summand_error(s_sub, ex, w),
            "exact_targets": k,
            "direct_pairs_per_s": float(k) * wl.N / dte}
    if s_mixed is not None:
        sm = s_mixed[:k].astype(np.float64)
        errs["mixed_exact_rel_l2"] = sliced.rel_l2(sm, ex)
        errs["mixed_exact_per_summand"] = sliced.per_summand_error(sm, ex, w)
    return out, errs, ex


GATE = 1e-3    # relative error against the exact sum the metric asks for


def error_gate(args, wl, sigma, xt, yt, wt, w_host, errs, exact):
    """One run at P* slices, the count where the slicing error (rate P^-1/2) reaches the
    gate, with the same directions extended (the first P are those of the main run).

    The gate metric is the relative l2 error for non-negative weights and the paper's
    per-summand error for signed weights.  P* = P (E / 1e-3)^2 x 1.2, rounded up to whole
    batches of 1024 slices; both the FP32 and the split-BF16 projection are run and
    their error is measured on the same exact targets as the main run."""
    import torch
    import paper_2401_08260_amd as ks
    from oracle import sliced

    signed = bool(np.any(w_host < 0))
    key = "exact_per_summand" if signed else "exact_rel_l2"
    e0 = errs[key]
    if e0 <= GATE:
        return {"metric": key, "P": wl.P, "error_at_P": e0, "note": "gate met at the workload's P"}
    Pstar = int(math.ceil(wl.P * (e0 / GATE) ** 2 * 1.2 / 1024.0)) * 1024
    k = errs["exact_targets"]
    out = {"metric": key, "error_at_P": e0, "P": Pstar, "slice_batch": 1024}
    dev = xt.device
    for prec in ("fp32", "split_bf16"):
        plan = ks.Plan(wl.d, Pstar, wl.kernel, slice_batch=1024, **plan_kwargs(wl, sigma, prec))
        s = torch.empty(wl.M, dtype=torch.float32, device=dev)
        stream = torch.cuda.current_stream(dev)
        e0v, e1v = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        e0v.record(stream)
        plan(xt, yt, wt, out=s)
        e1v.record(stream)
        torch.cuda.synchronize()
        ms = float(e0v.elapsed_time(e1v))
        sub = s[:k].cpu().numpy().astype(np.float64)
        err = sliced.per_summand_error(sub, exact, w_host) if signed else sliced.rel_l2(sub, exact)
        out[prec] = {"ms": ms, "value": wl.M * Pstar / (ms * 1e-3), "error": err, "meets_gate": err <= GATE}
        log(f"[bench] gate run P*={Pstar} {prec}: {ms:.1f} ms, {out[prec]['value']:.3e} {UNIT}, {key} {err:.2e}")
        del plan
    return out


# ---------------------------------------------------------------------------
# Serving mix: a Poisson stream of requests of uneven N, M, d, kernel and P.
# ---------------------------------------------------------------------------
SERVE_D = (16, 128, 784, 3072)
MAX_PTS = 500_000


def serve_params(kernel, sigma):
    if kernel == "gaussian":
        return dict(sigma=sigma, n_coeff=128, T=0.02, method="nfft", oversample=2, window_m=6)
    if kernel == "laplacian":
        return dict(sigma=sigma, n_coeff=256, T=0.125)
    return {}


def bench_serve(args):
    """Replays the serving stream twice on one GPU and reports latency and throughput:
      * served: the request server (continuous batching, `slots` concurrent streams,
        admission by HBM footprint) with the split-BF16 projection;
      * baseline: one request at a time in arrival order, FP32, on one stream.
    Point sets live in HBM: per dimension and distribution one pool of 5e5 sources and
    one of 5e5 targets, and each request takes a contiguous block of rows of each."""
    import torch
    import paper_2401_08260_amd as ks

    reqs = wlm.serving_stream(args.serve_requests, args.serve_rate, seed=4)
    dev = torch.device("cuda:0")
    gen = torch.Generator(device=dev)
    gen.manual_seed(4)
    pools, sig = {}, {}
    for d in SERVE_D:
        for kind in ("normal", "uniform"):
            mk = torch.randn if kind == "normal" else torch.rand
            xs = mk((MAX_PTS, d), device=dev, generator=gen)
            ys = mk((MAX_PTS, d), device=dev, generator=gen)
            pools[(d, kind)] = (xs, ys)
            sig[(d, kind)] = wlm.median_heuristic(xs[:250].cpu().numpy(), ys[:250].cpu().numpy())
    wpool = torch.rand(MAX_PTS, device=dev, generator=gen)
    gpool = torch.randn(MAX_PTS, device=dev, generator=gen)
    rng = np.random.default_rng(5)
    offs = [(int(rng.integers(0, MAX_PTS - r["N"] + 1)), int(rng.integers(0, MAX_PTS - r["M"] + 1))) for r in reqs]

    def inputs(i):
        r = reqs[i]
        xs, ys = pools[(r["d"], r["data"])]
        ox, oy = offs[i]
        return xs[ox:ox + r["N"]], ys[oy:oy + r["M"]], wpool[:r["N"]], gpool[:r["M"]]

    def params(i, precision):
        r = reqs[i]
        return dict(serve_params(r["kernel"], sig[(r["d"], r["data"])]), precision=precision, seed=r["P"])

    def outputs(i):
        r = reqs[i]
        s = torch.empty(r["M"], device=dev)
        gr = (None, None, None)
        if r["grad"]:
            gr = (torch.empty((r["N"], r["d"]), device=dev), torch.empty((r["M"], r["d"]), device=dev),
                  torch.empty(r["N"], device=dev))
        return s, gr

    work = float(sum(r["M"] * r["P"] for r in reqs))

    # plans made before any clock starts (server: one tiny request per plan key)
    srv = ks.Server(slots=args.serve_slots, hbm_bytes=int(args.serve_hbm_gb * (1 << 30)))
    first_of = {}
    for k, r in enumerate(reqs):
        first_of.setdefault((r["kernel"], r["d"], r["P"], r["data"]), k)
    for j, (key, i) in enumerate(sorted(first_of.items())):
        x, y, w, g = inputs(i)
        s = torch.empty(1000, device=dev)
        srv.submit(10**9 + j, key[0], key[1], key[2], x[:1000], y[:1000], w[:1000], s, params=params(i, "split_bf16"))
    srv.drain()
    srv.poll(100000)
    plans = {key: ks.Plan(reqs[i]["d"], reqs[i]["P"], reqs[i]["kernel"], **params(i, "fp32"))
             for key, i in first_of.items()}
    torch.cuda.synchronize()

    def summary(lat, makespan, extra):
        out = {"p50_ms": 1e3 * float(np.percentile(lat, 50)), "p99_ms": 1e3 * float(np.percentile(lat, 99)),
               "makespan_s": makespan, "value": work / makespan}
        out.update(extra)
        return out

    def run_served(scale):
        """Continuous batching with the split-BF16 projection; arrivals scaled by `scale`
        (0 = every request queued at once)."""
        lat, t_end_max, keep = [], 0.0, {}
        t0 = time.monotonic()
        i = pending = 0
        while i < len(reqs) or pending:
            now = time.monotonic() - t0
            while i < len(reqs) and reqs[i]["arrival"] * scale <= now:
                x, y, w, g = inputs(i)
                s, gr = outputs(i)
                keep[i] = (s, gr)
                srv.submit(i, reqs[i]["kernel"], reqs[i]["d"], reqs[i]["P"], x, y, w, s,
                           params=params(i, "split_bf16"), grad_s=g if reqs[i]["grad"] else None, grads=gr)
                i += 1
                pending += 1
            for c in srv.poll(4096):
                if c["status"] != 0:
                    raise RuntimeError(f"request {c['tag']} failed with status {c['status']}")
                lat.append(c["t_end"] - (t0 + reqs[c["tag"]]["arrival"] * scale))
                t_end_max = max(t_end_max, c["t_end"] - t0)
                keep.pop(c["tag"], None)
                pending -= 1
            time.sleep(5e-5)
        st = srv.stats()
        return summary(lat, t_end_max - reqs[0]["arrival"] * scale,
                       {"precision": "split_bf16", "slots": args.serve_slots,
                        "arena_peak_gb": st["arena_peak"] / 2**30})

    def run_baseline(scale):
        """One request at a time in arrival order, FP32, one stream."""
        stream = torch.cuda.current_stream(dev)
        lat = []
        t0 = time.monotonic()
        t_end = 0.0
        for i, r in enumerate(reqs):
            now = time.monotonic() - t0
            if r["arrival"] * scale > now:
                time.sleep(r["arrival"] * scale - now)
            plan = plans[(r["kernel"], r["d"], r["P"], r["data"])]
            x, y, w, g = inputs(i)
            s = torch.empty(r["M"], device=dev)
            plan(x, y, w, out=s, stream=stream)
            if r["grad"]:
                plan.backward(x, y, w, g, stream=stream)
            torch.cuda.synchronize()
            plan._ws = plan._bws = None        # one workspace at a time, reused through torch's cache
            t_end = time.monotonic() - t0
            lat.append(t_end - r["arrival"] * scale)
        return summary(lat, t_end - reqs[0]["arrival"] * scale, {"precision": "fp32", "slots": 1})

    served = run_served(1.0)
    log(f"[serve] served at {args.serve_rate:g} req/s: p50 {served['p50_ms']:.2f} ms p99 {served['p99_ms']:.2f} ms, "
        f"{served['value']:.3e} {UNIT} over {served['makespan_s']:.2f} s")
    base = run_baseline(1.0)
    log(f"[serve] one at a time at {args.serve_rate:g} req/s: p50 {base['p50_ms']:.2f} ms "
        f"p99 {base['p99_ms']:.2f} ms, {base['value']:.3e} {UNIT} over {base['makespan_s']:.2f} s")
    served_sat = run_served(0.0)
    log(f"[serve] served, all queued at once: {served_sat['value']:.3e} {UNIT} over {served_sat['makespan_s']:.2f} s")
    base_sat = run_baseline(0.0)
    log(f"[serve] one at a time, all queued at once: {base_sat['value']:.3e} {UNIT} "
        f"over {base_sat['makespan_s']:.2f} s")
    srv.close()
    result = {
        "metric": METRIC, "value": served["value"], "unit": UNIT, "n_gpus": 1, "steps": len(reqs),
        "warmup": len(first_of),
        "ms_per_step": 1e3 * served["makespan_s"] / len(reqs), "p50_ms": served["p50_ms"], "p99_ms": served["p99_ms"],
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32+split_bf16",
        "data": "synthetic",
        "config": {"workload": "serve", "requests": len(reqs), "rate_per_s": args.serve_rate, "seed": 4,
                   "N_M": "log-uniform [1e3, 5e5]", "d": list(SERVE_D), "P": [64, 256],
                   "kernels": ["gaussian", "laplacian", "negdist"], "grad_fraction": 0.3},
        "served": served, "one_at_a_time_fp32": base,
        "p50_speedup": base["p50_ms"] / served["p50_ms"], "p99_speedup": base["p99_ms"] / served["p99_ms"],
        "saturated": {"served": served_sat, "one_at_a_time_fp32": base_sat,
                      "throughput_speedup": served_sat["value"] / base_sat["value"]},
    }
    print(json.dumps(result), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="negdist", choices=sorted(wlm.WORKLOADS) + ["serve"])
    ap.add_argument("--serve-requests", type=int, default=1000)
    ap.add_argument("--serve-rate", type=float, default=200.0)
    ap.add_argument("--serve-slots", type=int, default=8)
    ap.add_argument("--serve-hbm-gb", type=float, default=64.0)
    ap.add_argument("--cpu-budget", type=float, default=15.0, help="seconds of oracle work in the CPU leg")
    ap.add_argument("--exact-targets", type=int, default=500)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-mixed", action="store_true", help="skip the split-BF16 (mixed) leg")
    ap.add_argument("--no-gate", action="store_true", help="skip the run at the slice count of the error gate")
    ap.add_argument("--backward", action="store_true",
                    help="also time one gradient step (grad_x, grad_y, grad_w for an upstream grad_s)")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="only copy 1 GiB device to device (reference for the HBM traffic counters)")
    args = ap.parse_args()

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        log("bench.py measures one GPU: the library has no multi-GPU path "
            "(slices would be sharded across GPUs with one all-reduce of s; see the design notes).")
        sys.exit(2)

    import torch
    import paper_2401_08260_amd as ks

    if args.workload == "serve":
        bench_serve(args)
        return

    if args.calibrate_copy:
        nbytes = 1 << 30
        src = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda:0")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"calibrate_copy_bytes": nbytes, "copies": 3}), flush=True)
        return

    wl = wlm.WORKLOADS[args.workload]
    log(f"[bench] workload {wl.name}: N={wl.N} M={wl.M} d={wl.d} P={wl.P} kernel={wl.kernel}")
    x, y, w = wlm.generate(wl)
    sigma = wlm.kernel_scale(wl, x, y)
    dev = torch.device("cuda:0")
    xt, yt, wt = (torch.from_numpy(a).to(dev) for a in (x, y, w))
    plan = ks.Plan(wl.d, wl.P, wl.kernel, **plan_kwargs(wl, sigma))
    s = torch.empty(wl.M, dtype=torch.float32, device=dev)
    stream = torch.cuda.current_stream(dev)

    def step():
        plan(xt, yt, wt, out=s)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()

    # timed region 1: headline throughput and per-step latency
    evs = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps + 1)]
    torch.cuda.synchronize()
    t_wall = time.perf_counter()
    evs[0].record(stream)
    for i in range(args.steps):
        step()
        evs[i + 1].record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t_wall
    per = np.array([evs[i].elapsed_time(evs[i + 1]) for i in range(args.steps)])
    ms = float(evs[0].elapsed_time(evs[-1])) / args.steps
    value = wl.M * wl.P / (ms * 1e-3)
    log(f"[bench] {ms:.3f} ms/step ({wall / args.steps * 1e3:.3f} ms wall), {value:.4e} {UNIT}")

    # timed region 2: per-kernel durations with HIP events on the execution stream
    ks.ksum_set_timing(plan.handle, True)
    torch.cuda.synchronize()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    stages = ks.ksum_stage_times(plan.handle)
    ks.ksum_set_timing(plan.handle, False)
    stage_ms = {k: v[0] / max(v[1], 1) for k, v in stages.items() if v[1] > 0}
    stage_share = {k: v[0] / args.steps for k, v in stages.items() if v[1] > 0}
    for k in sorted(stage_share, key=lambda q: -stage_share[q]):
        log(f"[bench]   {k:14s} {stage_share[k]:8.4f} ms/step  ({stages[k][1] // args.steps} launches/step)")
    dom = max((k for k in stage_share if kernel_work(k, wl, wl.P)), key=lambda k: stage_share[k])
    bound, amount, unit, peak = kernel_work(dom, wl, wl.P)
    achieved = amount / (stage_ms[dom] * 1e-3)
    tr = measured_traffic(wl.name, dom)
    roofline = {"kernel": dom, "bound": bound, "achieved": achieved, "peak": peak, "unit": unit,
                "frac": achieved / peak, "traffic": tr["total_GB"] if tr else None,
                "traffic_unit": "GB per launch (FETCH_SIZE + WRITE_SIZE, copy-calibrated)",
                "traffic_detail": tr, "avg_launch_ms": stage_ms[dom],
                "share_of_step": stage_share[dom] / ms}

    # every stage against its roofline: algorithmic bytes (or flops) per launch over the
    # launch time, and for HBM-bound stages the measured HBM traffic over the same time,
    # as fractions of the nominal peak and of the copy bandwidth measured here
    stream_pk = measure_stream_peak(dev)
    stage_roofline = {}
    for k in stage_share:
        kw = kernel_work(k, wl, wl.P)
        if not kw:
            continue
        b, amt, u, pk = kw
        ach = amt / (stage_ms[k] * 1e-3)
        ent = {"bound": b, "avg_launch_ms": stage_ms[k], "achieved": ach, "unit": u, "frac_peak": ach / pk}
        trk = measured_traffic(wl.name, k)
        if b == "hbm" and trk:
            gbs = trk["total_GB"] / (stage_ms[k] * 1e-3)
            ent.update(measured_GBps=gbs, frac_peak_measured=gbs / PEAK_HBM_GBS,
                       frac_stream_measured=gbs / stream_pk["GBps"])
        stage_roofline[k] = ent

    # timed region 3: the same step with the split-BF16 projection ("mixed")
    mixed = None
    s_mixed = None
    if not args.no_mixed:
        plan_m = ks.Plan(wl.d, wl.P, wl.kernel, **plan_kwargs(wl, sigma, "split_bf16"))
        sm = torch.empty(wl.M, dtype=torch.float32, device=dev)
        for _ in range(args.warmup):
            plan_m(xt, yt, wt, out=sm)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(args.steps):
            plan_m(xt, yt, wt, out=sm)
        e1.record(stream)
        torch.cuda.synchronize()
        ms_m = float(e0.elapsed_time(e1)) / args.steps
        ks.ksum_set_timing(plan_m.handle, True)
        plan_m(xt, yt, wt, out=sm)
        torch.cuda.synchronize()
        st_m = ks.ksum_stage_times(plan_m.handle)
        ks.ksum_set_timing(plan_m.handle, False)
        s_mixed = sm.cpu().numpy().astype(np.float64)
        s_fp32 = s.cpu().numpy().astype(np.float64)
        mixed = {"precision": "split_bf16", "ms_per_step": ms_m, "value": wl.M * wl.P / (ms_m * 1e-3),
                 "speedup_vs_fp32": ms / ms_m, "project_ms": st_m["project"][0] if "project" in st_m else None,
                 "rel_l2_vs_fp32_result": float(np.linalg.norm(s_mixed - s_fp32) / np.linalg.norm(s_fp32))}
        log(f"[bench] mixed (split-BF16 projection): {ms_m:.3f} ms/step, {mixed['value']:.4e} {UNIT}, "
            f"x{mixed['speedup_vs_fp32']:.2f} vs FP32")

    # timed region 4 (--backward): the gradients of an MMD gradient-flow step, grad_x, grad_y
    # and grad_w of s for a seeded upstream grad_s, on the same inputs and plan
    backward = None
    if args.backward:
        gs = torch.from_numpy(np.random.default_rng(7).standard_normal(wl.M).astype(np.float32)).to(dev)
        for _ in range(args.warmup):
            plan.backward(xt, yt, wt, gs)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(args.steps):
            plan.backward(xt, yt, wt, gs)
        e1.record(stream)
        torch.cuda.synchronize()
        ms_b = float(e0.elapsed_time(e1)) / args.steps
        ks.ksum_set_timing(plan.handle, True)
        torch.cuda.synchronize()
        for _ in range(args.steps):
            plan.backward(xt, yt, wt, gs)
        torch.cuda.synchronize()
        st_b = ks.ksum_stage_times(plan.handle)
        ks.ksum_set_timing(plan.handle, False)
        share_b = {k: v[0] / args.steps for k, v in st_b.items() if v[1] > 0}
        backward = {"what": "grad_x, grad_y and grad_w of s for an upstream grad_s",
                    "ms_per_step": ms_b, "stage_ms_per_step": share_b}
        if st_b.get("backproject", (0.0, 0))[1] > 0:
            bms = st_b["backproject"][0] / st_b["backproject"][1]
            b_bound, b_amt, b_unit, b_pk = kernel_work("backproject", wl, wl.P)
            backward["backproject_roofline"] = {"bound": b_bound, "avg_launch_ms": bms,
                                                "achieved": b_amt / (bms * 1e-3), "peak": b_pk, "unit": b_unit,
                                                "frac": b_amt / (bms * 1e-3) / b_pk}
        log(f"[bench] backward (grad_x, grad_y, grad_w): {ms_b:.3f} ms/step")

    result = {
        "metric": METRIC, "value": value, "unit": UNIT, "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms, "p50_ms": float(np.percentile(per, 50)),
        "p99_ms": float(np.percentile(per, 99)), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": wl.name, "kernel": wl.kernel, "method": "sort" if wl.kernel == "negdist"
                   else wl.method, "N": wl.N, "M": wl.M, "d": wl.d, "P": wl.P, "precision": "fp32",
                   "input": wl.dtype, "sigma": sigma},
        "stage_ms_per_step": stage_share,
        "roofline": roofline,
        "stream_peak": stream_pk,
        "stage_roofline": stage_roofline,
        "mixed": mixed,
    }
    if backward is not None:
        result["backward"] = backward

    if not args.no_cpu_baseline:
        probe_t = torch.empty((wl.P, wl.M), dtype=torch.float32, device=dev)
        plan(xt, yt, wt, out=s, probe={"t": probe_t})
        torch.cuda.synchronize()
        base, errs, exact = cpu_baseline(wl, x, y, w, sigma, plan.directions(), s.cpu().numpy(),
                                  probe_t.cpu().numpy(), args.cpu_budget,
                                  args.exact_targets, s_mixed)
        result["cpu_baseline"] = base
        result["errors"] = errs
        log(f"[bench] cpu baseline {base['value']:.3e} {UNIT} ({base['sample']}); errors {errs}")
        if not args.no_gate:
            result["error_gate"] = error_gate(args, wl, sigma, xt, yt, wt, w, errs, exact)
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
