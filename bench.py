#!/usr/bin/env python3
"""Throughput of the sliced fast kernel summation on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload laplace]

The metric is target points x slices per second, M * P / t_step, at a relative
error of at most 1e-3 against the exact direct sum.  The slicing error falls like
P^-1/2 (Sec. 4), so the workload's own slice count P does not reach 1e-3; the run
first measures the error at P against the exact sum on a subsample of targets, then
sets P* = P (E_P / 1e-3)^2 x 1.2 (whole batches of 1024 slices), and a step is one
complete ksum_execute (projection, per-slice set-up, 1-D sums, slice average) over
all P* slices with the inputs resident in HBM.  The headline is the mixed form
(split-BF16 projection); the plain FP32 form runs the same P* beside it.  Prints
one JSON line on stdout (logs go to stderr).

Besides the headline number the line carries
  * p50 / p99 step latency,
  * the error of both forms against the exact sum at P*, and at the workload's P,
  * "roofline": the kernel with the largest share of the step, timed with HIP
    events on the library's stream, its algorithmic work over its launch time,
    against the MI355X peak of the resource that bounds it,
  * "cpu_baseline": the FP64 CPU oracle, threads over slices, timed on this host
    on a bounded sample of the workload (the first Q slices), with the GPU's
    per-slice sums compared against it on those slices.
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
GATE = 1e-3          # relative error against the exact sum the metric asks for
GATE_BATCH = 1024    # slices per batch of the runs at P*

# MI355X published peaks
PEAK_HBM_GBS = 8000.0
PEAK_FP32_MFMA_TFLOPS = 157.3
PEAK_BF16_MFMA_TFLOPS = 2500.0
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


def kernel_work(stage, wl, P, precision="fp32"):
    """Algorithmic work of a stage over P slices: (bound, amount, unit, peak).

    Per-unit figures (per slice unless noted; L = N + M):
      project       FP32: 2 d flops per point-slice -> 2 (N+M) d P flops (FP32 MFMA);
                    split-BF16: the three BF16 products hi.hi + hi.lo + lo.hi of each
                    FP32 product -> 3 x 2 (N+M) d P flops (BF16 MFMA)
      sort_group    8 B (key, index) per entry + 4 B weight per source + 4 B t per target
      sort_hist     4 B projection per entry + 4 B weight per source
      sort_scatter  4 B projection read + 8 B (key, index) write per entry
      nfft_spread   4 B projection + 4 B weight per source
      nfft_interp   4 B projection read + 4 B t write per target
      split_points  once per call, not per slice: 4 B read + 4 B (bf16 hi + lo) written per
                    point coordinate -> 8 (N+M) d bytes (split-BF16 plans with P > 2048)
      accumulate    4 B t per target-slice read
      backproject   2 P flops per output coordinate     -> 2 R P d flops per launch, R = M (grad_y)
                    or N (grad_x); counted as (N + M) P d, the mean of the two launches (MFMA FP32)
    The amount over all launches of a step divided by their summed duration is the
    achieved rate (the per-launch work times the launches over the same time).
    """
    N, M, d = wl.N, wl.M, wl.d
    L = N + M
    if stage == "project":
        if precision == "split_bf16":
            return "mfma", 6.0 * L * d * P / 1e12, "TFLOP/s", PEAK_BF16_MFMA_TFLOPS
        return "mfma", 2.0 * L * d * P / 1e12, "TFLOP/s", PEAK_FP32_MFMA_TFLOPS
    if stage == "backproject":
        return "mfma", 1.0 * L * d * P / 1e12, "TFLOP/s", PEAK_FP32_MFMA_TFLOPS
    if stage == "split_points":
        return "hbm", 8.0 * L * d / 1e9, "GB/s", PEAK_HBM_GBS
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
    "split_points": ("split_points_kernel", "k_project_bf16.hip"),
}
# split-BF16 projection: split inside the GEMM, or (P > TILED_MIN_P) fed from the
# once-per-call step-tiled split by direct LDS copies
PROJECT_BF16 = ("proj_gemm_bf16x3_kernel", "k_project_bf16.hip")
PROJECT_BF16_TILED = ("proj_gemm_bf16x3_dma_kernel", "k_project_bf16.hip")
TILED_MIN_P = 2048


def stage_kernel(stage, precision, P=0):
    if stage == "project" and precision == "split_bf16":
        return PROJECT_BF16_TILED if P > TILED_MIN_P else PROJECT_BF16
    return STAGE_KERNEL.get(stage)


def workload_tag(wl, P, precision):
    """Name of a workload's profile summaries: workload, sizes, slice count and precision."""
    return f"{wl.name}_N{wl.N}_d{wl.d}_P{P}_{precision}"


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


def measured_traffic(tag, stage, precision, launches, P=0):
    """HBM bytes per launch of a stage's kernel from the committed FETCH_SIZE / WRITE_SIZE
    summary profiles/hbm_traffic_<tag>.md (already scaled by the copy-kernel calibration
    and given per launch), or None when there is no summary or the kernel's source
    differs from the one the counters were taken with."""
    sk = stage_kernel(stage, precision, P)
    if sk is None:
        return None
    kname, src = sk
    path = os.path.join(ROOT, "profiles", f"hbm_traffic_{tag}.md")
    if not os.path.exists(path):
        return None
    rd = wr = None
    digest = None
    with open(path) as f:
        for line in f:
            head = "| `" + kname
            if line.startswith(head) and line[len(head):len(head) + 1] in ("`", "<"):
                cols = [c.strip() for c in line.strip().strip("|").split("|")]
                rd, wr = float(cols[3]), float(cols[4])
            elif line.startswith("- source-digest " + src + " "):
                digest = line.split()[-1]
    if rd is None or digest != source_digest(src):
        return None
    return {"read_GB": rd, "write_GB": wr, "total_GB": rd + wr, "source": os.path.relpath(path, ROOT)}


def worker_threads():
    """Threads for the CPU leg: the cores this process may run on, at most 16 (the host
    share of one GPU)."""
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:  # pragma: no cover
        n = os.cpu_count() or 1
    return max(1, min(16, n))


def cpu_baseline(wl, x64, y64, w, sigma, xi, t_gpu, budget_s, threads):
    """The FP64 oracle on the first Q slices, threads over slices (each thread runs the
    oracle's sliced sum on its own block of directions, BLAS single-threaded), and the
    GPU's per-slice sums against it on those slices."""
    from concurrent.futures import ThreadPoolExecutor

    from threadpoolctl import threadpool_limits

    from oracle import sliced

    method = "sort" if wl.kernel == "negdist" else wl.method

    def block(q0, q1):
        return sliced.sliced_sum(wl.kernel, x64, y64, w, xi[q0:q1], sigma, method, wl.n_coeff, wl.T,
                                 return_slices=True)[1]

    def run(Q):
        nt = min(threads, Q)
        cut = np.linspace(0, Q, nt + 1).astype(int)
        with threadpool_limits(limits=1), ThreadPoolExecutor(max_workers=nt) as ex:
            t0 = time.perf_counter()
            parts = list(ex.map(lambda ab: block(*ab), zip(cut[:-1], cut[1:])))
            dt = time.perf_counter() - t0
        return np.concatenate(parts, axis=0), dt, nt

    # one slice per thread sizes the sample, then as many rounds as the budget allows
    q1 = min(threads, wl.P)
    _, dt1, _ = run(q1)
    rounds = max(1, int(budget_s / max(dt1, 1e-3)))
    Q = int(min(wl.P, q1 * rounds))
    ts, dt, nt = run(Q)
    out = {"value": wl.M * Q / dt, "unit": UNIT, "cores": int(nt), "kind": "oracle",
           "sample": f"first {Q} of {wl.P} slices at full N={wl.N}, M={wl.M}, d={wl.d}, {nt} threads over "
                     f"slices ({dt:.1f} s; FP64 projection + per-slice 1-D sum as the oracle computes it)"}
    tg = t_gpu[:Q].astype(np.float64)
    par = {"parity_rel_l2_vs_oracle": sliced.rel_l2(tg, ts),
           "parity_max_elementwise_vs_oracle": float(np.max(np.abs(tg - ts)) / np.max(np.abs(ts))),
           "parity_slices": Q}
    return out, par


def exact_error(s, exact, w, signed):
    """The gate metric: relative l2 error for non-negative weights, the paper's
    per-summand error for signed weights (Sec. 4.1)."""
    from oracle import sliced
    sub = np.asarray(s[:exact.shape[0]], dtype=np.float64)
    return sliced.per_summand_error(sub, exact, w) if signed else sliced.rel_l2(sub, exact)


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


def serve_replay(n_requests, rate, slots, hbm_gb, saturated=True):
    """Replays the first n_requests of the serving stream on one GPU and reports latency and
    throughput:
      * served: the request server (continuous batching, `slots` concurrent streams,
        admission by HBM footprint) with the split-BF16 projection;
      * baseline: one request at a time in arrival order, FP32, on one stream;
    at the stream's arrival times and, if `saturated`, with every request queued at once.
    Point sets live in HBM: per dimension and distribution one pool of 5e5 sources and
    one of 5e5 targets, and each request takes a contiguous block of rows of each."""
    import torch
    import paper_2401_08260_amd as ks

    reqs = wlm.serving_stream(n_requests, rate, seed=4)
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
    srv = ks.Server(slots=slots, hbm_bytes=int(hbm_gb * (1 << 30)))
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

    def out_bytes(i):
        r = reqs[i]
        return 4 * (r["M"] + ((r["N"] + r["M"]) * r["d"] + r["N"] if r["grad"] else 0))

    def run_served(scale, window=64, window_bytes=16 << 30):
        """Continuous batching with the split-BF16 projection; arrivals scaled by `scale`.
        scale = 0 saturates the server: requests go in as fast as it takes them, at most
        `window` outstanding whose output buffers (allocated as they are submitted) take
        at most `window_bytes` together, or one if it alone is larger.  Large requests stay
        outstanding longest, so without the byte bound the window fills with them."""
        lat, t_end_max, keep = [], 0.0, {}
        t0 = time.monotonic()
        i = pending = held = 0
        while i < len(reqs) or pending:
            now = time.monotonic() - t0
            while i < len(reqs) and reqs[i]["arrival"] * scale <= now and (
                    scale > 0 or pending == 0 or (pending < window and held + out_bytes(i) <= window_bytes)):
                x, y, w, g = inputs(i)
                s, gr = outputs(i)
                keep[i] = (s, gr)
                held += out_bytes(i)
                srv.submit(i, reqs[i]["kernel"], reqs[i]["d"], reqs[i]["P"], x, y, w, s,
                           params=params(i, "split_bf16"), grad_s=g if reqs[i]["grad"] else None, grads=gr)
                i += 1
                pending += 1
            for c in srv.poll(4096):
                if c["status"] != 0:
                    raise RuntimeError(f"request {c['tag']} failed with status {c['status']}")
                lat.append(c["t_end"] - (t0 + reqs[c["tag"]]["arrival"] * scale))
                t_end_max = max(t_end_max, c["t_end"] - t0)
                if keep.pop(c["tag"], None) is not None:
                    held -= out_bytes(c["tag"])
                pending -= 1
            time.sleep(5e-5)
        st = srv.stats()
        return summary(lat, t_end_max - reqs[0]["arrival"] * scale,
                       {"precision": "split_bf16", "slots": slots,
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
    log(f"[serve] {len(reqs)} requests, served at {rate:g} req/s: p50 {served['p50_ms']:.2f} ms "
        f"p99 {served['p99_ms']:.2f} ms, {served['value']:.3e} {UNIT} over {served['makespan_s']:.2f} s")
    base = run_baseline(1.0)
    log(f"[serve] one at a time at {rate:g} req/s: p50 {base['p50_ms']:.2f} ms "
        f"p99 {base['p99_ms']:.2f} ms, {base['value']:.3e} {UNIT} over {base['makespan_s']:.2f} s")
    out = {"requests": len(reqs), "rate_per_s": rate, "plans": len(first_of), "served": served,
           "one_at_a_time_fp32": base, "p50_speedup": base["p50_ms"] / served["p50_ms"],
           "p99_speedup": base["p99_ms"] / served["p99_ms"]}
    if saturated:
        served_sat = run_served(0.0)
        log(f"[serve] served, saturated (<= 64 outstanding, <= 16 GiB of outputs): "
            f"{served_sat['value']:.3e} {UNIT} over {served_sat['makespan_s']:.2f} s")
        base_sat = run_baseline(0.0)
        log(f"[serve] one at a time, back to back: {base_sat['value']:.3e} {UNIT} "
            f"over {base_sat['makespan_s']:.2f} s")
        out["saturated"] = {"served": served_sat, "one_at_a_time_fp32": base_sat,
                            "throughput_speedup": served_sat["value"] / base_sat["value"]}
    srv.close()
    del plans, pools
    torch.cuda.empty_cache()
    return out


def graph_probe():
    """`--graph-probe`: what a HIP graph would save a served request.  For small and
    medium requests of each path: median latency of one call waiting for its result,
    launched directly or replayed from a graph captured once, the same back to back,
    and the host cost of capturing and instantiating a graph (what a request pays when
    no earlier request had its shape and buffers)."""
    import torch
    import paper_2401_08260_amd as ks

    dev = torch.device("cuda:0")
    rows = []
    cases = (("negdist", {}), ("laplacian", dict(sigma=5.0, n_coeff=256, T=0.125)),
             ("gaussian", dict(sigma=5.0, n_coeff=128, T=0.02, method="nfft", oversample=2, window_m=6)))
    for kernel, kw in cases:
        for n in (1000, 10000, 100000):
            gen = torch.Generator(device=dev)
            gen.manual_seed(1)
            x = torch.rand((n, 128), device=dev, generator=gen)
            y = torch.rand((n, 128), device=dev, generator=gen)
            w = torch.rand(n, device=dev, generator=gen)
            plan = ks.Plan(128, 64, kernel, seed=64, **kw)
            s = torch.empty(n, device=dev)
            st = torch.cuda.Stream()

            def med(fn, reps=50):
                t = []
                for _ in range(reps):
                    t0 = time.perf_counter()
                    fn()
                    st.synchronize()
                    t.append(time.perf_counter() - t0)
                return 1e6 * float(np.median(t))

            def b2b(fn, reps=100):
                t0 = time.perf_counter()
                for _ in range(reps):
                    fn()
                st.synchronize()
                return 1e6 * (time.perf_counter() - t0) / reps

            with torch.cuda.stream(st):
                for _ in range(3):
                    plan(x, y, w, out=s)
                direct = lambda: plan(x, y, w, out=s)
                r = {"kernel": kernel, "N": n, "M": n, "d": 128, "P": 64,
                     "direct_p50_us": med(direct), "direct_b2b_us": b2b(direct)}
                gr = torch.cuda.CUDAGraph()
                with torch.cuda.graph(gr, stream=st):
                    plan(x, y, w, out=s)
                st.synchronize()
                r["graph_p50_us"] = med(gr.replay)
                r["graph_b2b_us"] = b2b(gr.replay)
                t0 = time.perf_counter()
                for _ in range(10):
                    g2 = torch.cuda.CUDAGraph()
                    with torch.cuda.graph(g2, stream=st):
                        plan(x, y, w, out=s)
                r["capture_instantiate_us"] = 1e6 * (time.perf_counter() - t0) / 10
            log(f"[graph] {kernel:9s} N=M={n:6d}: direct {r['direct_p50_us']:.1f} us ({r['direct_b2b_us']:.1f} "
                f"back to back), graph {r['graph_p50_us']:.1f} us ({r['graph_b2b_us']:.1f}), capture + "
                f"instantiate {r['capture_instantiate_us']:.1f} us")
            rows.append(r)
            del plan
    print(json.dumps({"graph_probe": rows}), flush=True)


def bench_serve(args):
    """`--workload serve`: the serving replay as its own bench line."""
    r = serve_replay(args.serve_requests, args.serve_rate, args.serve_slots, args.serve_hbm_gb, saturated=True)
    served = r["served"]
    result = {
        "metric": METRIC, "value": served["value"], "unit": UNIT, "n_gpus": 1, "steps": r["requests"],
        "warmup": r["plans"],
        "ms_per_step": 1e3 * served["makespan_s"] / r["requests"], "p50_ms": served["p50_ms"],
        "p99_ms": served["p99_ms"], "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32+split_bf16", "data": "synthetic",
        "config": {"workload": "serve", "requests": r["requests"], "rate_per_s": args.serve_rate, "seed": 4,
                   "N_M": "log-uniform [1e3, 5e5]", "d": list(SERVE_D), "P": [64, 256],
                   "kernels": ["gaussian", "laplacian", "negdist"], "grad_fraction": 0.3},
    }
    result.update({k: v for k, v in r.items() if k not in ("requests", "rate_per_s", "plans")})
    print(json.dumps(result), flush=True)


def timed_steps(step, K, W, stream):
    """W untimed steps, then K steps bracketed by a synchronisation on both sides, with an
    event after each step on the execution stream.  Returns (per-step ms, mean ms, wall s)."""
    import torch
    for _ in range(W):
        step()
    torch.cuda.synchronize()
    evs = [torch.cuda.Event(enable_timing=True) for _ in range(K + 1)]
    torch.cuda.synchronize()
    t_wall = time.perf_counter()
    evs[0].record(stream)
    for i in range(K):
        step()
        evs[i + 1].record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t_wall
    per = np.array([evs[i].elapsed_time(evs[i + 1]) for i in range(K)])
    return per, float(evs[0].elapsed_time(evs[-1])) / K, wall


def stage_breakdown(ks, plan, step, steps=1):
    """Per-stage kernel time of `steps` steps with HIP events on the execution stream
    (read back after every step): {stage: (ms per step, launches per step)}."""
    import torch
    ks.ksum_set_timing(plan.handle, True)
    torch.cuda.synchronize()
    for _ in range(steps):
        step()
        st = ks.ksum_stage_times(plan.handle)
    ks.ksum_set_timing(plan.handle, False)
    return {k: (v[0] / steps, v[1] / steps) for k, v in st.items() if v[1] > 0}


def roofline_of(stages, wl, P, precision, ms_step, tag):
    """The stage with the largest share of the step among those with an algorithmic
    work figure, against its roofline."""
    dom = max((k for k in stages if kernel_work(k, wl, P, precision)), key=lambda k: stages[k][0])
    bound, amount, unit, peak = kernel_work(dom, wl, P, precision)
    ms, launches = stages[dom]
    achieved = amount / (ms * 1e-3)
    tr = measured_traffic(tag, dom, precision, launches, P)
    return {"kernel": dom, "kernel_name": stage_kernel(dom, precision, P)[0], "bound": bound, "achieved": achieved,
            "peak": peak, "unit": unit, "frac": achieved / peak,
            "traffic": tr["total_GB"] if tr else None,
            "traffic_unit": "GB per launch (FETCH_SIZE + WRITE_SIZE, copy-calibrated)", "traffic_detail": tr,
            "avg_launch_ms": ms / launches, "launches_per_step": launches,
            "work_per_launch": amount / launches, "share_of_step": ms / ms_step}


def stage_rooflines(stages, wl, P, precision, tag, stream_gbps):
    """Every stage with a work figure against its roofline; HBM-bound stages also with the
    measured traffic of the committed counter summary where it matches the source."""
    out = {}
    for k, (ms, launches) in stages.items():
        kw = kernel_work(k, wl, P, precision)
        if not kw:
            continue
        b, amt, u, pk = kw
        ach = amt / (ms * 1e-3)
        ent = {"bound": b, "ms_per_step": ms, "launches_per_step": launches, "achieved": ach, "unit": u,
               "frac_peak": ach / pk}
        trk = measured_traffic(tag, k, precision, launches, P)
        if b == "hbm" and trk:
            gbs = trk["total_GB"] * launches / (ms * 1e-3)
            ent.update(measured_GBps=gbs, frac_peak_measured=gbs / PEAK_HBM_GBS,
                       frac_stream_measured=gbs / stream_gbps)
        out[k] = ent
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="laplace", choices=sorted(wlm.WORKLOADS) + ["serve"])
    ap.add_argument("--serve-requests", type=int, default=20000)
    ap.add_argument("--serve-rate", type=float, default=200.0)
    ap.add_argument("--serve-slots", type=int, default=8)
    ap.add_argument("--serve-hbm-gb", type=float, default=64.0)
    ap.add_argument("--serve-in-line", type=int, default=1000,
                    help="requests of the serving stream replayed at its arrival rate for the line's `serving` "
                         "field (0 = none)")
    ap.add_argument("--cpu-budget", type=float, default=15.0, help="seconds of oracle work in the CPU leg")
    ap.add_argument("--exact-targets", type=int, default=2000)
    ap.add_argument("--fp32-steps", type=int, default=3, help="timed steps of the plain FP32 form at P*")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-gate", action="store_true",
                    help="time the workload's own P instead of P* (no exact sum; stage detail and profiles)")
    ap.add_argument("--precision", default="split_bf16", choices=["split_bf16", "fp32"],
                    help="form of the headline (the other is timed beside it)")
    ap.add_argument("--backward", action="store_true",
                    help="also time one gradient step (grad_x, grad_y, grad_w for an upstream grad_s) at P")
    ap.add_argument("--graph-probe", action="store_true",
                    help="only measure what replaying a captured HIP graph saves a small request")
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

    if args.graph_probe:
        graph_probe()
        return
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
    stream = torch.cuda.current_stream(dev)
    signed = bool(np.any(w < 0))
    err_key = "per_summand" if signed else "rel_l2"
    head, other = args.precision, ("fp32" if args.precision == "split_bf16" else "split_bf16")

    # the exact sum on the first targets (FP64, CPU): the error of every run below
    exact = None
    if not args.no_gate:
        from oracle import direct
        k = min(args.exact_targets, wl.M)
        t0 = time.perf_counter()
        exact = direct.direct_sum(wl.kernel, x, y[:k], w, sigma if sigma > 0 else 1.0)
        dte = time.perf_counter() - t0
        log(f"[bench] exact sum on {k} targets: {dte:.1f} s ({k * wl.N / dte:.3e} pairs/s)")

    # the workload's own P: one run per form (error at P, stage detail, the probe for the CPU leg)
    at_P = {}
    probe_t = None
    for prec in (head, other):
        plan = ks.Plan(wl.d, wl.P, wl.kernel, **plan_kwargs(wl, sigma, prec))
        s = torch.empty(wl.M, dtype=torch.float32, device=dev)
        per, ms, _ = timed_steps(lambda: plan(xt, yt, wt, out=s), max(1, min(args.steps, 5)), 1, stream)
        ent = {"P": wl.P, "ms_per_step": ms, "value": wl.M * wl.P / (ms * 1e-3)}
        if exact is not None:
            ent["error"] = exact_error(s.cpu().numpy(), exact, w, signed)
        if prec == "fp32" and not args.no_cpu_baseline:
            probe_t = torch.empty((wl.P, wl.M), dtype=torch.float32, device=dev)
            plan(xt, yt, wt, out=s, probe={"t": probe_t})
            torch.cuda.synchronize()
            probe_t = probe_t.cpu().numpy()
            xi = plan.directions()
        at_P[prec] = ent
        log(f"[bench] P={wl.P} {prec}: {ms:.3f} ms, {ent['value']:.4e} {UNIT}"
            + (f", {err_key} error {ent['error']:.3e}" if "error" in ent else ""))
        del plan

    # P*: the slice count at which the slicing error reaches the gate
    if args.no_gate:
        Pstar, batch = wl.P, 0
    else:
        e_P = at_P["fp32"]["error"]
        Pstar = wl.P if e_P <= GATE else int(math.ceil(wl.P * (e_P / GATE) ** 2 * 1.2 / GATE_BATCH)) * GATE_BATCH
        batch = GATE_BATCH if Pstar > wl.P else 0
    log(f"[bench] timed slice count P* = {Pstar}" + (f" (batches of {batch})" if batch else ""))

    forms = {}
    stream_pk = measure_stream_peak(dev)
    for prec, K, W in ((head, args.steps, args.warmup), (other, max(1, min(args.fp32_steps, args.steps)), 1)):
        plan = ks.Plan(wl.d, Pstar, wl.kernel, slice_batch=batch, **plan_kwargs(wl, sigma, prec))
        s = torch.empty(wl.M, dtype=torch.float32, device=dev)

        def step():
            plan(xt, yt, wt, out=s)

        per, ms, wall = timed_steps(step, K, W, stream)
        tag = workload_tag(wl, Pstar, prec)
        stages = stage_breakdown(ks, plan, step, 1)
        ent = {"precision": prec, "P": Pstar, "steps": K, "warmup": W, "ms_per_step": ms, "wall_s": wall,
               "value": wl.M * Pstar / (ms * 1e-3), "p50_ms": float(np.percentile(per, 50)),
               "p99_ms": float(np.percentile(per, 99)),
               "stage_ms_per_step": {k: v[0] for k, v in stages.items()},
               "roofline": roofline_of(stages, wl, Pstar, prec, ms, tag),
               "stage_roofline": stage_rooflines(stages, wl, Pstar, prec, tag, stream_pk["GBps"]),
               "profile_tag": tag}
        if exact is not None:
            ent["error"] = exact_error(s.cpu().numpy(), exact, w, signed)
            ent["meets_gate"] = bool(ent["error"] <= GATE)
        forms[prec] = ent
        log(f"[bench] P*={Pstar} {prec}: {ms:.3f} ms/step over {K} steps ({wall / K * 1e3:.3f} ms wall), "
            f"{ent['value']:.4e} {UNIT}" + (f", {err_key} error {ent['error']:.3e}" if "error" in ent else ""))
        for kname in sorted(stages, key=lambda q: -stages[q][0]):
            log(f"[bench]   {kname:14s} {stages[kname][0]:9.4f} ms/step  ({stages[kname][1]:.0f} launches/step)")
        del plan

    # (--backward) the gradients of an MMD gradient-flow step at the workload's P, FP32
    backward = None
    if args.backward:
        plan = ks.Plan(wl.d, wl.P, wl.kernel, **plan_kwargs(wl, sigma, "fp32"))
        gs = torch.from_numpy(np.random.default_rng(7).standard_normal(wl.M).astype(np.float32)).to(dev)
        per, ms_b, _ = timed_steps(lambda: plan.backward(xt, yt, wt, gs), args.steps, args.warmup, stream)
        st_b = stage_breakdown(ks, plan, lambda: plan.backward(xt, yt, wt, gs), 1)
        backward = {"what": "grad_x, grad_y and grad_w of s for an upstream grad_s, FP32, at the workload's P",
                    "P": wl.P, "ms_per_step": ms_b, "stage_ms_per_step": {k: v[0] for k, v in st_b.items()}}
        if "backproject" in st_b:
            bms, bl = st_b["backproject"]
            # the work is per launch (the mean of the grad_y and grad_x launches): rate per launch
            b_bound, b_amt, b_unit, b_pk = kernel_work("backproject", wl, wl.P)
            b_rate = b_amt / (bms / bl * 1e-3)
            backward["backproject_roofline"] = {"bound": b_bound, "avg_launch_ms": bms / bl, "launches": bl,
                                                "achieved": b_rate, "peak": b_pk, "unit": b_unit,
                                                "frac": b_rate / b_pk}
        log(f"[bench] backward (grad_x, grad_y, grad_w) at P={wl.P}: {ms_b:.3f} ms/step")
        del plan

    hd = forms[head]
    result = {
        "metric": METRIC, "value": hd["value"], "unit": UNIT, "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": hd["ms_per_step"], "p50_ms": hd["p50_ms"], "p99_ms": hd["p99_ms"],
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "bf16" if head == "split_bf16" else "f32", "data": "synthetic",
        "config": {"workload": wl.name, "kernel": wl.kernel, "method": "sort" if wl.kernel == "negdist"
                   else wl.method, "N": wl.N, "M": wl.M, "d": wl.d, "P": Pstar, "slice_batch": batch,
                   "P_workload": wl.P, "precision": head, "input": wl.dtype, "sigma": sigma,
                   "error_metric": err_key, "exact_targets": int(exact.shape[0]) if exact is not None else 0},
        "error": hd.get("error"), "meets_gate": hd.get("meets_gate"),
        "roofline": hd["roofline"],
        "stage_ms_per_step": hd["stage_ms_per_step"],
        "stage_roofline": hd["stage_roofline"],
        "forms": forms,
        "mixed_vs_fp32": forms["fp32"]["ms_per_step"] / forms["split_bf16"]["ms_per_step"],
        "at_workload_P": at_P,
        "stream_peak": stream_pk,
    }
    if backward is not None:
        result["backward"] = backward
    if args.serve_in_line > 0:
        # free this workload's device memory before the serving pools are drawn
        del xt, yt, wt
        torch.cuda.empty_cache()
        result["serving"] = serve_replay(args.serve_in_line, args.serve_rate, args.serve_slots, args.serve_hbm_gb,
                                         saturated=False)
    if not args.no_cpu_baseline:
        x64, y64 = x.astype(np.float64), y.astype(np.float64)
        base, par = cpu_baseline(wl, x64, y64, w, sigma, xi, probe_t, args.cpu_budget, worker_threads())
        result["cpu_baseline"] = base
        result["parity_vs_oracle"] = par
        log(f"[bench] cpu baseline {base['value']:.3e} {UNIT} ({base['sample']}); parity {par}")
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
