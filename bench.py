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
    """
    N, M, d = wl.N, wl.M, wl.d
    L = N + M
    if stage == "project":
        return "mfma", 2.0 * L * d * P / 1e12, "TFLOP/s", PEAK_FP32_MFMA_TFLOPS
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
    # size the sample: one slice first, then as many as the budget allows
    t0 = time.perf_counter()
    _, ts1 = sliced.sliced_sum(wl.kernel, x, y, w, xi[:1], sigma, method, wl.n_coeff, wl.T, return_slices=True)
    one = time.perf_counter() - t0
    Q = int(max(1, min(wl.P, budget_s / max(one, 1e-3))))
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
    return out, errs


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="negdist", choices=sorted(wlm.WORKLOADS))
    ap.add_argument("--cpu-budget", type=float, default=15.0, help="seconds of oracle work in the CPU leg")
    ap.add_argument("--exact-targets", type=int, default=500)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-mixed", action="store_true", help="skip the split-BF16 (mixed) leg")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="only copy 1 GiB device to device (reference for the HBM traffic counters)")
    args = ap.parse_args()

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        log("bench.py measures one GPU: this build has no multi-GPU path "
            "(slices would be sharded across GPUs with one all-reduce of s; see the design notes).")
        sys.exit(2)

    import torch
    import paper_2401_08260_amd as ks

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
        "mixed": mixed,
    }

    if not args.no_cpu_baseline:
        probe_t = torch.empty((wl.P, wl.M), dtype=torch.float32, device=dev)
        plan(xt, yt, wt, out=s, probe={"t": probe_t})
        torch.cuda.synchronize()
        base, errs = cpu_baseline(wl, x, y, w, sigma, plan.directions(), s.cpu().numpy(),
                                  probe_t.cpu().numpy(), args.cpu_budget,
                                  args.exact_targets, s_mixed)
        result["cpu_baseline"] = base
        result["errors"] = errs
        log(f"[bench] cpu baseline {base['value']:.3e} {UNIT} ({base['sample']}); errors {errs}")
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
