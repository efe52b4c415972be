#!/usr/bin/env python3
"""Throughput of the fast kernel-regression hot path on one MI355X.

Headline workload (``--workload ll3d``, the default): 3-D local linear
regression with the heteroscedastic-variance second pass, N = 1e7 samples
x ~ U[0,1]^3, y = |x|^2 + (0.1 + 0.5 x1) e, h = 0.05 in every dimension,
M = 128^3 grid, eps = 1e-6, FP32 spreading, FP64 transforms and FP64 4x4
solves, seeded and synthetic.  One step is one pass of the whole path:

  set_points   bin and sort the samples (once per X)
  cv           spread of density, y and 10 Philox probes -> forward FFTs ->
               moment channels -> FP64 solves -> interpolation -> Girard DF,
               RSS and GCV over the supported samples (Sec. 2.1, eq. 22)
  variance     log-residual second pass (eq. 24-26): residuals, spread,
               FFTs, solves, kappa, sigma^2 on the grid

``--workload ll2d`` runs the 2-D mixture configuration (N = 1e6, M = 256^2,
h = (0.03, 0.05)) the same way; its working set (about 217 MB) fits the
256 MB Infinity Cache, so its HBM fractions are labelled cache-resident.

The headline value is samples/s = N x fits / step time, where a fit is one
weight vector through spread + FFT + solve (1 response + 10 probes + 1
variance pass = 12 per step).  ``roofline`` reports the dominant kernel, the
cv call's spreading launch, against FP32 FMA issue with its algorithmic flops
(2 w^d flops per sample and weight column) and against HBM with its
algorithmic bytes, timed with the HIP events the library records on the
launch stream; ``hbm_model`` sets the step's algorithmic bytes against HBM
bandwidth; ``cpu_baseline`` times the FP64 oracle on a bounded sample of grid
points and extrapolates to the full grid; ``accuracy`` compares the GPU grids
with the oracle on that sample; ``fp64_single`` times the plain FP64 form
(FP64 spreading, transforms and solves) of one regression on the same
samples, replayed as a HIP graph like the batched step, with its own error.

The timed steps replay a HIP graph captured from one step (the step's
launches are launch-bound on the host otherwise); before timing, replays are
compared with eager steps.  ``--eager`` times host-launched steps instead.
Stage times always come from eager steps, where the library brackets every
launch with HIP events on the launch stream.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload ll3d|ll2d]
                       [--transform fp64|fp32] [--eager] [--no-warm]
                       [--no-cpu-baseline] [--no-fp64-single] [--cpu-points G]
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import platform
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
# FP32 FMA issue: 256 CUs x 4 SIMDs x 16 lanes x 2 flops x 2.4 GHz (packed
# FP32 off); the published 157.3 TFLOP/s counts two FMAs per lane per cycle.
FP32_FMA_PEAK_TFLOPS = 78.6
FP32_PUBLISHED_TFLOPS = 157.3
# dense FP32 MFMA: 256 CUs x 4 SIMDs x 64 flops x 2.4 GHz
FP32_MFMA_PEAK_TFLOPS = 157.3
KERNEL_SOURCE = os.path.join(ROOT, "paper_2204_07716_amd", "csrc", "kernels.hip")
COUNTERS = {"ll3d": os.path.join(ROOT, "profiles", "k_spread_col3_ll3d_counters.json"),
            "ll2d": os.path.join(ROOT, "profiles", "k_spread_ll2d_counters.json")}
LABEL = {
    "ll3d": "3-D local linear + log-variance pass, N=1e7 uniform, h=0.05, M=128^3, eps=1e-6, "
            "10 Philox probes",
    "ll2d": "2-D local linear + log-variance pass, N=1e6 mixture, h=(0.03,0.05), M=256x256, "
            "eps=1e-6, 10 Philox probes (cache-resident: working set < 256 MB Infinity Cache)",
}


def _args():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", choices=["ll3d", "ll2d"], default="ll3d")
    ap.add_argument("--transform", choices=["fp64", "fp32"], default="fp64",
                    help="precision of the FFTs and moment channels (spreading is FP32)")
    ap.add_argument("--sigma", type=float, default=0.0,
                    help="oversampling of the spreading grid (0: the plan's default)")
    ap.add_argument("--eager", action="store_true",
                    help="launch every step's kernels from the host instead of replaying a HIP graph")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-fp64-single", action="store_true",
                    help="skip timing the plain FP64 single-regression form")
    ap.add_argument("--no-warm", action="store_true",
                    help="skip the warm-path timing (profiling runs count only the cold steps)")
    ap.add_argument("--cpu-points", type=int, default=0,
                    help="grid points per pass in the oracle's timed sample (0: 512 in 3-D, 2048 in 2-D)")
    ap.add_argument("--no-batch", action="store_true",
                    help="skip the batch workload (256 independent regressions; 64-probe x 32-bandwidth DF sweep)")
    ap.add_argument("--no-kernels", action="store_true",
                    help="skip the kernel and bandwidth generality timing (full H, compact kernels)")
    ap.add_argument("--no-grad", action="store_true",
                    help="skip the differentiated workload (GCV and its gradients, complex y, N=4e6)")
    ap.add_argument("--no-inference", action="store_true",
                    help="skip the variance-of-fit / band / spline-prediction timing")
    ap.add_argument("--copy-probe", action="store_true",
                    help="after the run, copy a 256 MiB buffer once (counter calibration)")
    return ap.parse_args()


# Source region of the cv spread kernel of each workload (its launcher
# included): the committed counters stay valid while that text is unchanged.
KERNEL_REGION = {"ll3d": ("// 3-D spread on the matrix cores", "static void spread_wave("),
                 "ll2d": ("// 2-D spread with one sample stream per wave", "// 3-D spread on the matrix cores")}


def _kernel_hash(workload: str) -> str:
    with open(KERNEL_SOURCE, "rb") as f:
        src = f.read().decode()
    a, b = KERNEL_REGION[workload]
    i = src.index(a)
    j = src.index(b, i)
    return hashlib.sha256(src[i:j].encode()).hexdigest()


def _traffic(workload: str):
    """HBM bytes per launch of the cv spread from the committed counter run,
    or None when the kernel source has changed since the counters were taken."""
    try:
        with open(COUNTERS[workload]) as f:
            c = json.load(f)
    except (OSError, ValueError):
        return None
    if c.get("kernel_source_sha256") != _kernel_hash(workload):
        return None
    try:
        return (c["fetch_kib_per_launch"] * 1024 * c["copy_fetch_scale"]
                + c["write_kib_per_launch"] * 1024 * c["copy_write_scale"])
    except (KeyError, TypeError):
        return None


import numpy as np  # noqa: E402  (host arithmetic of the byte model)


def _pass_bytes(npair, n_in, n_out, rows_in, b):
    """Bytes one transform pass moves: rows_in x n_in read, rows_in x n_out written."""
    return npair * rows_in * (n_in + n_out) * b


def _hbm_model(g, d, N, M, n_s, n_t, Np, n_jobs, stages, steps, ms_per_step, cache_resident):
    """Algorithmic bytes of the step for the plan actually run (sort, spread
    with its tile subgrids, forward passes with the fold, inverse passes from
    the band to the grid, solve), FP32 spreading and FP64 complex transforms,
    against HBM bandwidth: for spread + forward FFT and for the whole step."""
    Mr = [g.Mr[j] for j in range(d)]
    B = [2 * g.K[j] + 1 for j in range(d)]
    Mg = list(M)
    psub = (g.tile[0] + g.w - 1) ** d
    bx, bw, bs, bt = 4, 4, 8, 16
    b_sort = N * (d * bx + 4 * 8 + 32)                      # read X, write + read the tile record, write the sorted record
    calls = [dict(nw=2 + Np, ncp=(n_s + n_t * (1 + Np) + 1) // 2, keep=0, nsol=n_s + n_t * (1 + Np) + 1 + Np),
             dict(nw=2, ncp=(n_s + n_t + 1) // 2, keep=n_s // 2, nsol=n_s + n_t + 1)]   # cv, variance
    b_spread = b_fft = b_inv = b_solve = 0
    for c in calls:
        npair = (c["nw"] + 1) // 2
        b_spread += N * (d * bx + c["nw"] * bw) + n_jobs * npair * psub * bs    # samples in, subgrids out
        # forward: pass j reads its rows (the fold reads the subgrids) and keeps the band
        shape = list(Mr)
        fwd = n_jobs * npair * psub * bs
        for j in range(d):
            rows = 1
            for i in range(d):
                if i != j:
                    rows *= shape[i]
            fwd += _pass_bytes(npair, 0 if j == 0 else shape[j], B[j], rows, bt)
            shape[j] = B[j]
        b_fft += fwd
        # inverse: channel spectra from the pair spectra (pair band in,
        # channel band out), then band -> grid along dimensions d-1 .. 0
        ncp = c["ncp"] - c["keep"]
        shape = list(B)
        inv = (npair + ncp) * int(np.prod(B)) * bt
        for j in reversed(range(d)):
            rows = 1
            for i in range(d):
                if i != j:
                    rows *= shape[i]
            inv += _pass_bytes(ncp, shape[j], Mg[j], rows, bt)
            shape[j] = Mg[j]
        b_inv += inv
        b_solve += c["nsol"] * int(np.prod(Mg)) * 8
    t_sf = sum(stages[k][0] for k in ("spread", "fold", "fft_fwd")) * 1e-3 / steps
    b_all = b_sort + b_spread + b_fft + b_inv + b_solve
    out = {"spread_fft": {"bytes": b_spread + b_fft, "ms": round(t_sf * 1e3, 4),
                          "frac": round((b_spread + b_fft) / t_sf / 8e12, 4)},
           "whole_step": {"bytes": b_all, "ms": round(ms_per_step, 4),
                          "frac": round(b_all / (ms_per_step * 1e-3) / 8e12, 4)},
           "stage_bytes": {"sort": b_sort, "spread": b_spread, "fft_fwd": b_fft, "fft_inv": b_inv,
                           "solve": b_solve},
           "peak_GBs": HBM_PEAK_GBS}
    if cache_resident:
        out["cache_resident"] = True
    return out


def _cpu_info():
    model = platform.processor() or ""
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return model, os.cpu_count()


def main() -> int:
    args = _args()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(json.dumps({"error": "this benchmark runs on one GPU only: the path is not "
                          "sharded across GPUs", "n_gpus": args.gpus}))
        return 2

    import numpy as np
    import torch

    import workloads
    from paper_2204_07716_amd import Plan

    if not torch.cuda.is_available():
        print(json.dumps({"error": "no GPU visible"}))
        return 1
    dev = torch.device("cuda:0")
    w = workloads.make(args.workload)
    d, N, M, h = w.d, w.N, w.M, w.h[0]
    Np, seed = w.n_probes, w.probe_seed
    Xd = torch.as_tensor(w.X.astype(np.float32), device=dev)
    Yd = torch.as_tensor(w.Y.astype(np.float32), device=dev)
    plan = Plan(d, 1, M, w.lo, w.hi, h, h, w.eps, precision="fp32", n_max=N,
                max_weights=2 + Np, max_h=1, transform_precision=args.transform, sigma=args.sigma)
    g = plan.geometry
    torch.cuda.synchronize()

    def step():
        plan.set_points(Xd)
        out = plan.cv(h, Yd, Np, seed=seed)
        s2, vhat, kappa = plan.variance(h, Yd, out["mhat"][0, 0], mode="log")
        return out, s2, vhat, kappa

    def graph_of(fn):
        s_cap = torch.cuda.Stream()
        s_cap.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(s_cap):
            fn()                         # warm the capture stream's allocator pool
        torch.cuda.current_stream().wait_stream(s_cap)
        torch.cuda.synchronize()
        gr = torch.cuda.CUDAGraph()
        with torch.cuda.graph(gr):
            res = fn()
        return gr, res

    def same(a, b, rel=1e-6):
        # samples of one cell are ranked with LDS atomics, so the FP32
        # summation order (and the last bits) may differ between runs
        fin = torch.isfinite(b)
        scale = b[fin].abs().max() if fin.any() else torch.tensor(0.0, device=b.device)
        return torch.equal(torch.isnan(a), torch.isnan(b)) and \
            bool((a[fin] - b[fin]).abs().max() <= rel * scale) if fin.any() else True

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    args.graph = not args.eager
    if args.graph:
        ref = step()
        torch.cuda.synchronize()
        ref_vals = [ref[0]["mhat"].clone(), ref[0]["rho"].clone(), ref[0]["gcv"].clone(), ref[1].clone()]
        graph, res_g = graph_of(step)
        for rep in range(2):
            graph.replay()
            torch.cuda.synchronize()
            got = [res_g[0]["mhat"], res_g[0]["rho"], res_g[0]["gcv"], res_g[1]]
            if not all(same(a, b) for a, b in zip(got, ref_vals)):
                print(json.dumps({"error": "graph replay differs from the eager step", "replay": rep}))
                return 1
            step()                       # eager work between replays
            torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            graph.replay()
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        res = res_g
    else:
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            res = step()
        torch.cuda.synchronize()
        t1 = time.perf_counter()
    ms_per_step = (t1 - t0) * 1e3 / args.steps
    n_fits = (1 + Np) + 1

    # Stage times and the cv spread launch alone, from eager profiled steps
    # (HIP events the library records on the launch stream).
    plan.profile(True)
    plan.profile_read()
    stages = {k: [0.0, 0] for k in plan.profile_read()}
    cv_spread_ms, cv_spread_n = 0.0, 0
    for _ in range(args.steps):
        plan.set_points(Xd)
        out_p = plan.cv(h, Yd, Np, seed=seed)
        a = plan.profile_read()
        cv_spread_ms += a["spread"][0]
        cv_spread_n += a["spread"][1]
        plan.variance(h, Yd, out_p["mhat"][0, 0], mode="log")
        b = plan.profile_read()
        for k in stages:
            stages[k][0] += a[k][0] + b[k][0]
            stages[k][1] += a[k][1] + b[k][1]
    plan.profile(False)

    # Warm path: X already sorted, set_points outside the timed region.
    def warm_step():
        out = plan.cv(h, Yd, Np, seed=seed)
        s2, vhat, kappa = plan.variance(h, Yd, out["mhat"][0, 0], mode="log")
        return out, s2, vhat, kappa

    warm_ms = None
    if not args.no_warm:
        plan.set_points(Xd)
        warm_step()
        torch.cuda.synchronize()
        if args.graph:
            wgraph, wres = graph_of(warm_step)
            wgraph.replay()
            torch.cuda.synchronize()
            if not (same(wres[0]["mhat"], res[0]["mhat"]) and same(wres[1], res[1])):
                print(json.dumps({"error": "warm graph replay differs from the timed steps"}))
                return 1
            tw0 = time.perf_counter()
            for _ in range(args.steps):
                wgraph.replay()
            torch.cuda.synchronize()
        else:
            tw0 = time.perf_counter()
            for _ in range(args.steps):
                warm_step()
            torch.cuda.synchronize()
        warm_ms = (time.perf_counter() - tw0) * 1e3 / args.steps
    value = N * n_fits / (ms_per_step * 1e-3)

    # Roofline of the cv spread (the step's largest kernel): 2 w^d flops per
    # sample and weight column; the 3-D spread runs on FP32 MFMA (dense peak
    # 157.3 TFLOP/s), the 2-D one on FP32 FMA issue without packed math
    # (78.6 TFLOP/s).  HBM view with its algorithmic bytes
    # N (d b_x + n_w b_w) + n_pair Mr^d b_c.
    Mr = 1
    for j in range(d):
        Mr *= g.Mr[j]
    nw = 2 + Np
    flops = 2.0 * N * g.w ** d * nw
    bytes_ = N * (d * 4 + nw * 4) + ((nw + 1) // 2) * Mr * 8
    launch_s = cv_spread_ms * 1e-3 / max(cv_spread_n, 1)
    achieved = flops / launch_s / 1e12
    if d == 3:
        kname, bound, peak = "k_spread_col3 (cv: 12 columns, 3 passes of 4; FP32 MFMA 16x16x4)", "mfma", \
            FP32_MFMA_PEAK_TFLOPS
    else:
        kname, bound, peak = "k_spread_wave (cv: 12 columns; FP32 FMA)", "alu", FP32_FMA_PEAK_TFLOPS
    roofline = {"bound": bound, "kernel": kname,
                "achieved": round(achieved, 2), "peak": peak, "unit": "TFLOP/s",
                "frac": round(achieved / peak, 4),
                "traffic": _traffic(args.workload),
                "algorithmic_flops_per_launch": flops,
                "algorithmic_bytes_per_launch": bytes_,
                "avg_launch_us": round(launch_s * 1e6, 2),
                "launches_measured": cv_spread_n,
                "hbm": {"achieved": round(bytes_ / launch_s / 1e9, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                        "frac": round(bytes_ / launch_s / 1e9 / HBM_PEAK_GBS, 4)}}
    if d != 3:
        roofline["frac_of_published_fp32_157"] = round(achieved / FP32_PUBLISHED_TFLOPS, 4)

    out, s2, vhat, kappa = res
    cache_resident = args.workload == "ll2d"
    line = {
        "metric": "samples/s (spread+FFT+solve) at stated rel err vs FP64 oracle; % of HBM BW",
        "value": round(value, 1), "unit": "samples/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(ms_per_step, 4), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None,
        "dtype": "f32 spread, %s transforms, f64 solves" % ("f64" if args.transform == "fp64" else "f32"),
        "data": "synthetic (seeded, %s)" % ("x ~ U[0,1]^3, N=1e7" if d == 3 else "4-component Gaussian mixture, N=1e6"),
        "config": {"workload": LABEL[args.workload],
                   "N": N, "M": list(M), "order": 1, "fits_per_step": n_fits,
                   "grid_points_per_s": round(float(np.prod(M)) * n_fits / (ms_per_step * 1e-3), 1),
                   "L": [g.L[j] for j in range(d)], "Mr": [g.Mr[j] for j in range(d)],
                   "K": [g.K[j] for j in range(d)], "spread_width": g.w,
                   "sigma": args.sigma or "default", "hip_graph": bool(args.graph)},
        "roofline": roofline,
        "warm": None if warm_ms is None else
                {"ms_per_step": round(warm_ms, 4), "value": round(N * n_fits / (warm_ms * 1e-3), 1),
                 "unit": "samples/s", "note": "X already sorted: set_points outside the timed region"},
        "hbm_model": _hbm_model(g, d, N, M, plan.n_s, plan.n_t, Np, plan.diagnostics()["n_jobs"], stages,
                                args.steps, ms_per_step, cache_resident),
        "stages_ms_per_step": {k: round(v[0] / args.steps, 4) for k, v in stages.items()},
        "gcv": float(out["gcv"][0, 0]), "n_supported": float(out["nused"][0]),
        "df": float(out["nused"][0] * (1 - out["rho"][0].mean())),
    }

    if args.copy_probe:
        a = torch.empty(64 << 20, dtype=torch.float32, device=dev).fill_(1.0)
        b = torch.empty_like(a)
        torch.cuda.synchronize()
        b.copy_(a)
        torch.cuda.synchronize()
        line["copy_probe_bytes"] = a.numel() * 4

    if not args.no_inference:
        line["inference"] = _inference(w, Xd, Yd, args.transform, args.sigma, args.steps)
    if not args.no_batch:
        line["batch"] = _batch_workload(min(args.steps, 5))
    if not args.no_grad:
        line["differentiated"] = _grad_workload(min(args.steps, 5))
    if not args.no_kernels:
        line["kernels"] = _kernel_generality(min(args.steps, 5))

    sample = None
    if not args.no_cpu_baseline or not args.no_fp64_single:
        rng = np.random.default_rng(2024)
        Mtot = int(np.prod(M))
        G = args.cpu_points or (512 if d == 3 else 2048)
        flat = rng.choice(Mtot, size=G, replace=False)
        flat[:2] = [0, Mtot - 1]
        sample = flat
    fp64 = None
    if not args.no_fp64_single:
        fp64 = _fp64_single(w, Xd, Yd, args.steps, args.warmup, value, args.graph)
        line["fp64_single"] = fp64
    if not args.no_cpu_baseline:
        line.update(_cpu_baseline(w, out, vhat, kappa, n_fits, value, sample, fp64))
    if fp64 is not None:
        fp64.pop("_mhat", None)
    del plan
    print(json.dumps(line), flush=True)
    return 0


def _inference(w, Xd, Yd, transform, sigma, steps, n_query=1_000_000):
    """Prediction and inference on the same samples (Sec. 4 fkreg_interval and
    fkreg_predict; eq. 27-28): the variance of the fit and its 95% band for
    the log-variance pass's sigma^2 grid (one call: density moments at h and
    sigma^2-weighted moments of the squared kernel at h / sqrt 2, which the
    plan's band must cover), then the spline coefficients of the fit and its
    values at n_query points drawn over the box widened by 10% per side.
    Eager calls, timed with device synchronisation around each loop."""
    import numpy as np
    import torch
    from paper_2204_07716_amd import Plan
    h = w.h[0]
    h2 = tuple(v / np.sqrt(2.0) for v in h)
    plan = Plan(w.d, 1, w.M, w.lo, w.hi, h2, h, w.eps, precision="fp32", n_max=w.N, max_weights=2,
                max_h=1, transform_precision=transform, sigma=sigma)
    plan.set_points(Xd)
    mh = plan.fit(h, Yd)[0, 0]
    s2 = plan.variance(h, Yd, mh, mode="log")[0]
    rng = np.random.default_rng(7)
    span = np.asarray(w.hi) - np.asarray(w.lo)
    Q = rng.uniform(np.asarray(w.lo) - 0.1 * span, np.asarray(w.hi) + 0.1 * span, (n_query, w.d))
    Qd = torch.as_tensor(Q.astype(np.float32), device=Xd.device)

    def timed(fn):
        fn()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            r = fn()
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) * 1e3 / steps, r

    t_int, iv = timed(lambda: plan.interval(h, s2, mhat=mh, alpha=0.05))
    t_spl, coef = timed(lambda: plan.spline(mh[None]))
    t_pred, _ = timed(lambda: plan.predict(coef, Qd))
    Mtot = int(np.prod(w.M))
    fin = torch.isfinite(iv["Sigma"])
    out = {"interval_ms": round(t_int, 4), "interval_grid_points_per_s": round(Mtot / (t_int * 1e-3), 1),
           "spline_ms": round(t_spl, 4), "predict_ms": round(t_pred, 4), "predict_points": n_query,
           "predict_points_per_s": round(n_query / (t_pred * 1e-3), 1),
           "band_halfwidth_median": float(torch.median(iv["upper"][fin] - iv["lower"][fin]).item() / 2),
           "plan": "FP32 spreading, %s transforms, h_min = h / sqrt 2" % transform}
    del plan
    return out


def _kernel_generality(reps):
    """Fits on the 2-D workload's samples (N = 1e6 mixture, M = 256^2, one
    response, FP32 spreading, FP64 transforms) with the Gaussian at
    h = (0.03, 0.05), with a full bandwidth matrix of those marginal widths
    and correlation 0.5, and with the Epanechnikov kernel of half-widths
    (0.07, 0.11) (about the Gaussian's variance; the binned approximation
    keeps every mode of the period), each replayed as a HIP graph with the
    points already sorted."""
    import numpy as np
    import torch
    import workloads
    from paper_2204_07716_amd import Plan
    w = workloads.make("ll2d")
    dev = torch.device("cuda:0")
    X = torch.as_tensor(w.X.astype(np.float32), device=dev)
    Y = torch.as_tensor(w.Y.astype(np.float32), device=dev)
    h = np.asarray(w.h[0])
    H = np.array([[h[0] ** 2, 0.5 * h[0] * h[1]], [0.5 * h[0] * h[1], h[1] ** 2]])
    reach = 1.0 / np.sqrt(np.diag(np.linalg.inv(H)))
    he = np.array([0.07, 0.11])

    def replay_ms(fn):
        s = torch.cuda.Stream()
        s.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(s):
            fn()
        torch.cuda.current_stream().wait_stream(s)
        torch.cuda.synchronize()
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g):
            fn()
        g.replay()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            g.replay()
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) * 1e3 / reps

    out = {"N": w.N, "M": list(w.M)}
    pg = Plan(2, 1, w.M, w.lo, w.hi, tuple(reach), tuple(h), w.eps, precision="fp32", n_max=w.N,
              transform_precision="fp64")
    pg.set_points(X)
    out["gauss_fit_ms"] = round(replay_ms(lambda: pg.fit(h, Y)), 4)
    out["full_h_fit_ms"] = round(replay_ms(lambda: pg.fit_full(H, Y)), 4)
    out["band"] = list(pg.band)
    del pg
    pe = Plan(2, 1, w.M, w.lo, w.hi, tuple(he), tuple(he), w.eps, precision="fp32", n_max=w.N,
              transform_precision="fp64", reg_kernel="epanechnikov")
    pe.set_points(X)
    out["epanechnikov_fit_ms"] = round(replay_ms(lambda: pe.fit(he, Y)), 4)
    out["epanechnikov_band"] = list(pe.band)
    del pe
    return out


def _grad_workload(reps):
    """The differentiated workload (complex y = 8 Lorentzian peaks + noise,
    N = 4e6, M = 512^2, local quadratic, h = 0.02, 10 Philox probes, FP32
    spreading, FP64 transforms and 6x6 solves), both replayed as HIP graphs
    with the points already sorted: the forward GCV (fit, DF and GCV in one
    fkr_cv call) and the forward plus the hand-written backward
    (fkr_gcv_grad: GCV, its gradient in log h and in y)."""
    import numpy as np
    import torch
    import workloads
    from paper_2204_07716_amd import Plan
    w = workloads.make("cplx2d")
    h = np.asarray(w.h[0])
    Np, seed = w.n_probes, w.probe_seed
    dev = torch.device("cuda:0")
    plan = Plan(2, 2, w.M, w.lo, w.hi, tuple(h), tuple(h), w.eps, precision="fp32", n_max=w.N, max_weights=28,
                max_h=1, transform_precision="fp64")
    plan.set_points(torch.as_tensor(w.X.astype(np.float32), device=dev))
    Y = torch.as_tensor(w.Y[:, 0].astype(np.complex64), device=dev)

    def replay_ms(fn):
        s = torch.cuda.Stream()
        s.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(s):
            fn()
        torch.cuda.current_stream().wait_stream(s)
        torch.cuda.synchronize()
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g):
            res = fn()
        g.replay()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            g.replay()
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) * 1e3 / reps, res

    t_fwd, f = replay_ms(lambda: plan.cv(h, Y, Np, seed=seed, want_mhat=False))
    t_both, r = replay_ms(lambda: plan.gcv_grad(h, Y, Np, seed))
    del plan
    # the plain FP64 form: one fit of the same response (spreading,
    # transforms and solves in FP64 at eps = 1e-9), points sorted outside
    p64 = Plan(2, 2, w.M, w.lo, w.hi, tuple(h), tuple(h), 1e-9, precision="fp64", n_max=w.N, max_weights=3,
               max_h=1)
    p64.set_points(torch.as_tensor(w.X, device=dev))
    Y64 = torch.as_tensor(w.Y[:, 0], device=dev)
    t_64, _ = replay_ms(lambda: p64.fit(h, Y64))
    del p64
    out = {"N": w.N, "M": list(w.M), "order": 2, "probes": Np, "ms_forward": round(t_fwd, 3),
           "ms_forward_backward": round(t_both, 3), "backward_over_forward": round(t_both / t_fwd - 1, 3),
           "samples_per_s": round(w.N / (t_both * 1e-3), 1), "gcv": float(r["gcv"].item()),
           "fp64_single_fit_ms": round(t_64, 3),
           "forward_over_fp64_single": round(t_64 / t_fwd, 3),
           "forward_backward_over_fp64_single": round(t_64 / t_both, 3),
           "gcv_forward_only": float(f["gcv"][0, 0].item()),
           "dlogh": [float(v) for v in r["dlogh"].cpu().numpy()],
           "note": "points sorted outside the timed graphs; forward = fkr_cv (fit, DF from 10 probes, GCV), "
                   "forward + backward = fkr_gcv_grad; fp64_single = one FP64 fit of y alone"}
    return out


def _batch_workload(reps):
    """The batch workload on one GPU (Sec. 2.1, Fig. 3, Sec. 4.3), both parts
    replayed as HIP graphs:
    * its 256 independent regressions (N log-uniform in [1e3, 1e6], x ~
      U[0,1]^2, M = 256^2, h = 0.05, 4 Philox probes each, fit + DF + GCV) in
      one fkr_batch_cv call, with the lane count and job size the autotuner
      picks, against the same batch on one lane (the regressions one after
      another on one stream);
    * the shared-grid DF sweep: N = 2e6 mixture samples, 64 probes x 32
      log-spaced bandwidths in [0.01, 0.2], one fkr_cv call (one spread and
      forward FFT of all 66 weight vectors, then channels, solves and
      reductions per bandwidth)."""
    import numpy as np
    import torch
    import workloads
    from paper_2204_07716_amd import Batch, Plan
    w = workloads.make("batch2d")
    sizes = w.extra["regression_sizes"]
    Xs, Ys = zip(*(workloads.independent_regression(w, k) for k in range(len(sizes))))
    off = np.concatenate([[0], np.cumsum(sizes)])
    dev = torch.device("cuda:0")
    X = torch.as_tensor(np.concatenate(Xs).astype(np.float32), device=dev)
    Y = torch.as_tensor(np.concatenate(Ys).astype(np.float32), device=dev)
    h = (w.extra["regression_h"],) * 2
    Np = 4
    b = Batch(2, 1, w.M, w.lo, w.hi, h, h, w.eps, precision="fp32", n_max=int(sizes.max()),
              max_weights=2 + Np, n_lanes=8, transform_precision="fp64")

    def replay_ms(fn):
        s = torch.cuda.Stream()
        s.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(s):
            fn()
        torch.cuda.current_stream().wait_stream(s)
        torch.cuda.synchronize()
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g):
            res = fn()
        g.replay()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            g.replay()
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) * 1e3 / reps, res

    run = lambda: b.cv(off, X, h, Y, Np, seed=4100, want_mhat=False)   # noqa: E731
    b.config(1)
    t_loop, _ = replay_ms(run)
    tuned = b.tune(off, X, h, Y, Np, seed=4100, reps=2)
    t_batch, res = replay_ms(run)
    n_tot = int(off[-1])
    gcv = res["gcv"][:, 0, 0]
    out = {"regressions": len(sizes), "samples": n_tot, "ms_batched": round(t_batch, 3),
           "ms_one_lane": round(t_loop, 3), "samples_per_s": round(n_tot / (t_batch * 1e-3), 1),
           "speedup_over_one_lane": round(t_loop / t_batch, 3), "tuned": tuned,
           "finite_gcv": int(torch.isfinite(gcv).sum().item())}
    del b
    # the DF sweep
    hs = w.h
    Npd = w.n_probes
    plan = Plan(2, 1, w.M, w.lo, w.hi, hs[0], hs[-1], w.eps, precision="fp32", n_max=w.N,
                max_weights=2 + Npd, max_h=len(hs), transform_precision="fp64")
    Xd = torch.as_tensor(w.X.astype(np.float32), device=dev)
    Yd = torch.as_tensor(w.Y.astype(np.float32), device=dev)
    plan.set_points(Xd)
    t_df, r = replay_ms(lambda: plan.cv(hs, Yd, Npd, seed=w.probe_seed, want_mhat=False))
    g2 = r["gcv"][:, 0]
    out["df_sweep"] = {"N": w.N, "probes": Npd, "bandwidths": len(hs), "ms": round(t_df, 3),
                       "probe_fits_per_s": round(w.N * Npd * len(hs) / (t_df * 1e-3), 1),
                       "finite_gcv": int(torch.isfinite(g2).sum().item()),
                       "note": "set_points outside the timed graph; one fkr_cv call per sweep"}
    del plan
    return out


def _fp64_single(w, Xd, Yd, steps, warmup, batched_value, use_graph):
    """The plain FP64 form of one regression on the same samples and grid:
    FP64 spreading, transforms and solves at the same requested accuracy; one
    step is set_points and one fit (density and y), replayed as a HIP graph
    when the batched step is.  samples/s counts the response only (1 fit per
    step), as `value` counts the 12 responses, probes and variance fits."""
    import torch
    from paper_2204_07716_amd import Plan
    h = w.h[0]
    p64 = Plan(w.d, 1, w.M, w.lo, w.hi, h, h, w.eps, precision="fp64", n_max=w.N, max_weights=2,
               max_h=1, transform_precision="fp64")
    X64, Y64 = Xd.double(), Yd.double()

    def st():
        p64.set_points(X64)
        return p64.fit(h, Y64)

    for _ in range(max(1, warmup)):
        st()
    torch.cuda.synchronize()
    if use_graph:
        s_cap = torch.cuda.Stream()
        s_cap.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(s_cap):
            st()
        torch.cuda.current_stream().wait_stream(s_cap)
        torch.cuda.synchronize()
        gr = torch.cuda.CUDAGraph()
        with torch.cuda.graph(gr):
            mh = st()
        gr.replay()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            gr.replay()
        torch.cuda.synchronize()
    else:
        t0 = time.perf_counter()
        for _ in range(steps):
            mh = st()
        torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / steps
    v = w.N * 1 / (ms * 1e-3)
    res = {"ms_per_step": round(ms, 4), "value": round(v, 1), "unit": "samples/s",
           "fits_per_step": 1, "batched_fp32_over_fp64": round(batched_value / v, 2),
           "hip_graph": bool(use_graph),
           "note": "FP64 plan (spreading, transforms, solves), one response, set_points + fit per step",
           "_mhat": mh[0, 0].cpu().numpy()}
    del p64
    return res


def _cpu_baseline(w, out, vhat, kappa, n_fits, gpu_value, flat, fp64):
    """The oracle on G seeded grid points per pass: the fits of y and the 10
    probes, then the log-variance fit, timed on the host cores and
    extrapolated to the full grid; its values at those points check the GPU
    grids (mask: s_0 >= 1e-3 max s_0 over the sample, resolved points)."""
    import numpy as np

    from oracle import oracle as orc

    N, M, h, d = w.N, w.M, w.h[0], w.d
    Mtot = int(np.prod(M))
    G = len(flat)
    gp = orc.grid_points(M, w.lo, w.hi)[flat]
    X = w.X.astype(np.float32).astype(np.float64)
    y = w.Y[:, 0].astype(np.float32).astype(np.float64)
    probes = orc.probes(w.probe_seed, N, w.n_probes).astype(np.float32).astype(np.float64)
    mh_gpu = out["mhat"][0, 0].cpu().numpy()
    # the variance pass's input: residuals against the GPU mean grid
    r = (y - orc.interp(mh_gpu, M, w.lo, w.hi, X)) ** 2
    keep = np.isfinite(r)
    z = np.log(r + 1.0 / N)
    Wfit = np.concatenate([y[:, None], probes], axis=1)
    orc.fit(X[:1000], Wfit[:1000], h, 1, gp[:2])          # load / warm the library
    t0 = time.perf_counter()
    ref, S, T, r0, ill = orc.fit(X, Wfit, h, 1, gp, return_all=True)
    v_ref = orc.fit(X[keep], z[keep], h, 1, gp)[:, 0]
    t_sample = time.perf_counter() - t0
    t_full = t_sample * Mtot / G
    cpu_value = N * n_fits / t_full
    mask = (S[:, 0] >= 1e-3 * S[:, 0].max()) & orc.resolved(S, h, 1, d)

    def rel(a, b):
        a, b = a[mask], b[mask]
        return float(np.abs(a - b).max() / np.abs(b).max())

    model, nproc = _cpu_info()
    acc = {"mhat_rel_err": rel(mh_gpu[flat], ref[:, 0]),
           "vhat_rel_err": rel(vhat.cpu().numpy()[flat], v_ref),
           "mask": "s0 >= 1e-3 max s0, resolved", "points": int(mask.sum()), "bar": 1e-5}
    if fp64 is not None:
        acc["fp64_single_mhat_rel_err"] = rel(fp64.pop("_mhat")[flat], ref[:, 0])
    return {
        "cpu_baseline": {
            "value": round(cpu_value, 2), "unit": "samples/s", "cores": orc.threads(),
            "kind": "oracle",
            "sample": f"FP64 direct sums of the {n_fits} fits at {G} of {Mtot} grid points per pass "
                      f"(N={N}), {t_sample:.2f} s, extrapolated x{Mtot / G:.0f} to the grid",
            "nproc": nproc, "omp_threads": orc.threads(), "cpu_model": model,
            "gpu_over_cpu": round(gpu_value / cpu_value, 1)},
        "accuracy": acc,
    }


if __name__ == "__main__":
    sys.exit(main())
