#!/usr/bin/env python3
"""Throughput of the fast kernel-regression hot path on one MI355X.

Workload: the 2-D local-linear mixture regression (N = 1e6 samples from a
4-component Gaussian mixture clipped to the unit square, y = sin(4 x1)
cos(3 x2) + 0.2 e, h = (0.03, 0.05), M = 256^2 grid, order 1, eps = 1e-6,
FP32 spreading, FP64 transforms by default, FP64 3x3 solves), seeded and
synthetic.  One step is one pass of the whole path:

  set_points   bin and sort the samples (once per X)
  cv           spread of density, y and 10 Philox probes -> forward FFTs ->
               moment channels -> FP64 solves -> interpolation -> Girard DF,
               RSS and GCV (Sec. 2.1, eq. 22)
  variance     log-residual second pass (eq. 24-26): residuals, spread,
               FFTs, solves, kappa, sigma^2 on the grid

The headline value is samples/s = N x fits / step time, where a fit is one
weight vector through spread + FFT + solve (1 response + 10 probes + 1
variance pass = 12 per step).  The ``roofline`` object reports the spreading
kernel (the largest single kernel of the step) against FP32 FMA issue with its
algorithmic flops per launch, and against HBM bandwidth with its algorithmic
bytes, timed with HIP events that the library records on the launch stream;
``warm`` times the same step without set_points (X already sorted);
``hbm_model`` sets the step's algorithmic bytes against HBM bandwidth;
``cpu_baseline`` times the FP64 oracle on a bounded sample of grid points and
extrapolates to the full grid; ``accuracy`` compares the GPU grids with the
oracle on that same sample; ``fp64_single`` times the plain FP64 form (FP64
spreading, transforms and solves) of one regression on the same samples, for
comparison with the batched FP32-spreading step.

By default the timed steps replay a HIP graph captured from one step (the
step's ~30 kernel launches are launch-bound on the host otherwise); before
timing, three replays are compared with eager steps.  ``--eager`` times
host-launched steps instead.  Stage times always come from eager steps, where
the library brackets every launch with HIP events on the launch stream.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--transform fp64|fp32] [--eager]
                       [--no-warm] [--no-cpu-baseline] [--no-fp64-single]
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

HBM_PEAK_GBS = 8000.0
# FP32 FMA issue: 256 CUs x 4 SIMDs x 16 lanes x 2 flops x 2.4 GHz (no packed FP32)
FP32_FMA_PEAK_TFLOPS = 78.6
COUNTERS = os.path.join(ROOT, "profiles", "k_spread_ll2d_counters.json")
KERNEL_SOURCE = os.path.join(ROOT, "paper_2204_07716_amd", "csrc", "kernels.hip")


def _args():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
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
    ap.add_argument("--cpu-points", type=int, default=4096,
                    help="grid points in the oracle's timed sample")
    ap.add_argument("--copy-probe", action="store_true",
                    help="after the run, copy a 256 MiB buffer once (counter calibration)")
    return ap.parse_args()


def _kernel_hash() -> str:
    with open(KERNEL_SOURCE, "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()


def _traffic(launches_per_step: int):
    """HBM bytes per spread launch from the committed counter run, or None when
    the kernel source has changed since the counters were taken."""
    try:
        with open(COUNTERS) as f:
            c = json.load(f)
    except (OSError, ValueError):
        return None
    if c.get("kernel_source_sha256") != _kernel_hash():
        return None
    per_step = (c["fetch_kib_per_step"] * 1024 * c["copy_fetch_scale"]
                + c["write_kib_per_step"] * 1024 * c["copy_write_scale"])
    return per_step / launches_per_step


def _hbm_model(g, N, M, Np, stages, steps, ms_per_step):
    """Algorithmic bytes of the step (sort, spread, forward FFT, inverse FFT,
    solve; FP32 spreading, FP64 complex transforms) against HBM bandwidth, for
    spread + FFT and for the whole step."""
    d = 2
    Mr = g.Mr[0] * g.Mr[1]
    L = g.L[0] * g.L[1]
    Mg = M[0] * M[1]
    bx, bw, bc_s, bc_t = 4, 4, 8, 16
    n_s, n_t = 6, 3
    calls = [dict(nw=2 + Np, q=1, np_=Np), dict(nw=2, q=1, np_=0)]   # cv, variance
    b_sort = N * (d * bx + 24)
    b_spread = b_fft = b_inv = b_solve = 0
    for c in calls:
        npair = (c["nw"] + 1) // 2
        n_ch = n_s + n_t * (c["nw"] - 1)
        b_spread += N * (d * bx + c["nw"] * bw) + npair * Mr * bc_s
        b_fft += d * 2 * npair * Mr * bc_t
        b_inv += ((n_ch + 1) // 2) * L * bc_t * (1 + 2 * d)
        b_solve += (n_ch + c["q"] + c["np_"]) * Mg * 8
    t_sf = sum(stages[k][0] for k in ("spread", "fold", "fft_fwd")) * 1e-3 / steps
    b_all = b_sort + b_spread + b_fft + b_inv + b_solve
    return {"spread_fft": {"bytes": b_spread + b_fft, "ms": round(t_sf * 1e3, 4),
                           "frac": round((b_spread + b_fft) / t_sf / 8e12, 4)},
            "whole_step": {"bytes": b_all, "ms": round(ms_per_step, 4),
                           "frac": round(b_all / (ms_per_step * 1e-3) / 8e12, 4)},
            "peak_GBs": 8000.0}


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
    w = workloads.make("ll2d")
    N, M, h = w.N, w.M, w.h[0]
    Np, seed = w.n_probes, w.probe_seed
    Xd = torch.as_tensor(w.X.astype(np.float32), device=dev)
    Yd = torch.as_tensor(w.Y.astype(np.float32), device=dev)
    plan = Plan(2, 1, M, w.lo, w.hi, h, h, w.eps, precision="fp32", n_max=N,
                max_weights=2 + Np, max_h=1, transform_precision=args.transform, sigma=args.sigma)
    g = plan.geometry
    torch.cuda.synchronize()

    def step():
        plan.set_points(Xd)
        out = plan.cv(h, Yd, Np, seed=seed)
        s2, vhat, kappa = plan.variance(h, Yd, out["mhat"][0, 0], mode="log")
        return out, s2, vhat, kappa

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    args.graph = not args.eager
    if args.graph:
        # eager reference, then capture; every replay must reproduce it
        ref = step()
        torch.cuda.synchronize()
        ref_vals = [ref[0]["mhat"].clone(), ref[0]["rho"].clone(), ref[0]["gcv"].clone(), ref[1].clone()]
        s_cap = torch.cuda.Stream()
        s_cap.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(s_cap):
            step()                       # warm the capture stream's allocator pool
        torch.cuda.current_stream().wait_stream(s_cap)
        torch.cuda.synchronize()
        graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(graph):
            res_g = step()
        for rep in range(3):
            graph.replay()
            torch.cuda.synchronize()
            got = [res_g[0]["mhat"], res_g[0]["rho"], res_g[0]["gcv"], res_g[1]]
            for a, b in zip(got, ref_vals):
                # samples of one cell are ranked with LDS atomics, so the FP32
                # summation order (and the last bits) may differ between runs
                fin = torch.isfinite(b)
                scale = b[fin].abs().max() if fin.any() else torch.tensor(0.0, device=b.device)
                same_nan = torch.equal(torch.isnan(a), torch.isnan(b))
                if not same_nan or (a[fin] - b[fin]).abs().max() > 1e-6 * scale:
                    print(json.dumps({"error": "graph replay differs from the eager step", "replay": rep}))
                    return 1
            step()                       # eager work between replays
            torch.cuda.synchronize()
    t0 = time.perf_counter()
    if args.graph:
        for _ in range(args.steps):
            graph.replay()
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        res = res_g
        # stage times come from an eager pass over the same steps
        plan.profile(True)
        plan.profile_read()
        for _ in range(args.steps):
            step()
        torch.cuda.synchronize()
        stages = plan.profile_read()
        plan.profile(False)
    else:
        plan.profile(True)
        plan.profile_read()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            res = step()
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        stages = plan.profile_read()
        plan.profile(False)
    ms_per_step = (t1 - t0) * 1e3 / args.steps
    n_fits = (1 + Np) + 1

    # Warm path: X already sorted, set_points outside the timed region.
    def warm_step():
        out = plan.cv(h, Yd, Np, seed=seed)
        s2, vhat, kappa = plan.variance(h, Yd, out["mhat"][0, 0], mode="log")
        return out, s2, vhat, kappa

    warm_ms = None
    if args.no_warm:
        pass
    elif args.graph:
        plan.set_points(Xd)
        warm_step()
        torch.cuda.synchronize()
        s_cap = torch.cuda.Stream()
        s_cap.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(s_cap):
            warm_step()
        torch.cuda.current_stream().wait_stream(s_cap)
        torch.cuda.synchronize()
        wgraph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(wgraph):
            wres = warm_step()
        wgraph.replay()
        torch.cuda.synchronize()
        for a, b in zip([wres[0]["mhat"], wres[1]], [res[0]["mhat"], res[1]]):
            fin = torch.isfinite(b)
            if not torch.equal(torch.isnan(a), torch.isnan(b)) or \
                    (a[fin] - b[fin]).abs().max() > 1e-6 * b[fin].abs().max():
                print(json.dumps({"error": "warm graph replay differs from the timed steps"}))
                return 1
        tw0 = time.perf_counter()
        for _ in range(args.steps):
            wgraph.replay()
        torch.cuda.synchronize()
        tw1 = time.perf_counter()
    else:
        plan.set_points(Xd)
        warm_step()
        torch.cuda.synchronize()
        tw0 = time.perf_counter()
        for _ in range(args.steps):
            warm_step()
        torch.cuda.synchronize()
        tw1 = time.perf_counter()
    if not args.no_warm:
        warm_ms = (tw1 - tw0) * 1e3 / args.steps
    value = N * n_fits / (ms_per_step * 1e-3)

    # Roofline of the spreading kernel.  Its arithmetic is 2 W^d n_w flops per
    # sample (one FMA per footprint cell and weight column) against N (d b_x +
    # n_w b_w) + n_pair Mr^d b_c algorithmic bytes: about 13 flop/B for the
    # step's two launches, above the 9.8 flop/B ridge of FP32 FMA issue
    # (78.6 TFLOP/s) over HBM (8 TB/s), so the bound is the ALU.
    Mr2 = g.Mr[0] * g.Mr[1]
    bx, bw, bc = 4, 4, 8
    nw_launch = [2 + Np, 2]              # cv (density, y, probes), variance (density, z)
    bytes_step = sum(N * (2 * bx + nw * bw) + ((nw + 1) // 2) * Mr2 * bc for nw in nw_launch)
    flops_step = sum(2.0 * N * g.w ** 2 * nw for nw in nw_launch)
    spread_ms, spread_n = stages["spread"]
    launches_per_step = spread_n / args.steps
    spread_s = spread_ms * 1e-3 / args.steps
    achieved = flops_step / spread_s / 1e12
    hbm_achieved = bytes_step / spread_s / 1e9
    roofline = {"bound": "alu", "kernel": "spread: k_spread_wave (cv, 12 columns; variance, 2 columns)",
                "achieved": round(achieved, 2), "peak": FP32_FMA_PEAK_TFLOPS, "unit": "TFLOP/s",
                "frac": round(achieved / FP32_FMA_PEAK_TFLOPS, 4),
                "traffic": _traffic(launches_per_step),
                "algorithmic_flops_per_launch": flops_step / launches_per_step,
                "algorithmic_bytes_per_launch": bytes_step / launches_per_step,
                "avg_launch_us": round(spread_ms * 1e3 / max(spread_n, 1), 2),
                "launches_per_step": launches_per_step,
                "hbm": {"achieved": round(hbm_achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                        "frac": round(hbm_achieved / HBM_PEAK_GBS, 4)}}

    out, s2, vhat, kappa = res
    line = {
        "metric": "samples/s (spread+FFT+solve) at stated rel err vs FP64 oracle; % of HBM BW",
        "value": round(value, 1), "unit": "samples/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(ms_per_step, 4), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None,
        "dtype": "f32 spread, %s transforms, f64 solves" % ("f64" if args.transform == "fp64" else "f32"),
        "data": "synthetic (seeded 4-component Gaussian mixture, N=1e6)",
        "config": {"workload": "2-D local linear, N=1e6 mixture, h=(0.03,0.05), M=256x256, "
                               "eps=1e-6, 10 Philox probes, log-variance pass",
                   "N": N, "M": list(M), "order": 1, "fits_per_step": n_fits,
                   "grid_points_per_s": round(M[0] * M[1] * n_fits / (ms_per_step * 1e-3), 1),
                   "L": [g.L[0], g.L[1]], "Mr": [g.Mr[0], g.Mr[1]], "K": [g.K[0], g.K[1]],
                   "spread_width": g.w, "sigma": args.sigma or "default",
                   "hip_graph": bool(args.graph)},
        "roofline": roofline,
        "warm": None if warm_ms is None else
                {"ms_per_step": round(warm_ms, 4), "value": round(N * n_fits / (warm_ms * 1e-3), 1),
                 "unit": "samples/s", "note": "X already sorted: set_points outside the timed region"},
        "hbm_model": _hbm_model(g, N, M, Np, stages, args.steps, ms_per_step),
        "stages_ms_per_step": {k: round(v[0] / args.steps, 4) for k, v in stages.items()},
        "gcv": float(out["gcv"][0, 0]), "df": float(N * (1 - out["rho"][0].mean())),
    }

    if args.copy_probe:
        a = torch.empty(64 << 20, dtype=torch.float32, device=dev).fill_(1.0)
        b = torch.empty_like(a)
        torch.cuda.synchronize()
        b.copy_(a)
        torch.cuda.synchronize()
        line["copy_probe_bytes"] = a.numel() * 4

    if not args.no_fp64_single:
        line["fp64_single"] = _fp64_single(w, Xd, Yd, args.steps, args.warmup, value)
    if not args.no_cpu_baseline:
        line.update(_cpu_baseline(args, w, plan, out, vhat, kappa, n_fits, value))
    print(json.dumps(line), flush=True)
    return 0


def _fp64_single(w, Xd, Yd, steps, warmup, batched_value):
    """The plain FP64 form of one regression on the same samples and grid:
    FP64 spreading, transforms and solves, at the same requested accuracy;
    one step is set_points and one fit (density and y, 2 weight vectors),
    launched eagerly.  samples/s counts N per weight vector, as `value` does."""
    import torch
    from paper_2204_07716_amd import Plan
    h = w.h[0]
    p64 = Plan(2, 1, w.M, w.lo, w.hi, h, h, w.eps, precision="fp64", n_max=w.N, max_weights=2,
               max_h=1, transform_precision="fp64")
    X64, Y64 = Xd.double(), Yd.double()

    def st():
        p64.set_points(X64)
        return p64.fit(h, Y64)

    for _ in range(max(1, warmup)):
        st()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        st()
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / steps
    v = w.N * 2 / (ms * 1e-3)
    del p64
    return {"ms_per_step": round(ms, 4), "value": round(v, 1), "unit": "samples/s",
            "fits_per_step": 2, "batched_fp32_over_fp64": round(batched_value / v, 2),
            "note": "FP64 plan, one response, eager launches"}


def _cpu_baseline(args, w, plan, out, vhat, kappa, n_fits, gpu_value):
    """The oracle on G seeded grid points (plus the corners): the fits of y and
    the 10 probes and the log-variance fit, timed on the host cores and
    extrapolated to the full grid; its values at those points check the GPU
    grids (density mask s_0 >= 1e-3 max s_0 over the sample)."""
    import numpy as np

    from oracle import oracle as orc

    N, M, h = w.N, w.M, w.h[0]
    G = max(16, int(args.cpu_points))
    rng = np.random.default_rng(2024)
    flat = rng.choice(M[0] * M[1], size=G, replace=False)
    flat[:4] = [0, M[0] - 1, M[0] * (M[1] - 1), M[0] * M[1] - 1]
    gp = orc.grid_points(M, w.lo, w.hi)[flat]
    X = w.X.astype(np.float32).astype(np.float64)
    y = w.Y[:, 0].astype(np.float32).astype(np.float64)
    probes = orc.probes(w.probe_seed, N, w.n_probes).astype(np.float32).astype(np.float64)
    mh_gpu = out["mhat"][0, 0].cpu().numpy()
    # the variance pass's input: residuals against the GPU mean grid
    r = (y - orc.interp(mh_gpu, M, w.lo, w.hi, X)) ** 2
    z = np.log(r + 1.0 / N)
    Wfit = np.concatenate([y[:, None], probes], axis=1)
    orc.fit(X[:1000], Wfit[:1000], h, 1, gp[:2])          # load / warm the library
    t0 = time.perf_counter()
    ref, S, T, r0, ill = orc.fit(X, Wfit, h, 1, gp, return_all=True)
    v_ref = orc.fit(X, z, h, 1, gp)[:, 0]
    t_sample = time.perf_counter() - t0
    t_full = t_sample * (M[0] * M[1]) / G
    cpu_value = N * n_fits / t_full
    mask = S[:, 0] >= 1e-3 * S[:, 0].max()

    def rel(a, b):
        a, b = a[mask], b[mask]
        return float(np.abs(a - b).max() / np.abs(b).max())

    return {
        "cpu_baseline": {
            "value": round(cpu_value, 2), "unit": "samples/s", "cores": orc.threads(),
            "kind": "oracle",
            "sample": f"FP64 direct sums of the 12 fits at {G} of {M[0] * M[1]} grid points "
                      f"(N={N}), {t_sample:.2f} s, extrapolated x{M[0] * M[1] / G:.0f} to the grid",
            "gpu_over_cpu": round(gpu_value / cpu_value, 1)},
        "accuracy": {"mhat_rel_err": rel(mh_gpu[flat], ref[:, 0]),
                     "vhat_rel_err": rel(vhat.cpu().numpy()[flat], v_ref),
                     "mask": "s0 >= 1e-3 max s0", "points": int(mask.sum()),
                     "bar": 1e-5},
    }


if __name__ == "__main__":
    sys.exit(main())
