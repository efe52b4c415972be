"""Batches of independent regressions (fkr_batch_*): uneven-N regressions on
one plan geometry over several lanes (plans with their own streams), against
single-plan calls (themselves pinned to the oracle) and, for whole
regressions, against the oracle; graph capture of a whole batch; the
autotuner; the 256 regressions of the batch workload at full size."""
import numpy as np
import pytest

import workloads
from gpu_common import compare_fit, make_plan, match_dof, support_variants, to_dev

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _batch(w, sizes, h, Np, n_lanes=4, max_h=1):
    from paper_2204_07716_amd import Batch
    return Batch(2, 1, w.M, w.lo, w.hi, h, h if max_h == 1 else (0.2, 0.2), w.eps, precision="fp32",
                 n_max=int(max(sizes)), max_weights=2 + Np, max_h=max_h, n_lanes=n_lanes,
                 transform_precision="fp64")


def _concat(w, ks):
    Xs, Ys = zip(*(workloads.independent_regression(w, k) for k in ks))
    off = np.concatenate([[0], np.cumsum([len(x) for x in Xs])])
    return np.concatenate(Xs), np.concatenate(Ys), off


def _same(a, b, rel):
    a, b = np.asarray(a), np.asarray(b)
    assert np.array_equal(np.isnan(a), np.isnan(b))
    f = ~np.isnan(b)
    if f.any():
        assert np.abs(a[f] - b[f]).max() <= rel * max(np.abs(b[f]).max(), 1e-300)


def _small_set(w, n=10):
    sizes = w.extra["regression_sizes"]
    ks = [int(k) for k in np.argsort(sizes)[:n]]   # the smallest regressions of the workload
    return ks


def test_batch_matches_single_plans_and_oracle(orc):
    """Ten of the smallest regressions (N from about 1e3 upward) plus an empty
    one, two bandwidths, 4 probes: every output equals the single-plan call
    with seed + r (up to the order of FP32 sums), and the smallest
    regression's fit and DF match the oracle on the whole grid."""
    w = workloads.make("batch2d", M=(64, 64))
    ks = _small_set(w)
    X, Y, off = _concat(w, ks)
    off = np.concatenate([off[:4], [off[3]], off[4:]])      # an empty regression at index 3
    R = len(off) - 1
    hs = np.array([[0.06, 0.06], [0.1, 0.1]])
    Np, seed = 4, 9000
    b = _batch(w, np.diff(off), (0.06, 0.06), Np, max_h=2)
    out = b.cv(off, to_dev(X, torch.float32), hs, to_dev(Y, torch.float32), Np, seed=seed)
    res = {k: v.cpu().numpy() for k, v in out.items()}
    assert np.isnan(res["gcv"][3]).all() and (res["nused"][3] == 0).all() and np.isnan(res["mhat"][3]).all()
    plan = make_plan(2, 1, w.M, (0.06, 0.06), (0.2, 0.2), w.eps, "fp32", n_max=int(np.diff(off).max()),
                     max_weights=2 + Np, max_h=2, tprec="fp64")
    for r in range(R):
        if off[r + 1] == off[r]:
            continue
        plan.set_points(to_dev(X[off[r]:off[r + 1]], torch.float32))
        one = plan.cv(hs, to_dev(Y[off[r]:off[r + 1]], torch.float32), Np, seed=seed + r)
        for k in ("mhat", "rho", "rss", "gcv", "nused"):
            _same(res[k][r], one[k].cpu().numpy(), 1e-6)
    # the smallest regression against the oracle, every grid point
    r = int(np.argmin(np.where(np.diff(off) > 0, np.diff(off), 1 << 40)))
    Xr = X[off[r]:off[r + 1]].astype(np.float32).astype(np.float64)
    yr = Y[off[r]:off[r + 1], 0].astype(np.float32).astype(np.float64)
    probes = orc.probes(seed + r, len(Xr), Np)
    gp = orc.grid_points(w.M, w.lo, w.hi)
    for hi_, h in enumerate(hs):
        ref, S, T, r0, ill = orc.fit(Xr, np.concatenate([yr[:, None], probes], axis=1), h, 1, gp, return_all=True)
        compare_fit(res["mhat"][r, hi_, 0], ref[:, 0], S, h, 1, 2, 1e-5)
        what = orc.interp(ref[:, 1:], w.M, w.lo, w.hi, Xr)
        match_dof(res["rho"][r, hi_], res["nused"][r, hi_], probes, what,
                  support_variants(S, ill, h, 1, 2, w.M, w.lo, w.hi, Xr), 1e-6)


def test_batch_graph_capture_and_tune():
    """A whole batch captured into one HIP graph (fork and join through
    events) replays to the eager result, with eager batch calls in between;
    the autotuner returns a valid configuration and the outputs after tuning
    agree with those before."""
    w = workloads.make("batch2d", M=(64, 64))
    ks = _small_set(w, 16)
    X, Y, off = _concat(w, ks)
    Np, seed, h = 2, 77, (0.08, 0.08)
    b = _batch(w, np.diff(off), h, Np)
    Xd, Yd = to_dev(X, torch.float32), to_dev(Y, torch.float32)
    ref = b.cv(off, Xd, h, Yd, Np, seed=seed)
    torch.cuda.synchronize()
    ref = {k: v.clone() for k, v in ref.items()}
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        b.cv(off, Xd, h, Yd, Np, seed=seed)
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        got = b.cv(off, Xd, h, Yd, Np, seed=seed)
    for _ in range(3):
        g.replay()
        torch.cuda.synchronize()
        for k in ref:
            _same(got[k].cpu().numpy(), ref[k].cpu().numpy(), 1e-6)
        b.cv(off, Xd, h, Yd, Np, seed=seed + 1)           # eager work between replays
        torch.cuda.synchronize()
    t = b.tune(off, Xd, h, Yd, Np, seed=seed, reps=1)
    assert t["lanes"] in (1, 2, 4) and t["chunk"] in (1024, 2048, 4096) and t["ms"] > 0
    after = b.cv(off, Xd, h, Yd, Np, seed=seed)
    for k in ref:
        _same(after[k].cpu().numpy(), ref[k].cpu().numpy(), 1e-6)


def test_batch_rejects_bad_offsets():
    from paper_2204_07716_amd._lib import FkrError
    w = workloads.make("batch2d", M=(64, 64))
    b = _batch(w, [100], (0.08, 0.08), 2)
    X = to_dev(np.random.default_rng(0).random((100, 2)), torch.float32)
    Y = to_dev(np.zeros((100, 1)), torch.float32)
    for off in ([0, 60, 40, 100], [1, 100], [0, 101]):      # decreasing, not from 0, above n_max
        with pytest.raises(FkrError):
            b.cv(off, X, (0.08, 0.08), Y, 2)
    with pytest.raises(FkrError):
        b.cv([0, 100], X, (0.05, 0.05), Y, 2)             # bandwidth outside the plan's range


def test_batch_workload_full_size(orc):
    """The batch workload's 256 independent regressions (N log-uniform in
    [1e3, 1e6], about 3.7e7 samples, M = 256^2, h = 0.05, 4 probes) in one
    batch call: every GCV finite; the smallest, median and largest match their
    single-plan calls (pinned to the oracle in test_gpu_fullsize_dof.py)."""
    w = workloads.make("batch2d")
    sizes = w.extra["regression_sizes"]
    X, Y, off = _concat(w, range(len(sizes)))
    Np, seed = 4, 4100
    h = (w.extra["regression_h"],) * 2
    b = _batch(w, sizes, h, Np)
    out = b.cv(off, to_dev(X, torch.float32), h, to_dev(Y, torch.float32), Np, seed=seed, want_mhat=False)
    gcv = out["gcv"].cpu().numpy()[:, 0, 0]
    assert np.isfinite(gcv).all()
    plan = make_plan(2, 1, w.M, h, h, w.eps, "fp32", n_max=int(sizes.max()), max_weights=2 + Np, tprec="fp64")
    for k in (int(np.argmin(sizes)), int(np.argsort(sizes)[128]), int(np.argmax(sizes))):
        plan.set_points(to_dev(X[off[k]:off[k + 1]], torch.float32))
        one = plan.cv(h, to_dev(Y[off[k]:off[k + 1]], torch.float32), Np, seed=seed + k)
        for key in ("rho", "rss", "gcv", "nused"):
            _same(out[key].cpu().numpy()[k], one[key].cpu().numpy(), 1e-6)
