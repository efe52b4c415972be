"""DF, N_I and GCV at the workloads' full sizes (Sec. 2.1, eq. 22): the 1-D
Nadaraya-Watson workload against the direct oracle on every grid point; the
3-D and the complex 2-D workloads by stage isolation (the GPU's grid
moments and probe fits, checked at seeded grid points against the oracle,
feed the oracle's support rule, Girard ratios and GCV); and a sample of the
batch workload's independent regressions of uneven size."""
import numpy as np
import pytest

import workloads
from gpu_common import compare_fit, make_plan, match_dof, sample_flat, stage_isolated_dof, support_variants, to_dev

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def test_nw1d_full_size_dof_gcv(orc):
    """N = 1e5, M = 1024, h = 0.02, order 0, FP64, eps = 1e-9, 10 Philox
    probes: ratios, N_I and GCV against the direct oracle on the full grid."""
    w = workloads.make("nw1d")
    h, Np, seed = w.h[0], w.n_probes, w.probe_seed
    plan = make_plan(1, 0, w.M, h, h, w.eps, "fp64", n_max=w.N, max_weights=2 + Np)
    plan.set_points(to_dev(w.X))
    out = plan.cv(h, to_dev(w.Y), Np, seed=seed)
    rho, nused = out["rho"].cpu().numpy()[0], out["nused"].cpu().numpy()[0]
    gcv, mh = out["gcv"].cpu().numpy()[0, 0], out["mhat"].cpu().numpy()[0, 0]
    probes = orc.probes(seed, w.N, Np)
    gp = orc.grid_points(w.M, w.lo, w.hi)
    W = np.concatenate([w.Y, probes], axis=1)
    ref, S, T, r0, ill = orc.fit(w.X, W, h, 0, gp, return_all=True)
    compare_fit(mh, ref[:, 0], S, h, 0, 1, 10 * w.eps)
    what = orc.interp(ref[:, 1:], w.M, w.lo, w.hi, w.X)
    inc = match_dof(rho, nused, probes, what, support_variants(S, ill, h, 0, 1, w.M, w.lo, w.hi, w.X), 1e-9)
    assert inc.all()
    mean = float(np.mean(orc.girard_ratios(probes, what)))
    g_ref = orc.gcv(w.Y[:, 0], orc.interp(ref[:, 0], w.M, w.lo, w.hi, w.X), mean, include=inc)[0]
    assert abs(gcv / g_ref - 1) < 1e-9


def test_ll3d_full_size_dof_gcv(orc):
    """N = 1e7, M = 128^3, h = 0.05, order 1, 10 Philox probes in one cv
    call; two probes and the GCV by stage isolation."""
    w = workloads.make("ll3d")
    h, Np, seed = w.h[0], w.n_probes, w.probe_seed
    plan = make_plan(3, 1, w.M, h, h, w.eps, "fp32", n_max=w.N, max_weights=2 + Np, tprec="fp64")
    plan.set_points(to_dev(w.X, torch.float32))
    out = plan.cv(h, to_dev(w.Y, torch.float32), Np, seed=seed)
    rho, nused = out["rho"].cpu().numpy()[0], out["nused"].cpu().numpy()[0]
    gcv, mh = out["gcv"].cpu().numpy()[0, 0], out["mhat"].cpu().numpy()[0, 0]
    assert np.isfinite(gcv) and nused == w.N
    rng = np.random.default_rng(35)
    flat = sample_flat(rng, w.M, 20)
    stage_isolated_dof(orc, plan, w, h, orc.probes(seed, w.N, 2), rho, nused, gcv, mh, flat)


def test_cplx2d_full_size_dof_gcv(orc):
    """Complex y (8 Lorentzian peaks, SNR 10), N = 4e6, M = 512^2, local
    quadratic, h = 0.02, 10 Philox probes; two probes and the GCV (|.|^2)
    by stage isolation."""
    w = workloads.make("cplx2d")
    h, Np, seed = w.h[0], w.n_probes, w.probe_seed
    plan = make_plan(2, 2, w.M, h, h, w.eps, "fp32", n_max=w.N, max_weights=3 + Np, tprec="fp64")
    plan.set_points(to_dev(w.X, torch.float32))
    yc = torch.as_tensor(w.Y.astype(np.complex64), device="cuda")
    out = plan.cv(h, yc, Np, seed=seed)
    rho, nused = out["rho"].cpu().numpy()[0], out["nused"].cpu().numpy()[0]
    gcv, mh = out["gcv"].cpu().numpy()[0, 0], out["mhat"].cpu().numpy()[0, 0]
    assert np.isfinite(gcv) and nused > 0.99 * w.N
    rng = np.random.default_rng(57)
    flat = sample_flat(rng, w.M, 20)
    stage_isolated_dof(orc, plan, w, h, orc.probes(seed, w.N, 2), rho, nused, gcv, mh, flat, Y=w.Y[:, 0])


@pytest.mark.parametrize("which", ["smallest", "median", "largest"])
def test_batch_independent_regressions_sample(orc, which):
    """Three of the batch workload's 256 independent regressions (the
    smallest, median and largest N, log-uniform in [1e3, 1e6]): h = 0.05,
    M = 256^2, order 1, 4 Philox probes.  Fits at seeded grid points and the
    DF over the supported samples against the oracle (the full grid when N
    is small, by stage isolation otherwise)."""
    w = workloads.make("batch2d")
    sizes = w.extra["regression_sizes"]
    k = {"smallest": int(np.argmin(sizes)), "largest": int(np.argmax(sizes)),
         "median": int(np.argsort(sizes)[len(sizes) // 2])}[which]
    X, Y = workloads.independent_regression(w, k)
    N = X.shape[0]
    h = (w.extra["regression_h"],) * 2
    Np, seed = 4, 4100 + k
    plan = make_plan(2, 1, w.M, h, h, w.eps, "fp32", n_max=N, max_weights=2 + Np, tprec="fp64")
    plan.set_points(to_dev(X, torch.float32))
    out = plan.cv(h, to_dev(Y, torch.float32), Np, seed=seed)
    rho, nused = out["rho"].cpu().numpy()[0], out["nused"].cpu().numpy()[0]
    gcv, mh = out["gcv"].cpu().numpy()[0, 0], out["mhat"].cpu().numpy()[0, 0]
    assert np.isfinite(gcv)
    X32 = X.astype(np.float32).astype(np.float64)
    y32 = Y[:, 0].astype(np.float32).astype(np.float64)
    probes = orc.probes(seed, N, Np)
    if N <= 20_000:
        gp = orc.grid_points(w.M, w.lo, w.hi)
        W = np.concatenate([y32[:, None], probes], axis=1)
        ref, S, T, r0, ill = orc.fit(X32, W, h, 1, gp, return_all=True)
        compare_fit(mh, ref[:, 0], S, h, 1, 2, 1e-5)
        what = orc.interp(ref[:, 1:], w.M, w.lo, w.hi, X32)
        inc = match_dof(rho, nused, probes, what, support_variants(S, ill, h, 1, 2, w.M, w.lo, w.hi, X32),
                        1e-6)
        mean = float(np.mean(orc.girard_ratios(probes[inc], what[inc])))
        g_ref = orc.gcv(y32, orc.interp(ref[:, 0], w.M, w.lo, w.hi, X32), mean, include=inc)[0]
        assert abs(gcv / g_ref - 1) < 1e-5
    else:
        class Wl:   # the regression in the shape the stage-isolation helper reads
            pass
        wl = Wl()
        wl.d, wl.order, wl.M, wl.lo, wl.hi, wl.X, wl.Y = 2, 1, w.M, w.lo, w.hi, X, Y
        rng = np.random.default_rng(400 + k)
        flat = sample_flat(rng, w.M, 24)
        stage_isolated_dof(orc, plan, wl, h, probes, rho, nused, gcv, mh, flat)
