"""GPU parity of the Monte-Carlo DF (Sec. 2.1), GCV (eq. 22) and the
conditional-variance pass (Sec. 3) against the FP64 oracle.

The DF path uses identical probes on both sides: the GPU generates them with
Philox4x32-10 + Box-Muller from the sample index and the oracle's generator
(pinned to the generator's published known-answer vectors) produces the same
uniforms; a second case
passes the oracle's probes in as an array.
"""
import numpy as np
import pytest

from gpu_common import density_mask, make_plan, rel_err, to_dev

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _data(seed, N, d):
    rng = np.random.default_rng(seed)
    X = rng.random((N, d))
    y = np.sin(3 * X).sum(axis=1) + 0.3 * rng.standard_normal(N)
    return X, y


@pytest.mark.parametrize("d,order,prec,tprec", [(1, 1, "fp64", "same"), (2, 1, "fp32", "fp64"),
                                                 (2, 0, "fp32", "fp32"), (3, 1, "fp32", "fp64")])
def test_dof_matches_oracle_with_identical_probes(orc, d, order, prec, tprec):
    N, Np, seed = 2500, 6, 11
    X, y = _data(400 + d, N, d)
    M, h = {1: ((80,), (0.05,)), 2: ((36, 30), (0.1, 0.12)), 3: ((12, 11, 10), (0.17, 0.16, 0.18))}[d]
    plan = make_plan(d, order, M, h, h, 1e-9 if prec == "fp64" else 1e-6, prec, n_max=N,
                     max_weights=2 + Np, tprec=tprec)
    dt = torch.float64 if prec == "fp64" else torch.float32
    plan.set_points(to_dev(X, dt))
    rho, nused = plan.dof(h, Np, seed=seed, want_nused=True)
    rho, nused = rho.cpu().numpy()[0], nused.cpu().numpy()[0]
    probes = orc.probes(seed, N, Np)
    ref, mean, df, inc = orc.dof(X, h, order, M, (0,) * d, (1,) * d, probes)
    # uniform samples on a grid coarser than the kernel: every sample is supported
    assert inc.all() and nused == N
    bar = 1e-9 if prec == "fp64" else (1e-6 if tprec == "fp64" else 2e-5)
    assert np.abs(rho - ref).max() < bar, (rho, ref)
    # the same probes passed in as an array
    rho2 = plan.dof(h, Np, probes=to_dev(probes, dt)).cpu().numpy()[0]
    assert np.abs(rho2 - ref).max() < bar


def test_cv_gcv_matches_oracle(orc):
    """Batched cross-validation (fit + DF + GCV sharing the spreads) over a
    bandwidth list, with rGCV selection, against the oracle."""
    N, Np, seed = 3000, 8, 5
    X, y = _data(410, N, 2)
    M = (40, 36)
    hs = np.stack([orc.get_hlist(4, [0.06, 0.2], "log")[:, 0]] * 2, axis=1)
    plan = make_plan(2, 1, M, hs[0], hs[-1], 1e-6, "fp32", n_max=N, max_weights=2 + Np,
                     max_h=len(hs), tprec="fp64")
    plan.set_points(to_dev(X, torch.float32))
    out = plan.cv(hs, to_dev(y[:, None], torch.float32), Np, seed=seed)
    gcv = out["gcv"].cpu().numpy()[:, 0]
    rss = out["rss"].cpu().numpy()[:, 0]
    rho = out["rho"].cpu().numpy()
    nused = out["nused"].cpu().numpy()
    probes = orc.probes(seed, N, Np)
    gp = orc.grid_points(M, (0, 0), (1, 1))
    for k, h in enumerate(hs):
        mh = orc.fit(X, y, h, 1, gp)
        yhat = orc.interp(mh[:, 0], M, (0, 0), (1, 1), X)
        r_ref, mean, _, inc = orc.dof(X, h, 1, M, (0, 0), (1, 1), probes)
        assert nused[k] == inc.sum()
        assert np.abs(rho[k] - r_ref).max() < 1e-6
        rss_ref = np.sum(((y - yhat) ** 2)[inc])
        assert abs(rss[k] / rss_ref - 1) < 1e-5
        g_ref = orc.gcv(y, yhat, mean, include=inc)[0]
        assert abs(gcv[k] / g_ref - 1) < 1e-5
    from paper_2204_07716_amd import select_bandwidth
    assert select_bandwidth(gcv, 0.0) == orc.rgcv_select(gcv, 0.0)
    assert select_bandwidth(gcv, 0.5) == orc.rgcv_select(gcv, 0.5)


@pytest.mark.parametrize("mode", ["log", "direct"])
def test_variance_matches_oracle(orc, mode):
    """Second pass on squared residuals: the mean grid comes from the GPU
    (stage isolation); the oracle repeats eq. 24-26 (or eq. 23) on it."""
    N = 4000
    rng = np.random.default_rng(420)
    X = rng.random((N, 2))
    y = (X ** 2).sum(axis=1) + (0.1 + 0.5 * X[:, 0]) * rng.standard_normal(N)
    M, h = (32, 30), (0.12, 0.12)
    plan = make_plan(2, 1, M, h, h, 1e-6, "fp32", n_max=N, max_weights=3, tprec="fp64")
    plan.set_points(to_dev(X, torch.float32))
    Yd = to_dev(y[:, None], torch.float32)
    mh = plan.fit(h, Yd)[0, 0]
    s2, vhat, kappa = plan.variance(h, Yd, mh, mode=mode)
    s2 = s2.cpu().numpy()
    mh_np = mh.cpu().numpy()
    yhat = orc.interp(mh_np, M, (0, 0), (1, 1), X)
    y32 = y.astype(np.float32).astype(np.float64)
    ref, extra = orc.variance(X, y32, yhat, h, 1, M, (0, 0), (1, 1),
                              mode="log" if mode == "log" else "direct")
    gp = orc.grid_points(M, (0, 0), (1, 1))
    S, _ = orc.moments(X, None, h, 1, gp)
    mask = density_mask(S[:, 0])
    assert rel_err(s2, ref, mask) < 1e-5
    if mode == "log":
        assert abs(kappa.item() / extra["kappa"] - 1) < 1e-6
        assert rel_err(vhat.cpu().numpy(), extra["v"], mask) < 1e-5


def test_complex_response_cv(orc):
    """Complex y: real and imaginary parts share the moment matrix; the GCV
    uses |y - yhat|^2."""
    N, Np = 2500, 4
    rng = np.random.default_rng(430)
    X = rng.random((N, 2))
    y = np.exp(2j * np.pi * X[:, 0]) * (1 + X[:, 1]) + 0.2 * (rng.standard_normal(N) + 1j * rng.standard_normal(N))
    M, h = (34, 30), (0.12, 0.1)
    plan = make_plan(2, 2, M, h, h, 1e-6, "fp32", n_max=N, max_weights=3 + Np, tprec="fp64")
    plan.set_points(to_dev(X, torch.float32))
    out = plan.cv(h, torch.as_tensor(y[:, None].astype(np.complex64), device="cuda"), Np, seed=3)
    mh = out["mhat"].cpu().numpy()[0, 0]
    gp = orc.grid_points(M, (0, 0), (1, 1))
    y32 = y.astype(np.complex64).astype(np.complex128)
    ref, S, T, r0, ill = orc.fit(X, y32, h, 2, gp, return_all=True)
    mask = density_mask(S[:, 0])
    assert rel_err(mh, ref[:, 0], mask) < 1e-5
    yhat = orc.interp(ref[:, 0], M, (0, 0), (1, 1), X)
    inc, _ = orc.support(X, h, 2, M, (0, 0), (1, 1))
    assert out["nused"].cpu().numpy()[0] == inc.sum()
    rss_ref = np.sum((np.abs(y32 - yhat) ** 2)[inc])
    assert abs(out["rss"].cpu().numpy()[0, 0] / rss_ref - 1) < 1e-5


def test_cv_many_probes_two_responses(orc):
    """More weight vectors than one spreading launch or one reduction launch
    holds (2 responses + 20 probes: the rows are staged in two column chunks,
    the spread runs in two launches of at most 8 pairs, the reduction in two
    probe launches, the fit rows without the response column): DF, RSS and
    GCV against the oracle with identical probes."""
    N, Np, seed = 2500, 20, 9
    X, y = _data(430, N, 2)
    y2 = np.cos(2 * X[:, 0]) + 0.1 * np.random.default_rng(431).standard_normal(N)
    Y = np.stack([y, y2], axis=1)
    M, h = (36, 32), (0.09, 0.1)
    plan = make_plan(2, 1, M, h, h, 1e-6, "fp32", n_max=N, max_weights=1 + 2 + Np, tprec="fp64")
    plan.set_points(to_dev(X, torch.float32))
    out = plan.cv(h, to_dev(Y, torch.float32), Np, seed=seed)
    rho = out["rho"].cpu().numpy()[0]
    rss = out["rss"].cpu().numpy()[0]
    gcv = out["gcv"].cpu().numpy()[0]
    probes = orc.probes(seed, N, Np)
    r_ref, mean, _, inc = orc.dof(X, h, 1, M, (0, 0), (1, 1), probes)
    assert np.abs(rho - r_ref).max() < 1e-6
    gp = orc.grid_points(M, (0, 0), (1, 1))
    for c in range(2):
        mh = orc.fit(X, Y[:, c], h, 1, gp)
        yhat = orc.interp(mh[:, 0], M, (0, 0), (1, 1), X)
        rss_ref = np.sum(((Y[:, c] - yhat) ** 2)[inc])
        assert abs(rss[c] / rss_ref - 1) < 1e-5
        g_ref = orc.gcv(Y[:, c], yhat, mean, include=inc)[0]
        assert abs(gcv[c] / g_ref - 1) < 1e-5


@pytest.mark.parametrize("d", [2, 3])
def test_variance_density_channel_reuse(orc, d):
    """The second pass keeps the density moments of the last fit at the same
    h on the same points, and makes them again after a fit at another h or
    after new points: every order agrees with the oracle, and the kept and
    remade moments give the same result to spreading round-off.  In 3-D the
    kept case spreads only the second column (the one-column MFMA pass) and
    the remade case the pair."""
    rng = np.random.default_rng(440)
    if d == 2:
        N = 3000
        X = rng.random((N, 2))
        M, h, h2 = (30, 28), (0.12, 0.11), (0.2, 0.2)
    else:
        N = 20000
        X = rng.random((N, 3))
        M, h, h2 = (18, 17, 16), (0.14, 0.15, 0.13), (0.2, 0.2, 0.2)
    y = (X ** 2).sum(axis=1) + (0.1 + 0.5 * X[:, 1]) * rng.standard_normal(N)
    plan = make_plan(d, 1, M, h, h2, 1e-6, "fp32", n_max=N, max_weights=3, tprec="fp64")
    if d == 3:
        assert plan.geometry.w == 8   # the MFMA spread
    Xd = to_dev(X, torch.float32)
    Yd = to_dev(y[:, None], torch.float32)
    plan.set_points(Xd)
    mh = plan.fit(h, Yd)[0, 0].clone()
    kept = plan.variance(h, Yd, mh)[0].cpu().numpy()
    plan.fit(h2, Yd)
    other = plan.variance(h, Yd, mh)[0].cpu().numpy()
    plan.set_points(Xd)
    fresh = plan.variance(h, Yd, mh)[0].cpu().numpy()
    again = plan.variance(h, Yd, mh)[0].cpu().numpy()
    lo, hi = (0,) * d, (1,) * d
    yhat = orc.interp(mh.cpu().numpy(), M, lo, hi, X)
    y32 = y.astype(np.float32).astype(np.float64)
    ref, _ = orc.variance(X, y32, yhat, h, 1, M, lo, hi, mode="log")
    gp = orc.grid_points(M, lo, hi)
    S, _ = orc.moments(X, None, h, 1, gp)
    mask = density_mask(S[:, 0])
    for got in (kept, other, fresh, again):
        assert rel_err(got, ref, mask) < 1e-5
    # kept and remade moments differ by spreading round-off only: the FP32
    # subgrid cells are rounded from FP64 sums whose order varies between
    # launches, and the pair partner of the density column differs (y or z)
    for got in (kept, other, again):
        assert rel_err(got, fresh, mask) < 1e-7


def test_gcv_call_from_stored_dof(orc):
    """fkr_gcv: GCV of a response against Girard ratios computed earlier by
    fkr_dof (the DF does not depend on y), over a bandwidth list; equals the
    batched cv call and the oracle."""
    N, Np, seed = 3000, 6, 17
    X, y = _data(450, N, 2)
    y2 = np.cos(3 * X[:, 1]) + 0.2 * np.random.default_rng(451).standard_normal(N)
    Y = np.stack([y, y2], axis=1)
    M = (36, 34)
    hs = np.stack([orc.get_hlist(3, [0.07, 0.18], "log")[:, 0]] * 2, axis=1)
    plan = make_plan(2, 1, M, hs[0], hs[-1], 1e-6, "fp32", n_max=N, max_weights=3 + Np,
                     max_h=len(hs), tprec="fp64")
    plan.set_points(to_dev(X, torch.float32))
    rho, nused = plan.dof(hs, Np, seed=seed, want_nused=True)
    Yd = to_dev(Y, torch.float32)
    g = plan.gcv(hs, Yd, rho)
    cv = plan.cv(hs, Yd, Np, seed=seed)
    gcv, gcv_cv = g["gcv"].cpu().numpy(), cv["gcv"].cpu().numpy()
    assert np.allclose(g["nused"].cpu().numpy(), nused.cpu().numpy())
    assert np.abs(gcv / gcv_cv - 1).max() < 1e-6
    probes = orc.probes(seed, N, Np)
    gp = orc.grid_points(M, (0, 0), (1, 1))
    rho = rho.cpu().numpy()
    for k, h in enumerate(hs):
        r_ref, mean, _, inc = orc.dof(X, h, 1, M, (0, 0), (1, 1), probes)
        assert np.abs(rho[k] - r_ref).max() < 1e-6
        for c in range(2):
            mh = orc.fit(X, Y[:, c], h, 1, gp)
            yhat = orc.interp(mh[:, 0], M, (0, 0), (1, 1), X)
            g_ref = orc.gcv(Y[:, c], yhat, mean, include=inc)[0]
            assert abs(gcv[k, c] / g_ref - 1) < 1e-5


def test_unresolved_points_are_left_out_of_dof(orc):
    """Samples on the line x1 = 0.3 plus a cloud in x1 > 0.6: grid points
    near the line see a collinear or nearly collinear local design (singular
    or unresolved), and the samples whose cell touches one are left out of
    the DF and RSS sums on both sides (a finite GCV, the same N_I)."""
    rng = np.random.default_rng(460)
    N, Np, seed = 4000, 6, 19
    X = np.concatenate([np.stack([rng.random(3000), np.full(3000, 0.3)], axis=1),
                        np.stack([rng.random(1000), 0.6 + 0.4 * rng.random(1000)], axis=1)])
    y = np.sin(3 * X[:, 0]) + 0.2 * rng.standard_normal(N)
    M, h = (24, 22), (0.06, 0.06)
    plan = make_plan(2, 1, M, h, h, 1e-9, "fp64", n_max=N, max_weights=2 + Np)
    plan.set_points(to_dev(X))
    out = plan.cv(h, to_dev(y[:, None]), Np, seed=seed)
    probes = orc.probes(seed, N, Np)
    r_ref, mean, _, inc = orc.dof(X, h, 1, M, (0, 0), (1, 1), probes)
    assert 0 < inc.sum() < N
    assert out["nused"].cpu().numpy()[0] == inc.sum()
    assert np.abs(out["rho"].cpu().numpy()[0] - r_ref).max() < 1e-8
    gcv = out["gcv"].cpu().numpy()[0, 0]
    assert np.isfinite(gcv)
    gp = orc.grid_points(M, (0, 0), (1, 1))
    yhat = orc.interp(orc.fit(X, y, h, 1, gp)[:, 0], M, (0, 0), (1, 1), X)
    g_ref = orc.gcv(y, yhat, mean, include=inc)[0]
    assert abs(gcv / g_ref - 1) < 1e-8
