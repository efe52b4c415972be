"""GPU parity of moments and fits with a full bandwidth matrix (eq. 2 with a
general H) against the FP64 oracle's direct sums."""
import numpy as np
import pytest

from gpu_common import compare_fit, make_plan, rel_err, to_dev

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _h_range(H):
    s = np.sqrt(np.diag(H))
    reach = 1.0 / np.sqrt(np.diag(np.linalg.inv(H)))
    return tuple(0.98 * reach), tuple(1.02 * s)


CASES = [
    # d, order, M, H, precision, transform precision
    (2, 1, (40, 36), [[0.010, 0.006], [0.006, 0.016]], "fp64", "same"),
    (2, 2, (32, 30), [[0.012, -0.007], [-0.007, 0.010]], "fp32", "fp64"),
    (3, 1, (14, 13, 12), [[0.030, 0.010, -0.008], [0.010, 0.025, 0.006], [-0.008, 0.006, 0.028]], "fp32", "fp64"),
]


@pytest.mark.parametrize("d,order,M,H,prec,tprec", CASES)
def test_full_h_moments_and_fit_match_oracle(orc, d, order, M, H, prec, tprec):
    H = np.array(H)
    N = 4000
    rng = np.random.default_rng(1000 + d + order)
    X = rng.random((N, d))
    y = np.sin(3 * X).sum(axis=1) + 0.2 * rng.standard_normal(N)
    hmin, hmax = _h_range(H)
    plan = make_plan(d, order, M, hmin, hmax, 1e-10 if prec == "fp64" else 1e-6, prec, n_max=N, max_weights=2,
                     tprec=tprec)
    dt = torch.float64 if prec == "fp64" else torch.float32
    Xr = X.astype(np.float32).astype(np.float64) if prec == "fp32" else X
    yr = y.astype(np.float32).astype(np.float64) if prec == "fp32" else y
    plan.set_points(to_dev(X, dt))
    S_eq, T_eq = plan.moments_full(H, to_dev(y[:, None], dt))
    mh = plan.fit_full(H, to_dev(y[:, None], dt)).cpu().numpy()[0, 0]
    gp = orc.grid_points(M, (0,) * d, (1,) * d)
    S, T = orc.moments_full(Xr, yr[:, None], H, order, gp)
    s = np.sqrt(np.diag(H))
    es = orc.multi_indices(d, 2 * order)
    et = orc.multi_indices(d, order)
    Sg = S_eq.cpu().numpy()[0].T * np.array([np.prod(s ** np.array(a)) for a in es])[None, :]
    Tg = T_eq.cpu().numpy()[0, 0].T * np.array([np.prod(s ** np.array(b)) for b in et])[None, :]
    bar = 1e-8 if prec == "fp64" else 1e-5
    for a in range(len(es)):
        assert rel_err(Sg[:, a], S[:, a]) < bar, (a, rel_err(Sg[:, a], S[:, a]))
    for b in range(len(et)):
        assert rel_err(Tg[:, b], T[:, 0, b]) < bar
    ref, S2, ill = orc.fit_full(Xr, yr, H, order, gp)
    err = compare_fit(mh, ref[:, 0], S2, s, order, d, bar)
    print(f"full H d={d} l={order} {prec}: S err {max(rel_err(Sg[:, a], S[:, a]) for a in range(len(es))):.2e}, "
          f"fit err {err:.2e}")


def test_full_h_diagonal_equals_product_fit():
    """A diagonal H through the full-matrix path equals fkr_fit with h."""
    N, d = 3000, 2
    rng = np.random.default_rng(1010)
    X = rng.random((N, d))
    y = np.cos(4 * X[:, 0]) * X[:, 1] + 0.1 * rng.standard_normal(N)
    h = np.array([0.06, 0.08])
    plan = make_plan(d, 1, (48, 40), tuple(h), tuple(h), 1e-6, "fp32", n_max=N, tprec="fp64")
    plan.set_points(to_dev(X, torch.float32))
    Y = to_dev(y[:, None], torch.float32)
    a = plan.fit_full(np.diag(h ** 2), Y).cpu().numpy()
    b = plan.fit(h, Y).cpu().numpy()
    f = np.isfinite(b)
    assert np.array_equal(np.isnan(a), np.isnan(b))
    # two launches: the FP64 tile sums are added in a varying order before
    # their FP32 store, so the last bit of a subgrid value may differ
    assert np.abs(a[f] - b[f]).max() <= 1e-6 * np.abs(b[f]).max()


def test_full_h_argument_checks():
    from paper_2204_07716_amd._lib import FkrError
    N = 500
    X = np.random.default_rng(3).random((N, 2))
    plan = make_plan(2, 1, (24, 24), (0.08, 0.08), (0.12, 0.12), 1e-6, "fp32", n_max=N, tprec="fp64")
    plan.set_points(to_dev(X, torch.float32))
    Y = to_dev(np.zeros((N, 1)), torch.float32)
    for H in ([[0.01, 0.002], [0.003, 0.01]],      # not symmetric
              [[0.01, 0.011], [0.011, 0.01]],      # not positive definite
              [[0.02, 0.0], [0.0, 0.01]],          # sqrt(H_00) beyond h_max
              [[0.01, 0.009], [0.009, 0.01]]):     # spectrum along w_0 beyond the band (1/sqrt((H^-1)_00) < h_min)
        with pytest.raises(FkrError):
            plan.fit_full(np.array(H), Y)


def test_ll2d_full_size_full_h(orc):
    """The 2-D workload's samples at full size (N = 1e6 mixture, M = 256^2)
    with a full H of marginal widths (0.03, 0.05) and correlation 0.5: the
    density moment and the fit at seeded grid points against the oracle's
    direct sums."""
    import workloads
    from gpu_common import density_mask, sample_flat
    w = workloads.make("ll2d")
    h = np.asarray(w.h[0])
    H = np.array([[h[0] ** 2, 0.5 * h[0] * h[1]], [0.5 * h[0] * h[1], h[1] ** 2]])
    hmin, hmax = _h_range(H)
    plan = make_plan(2, 1, w.M, hmin, hmax, w.eps, "fp32", n_max=w.N, tprec="fp64")
    plan.set_points(to_dev(w.X, torch.float32))
    mh, s0 = plan.fit_full(H, to_dev(w.Y, torch.float32), want_s0=True)
    mh, s0 = mh.cpu().numpy()[0, 0], s0.cpu().numpy()[0]
    flat = sample_flat(np.random.default_rng(66), w.M, 24)
    gp = orc.grid_points(w.M, w.lo, w.hi)[flat]
    X = w.X.astype(np.float32).astype(np.float64)
    y = w.Y[:, 0].astype(np.float32).astype(np.float64)
    ref, S, ill = orc.fit_full(X, y, H, 1, gp)
    assert rel_err(s0[flat], S[:, 0]) < 1e-5
    err = rel_err(mh[flat], ref[:, 0], density_mask(S[:, 0]))
    print(f"ll2d full H: s0 err {rel_err(s0[flat], S[:, 0]):.2e}, fit err {err:.2e}")
    assert err < 1e-5


def test_full_h_cv_matches_oracle(orc):
    """DF, RSS and GCV (eq. 22, Sec. 2.1) over a list of full bandwidth
    matrices, for choosing H by GCV: against the oracle's GCV with the same
    Philox probes; a diagonal H gives what fkr_cv gives at h = sqrt(diag H)."""
    d, order, M, N, Np, seed = 2, 1, (30, 28), 2500, 4, 77
    Hs = np.array([[[0.010, 0.006], [0.006, 0.016]], [[0.012, -0.005], [-0.005, 0.009]], [[0.011, 0.0], [0.0, 0.014]]])
    rng = np.random.default_rng(1010)
    X = rng.random((N, d))
    y = np.sin(3 * X).sum(axis=1) + 0.2 * rng.standard_normal(N)
    lo_r = [min(_h_range(H)[0][j] for H in Hs) for j in range(d)]
    hi_r = [max(_h_range(H)[1][j] for H in Hs) for j in range(d)]
    plan = make_plan(d, order, M, tuple(lo_r), tuple(hi_r), 1e-10, "fp64", n_max=N, max_weights=2 + Np, max_h=3)
    plan.set_points(to_dev(X))
    Y = to_dev(y[:, None])
    out = plan.cv_full(Hs, Y, Np, seed=seed)
    Wp = orc.probes(seed, N, Np)
    lo, hi = (0.0,) * d, (1.0,) * d
    for k, H in enumerate(Hs):
        inc = orc.support(X, None, order, M, lo, hi, H=H)[0]
        ref = orc.gcv_criterion(X, y, None, order, M, lo, hi, Wp, inc, H=H)
        rho, _, _, _ = orc.dof(X, np.sqrt(np.diag(H)), order, M, lo, hi, Wp, include=inc) if k == 2 else (None,) * 4
        got = out["gcv"][k, 0].item()
        print(f"H {k}: gcv {got:.12e} / {ref:.12e}; N_I {out['nused'][k].item():.0f} / {inc.sum()}")
        assert out["nused"][k].item() == inc.sum()
        assert got == pytest.approx(ref, rel=1e-9)
        if rho is not None:
            np.testing.assert_allclose(out["rho"][k].cpu().numpy(), rho, rtol=1e-9)
    # the diagonal matrix through fkr_cv at h = sqrt(diag H)
    base = plan.cv(tuple(np.sqrt(np.diag(Hs[2]))), Y, Np, seed=seed)
    assert out["gcv"][2, 0].item() == pytest.approx(base["gcv"][0, 0].item(), rel=1e-10)


@pytest.mark.parametrize("prec,tprec", [("fp64", "same"), ("fp32", "fp64")])
def test_full_h_interval_matches_oracle(orc, prec, tprec):
    """Variance of the fit and band (eq. 27-28) at a full bandwidth matrix:
    Q from the pass at H / 2; against the oracle's Sigma from its definition
    (full-H smoother weights), for a constant and a gridded sigma^2, and the
    diagonal H against fkr_interval at h = sqrt(diag H)."""
    d, order, M, N = 2, 1, (26, 24), 3000
    H = np.array([[0.012, 0.005], [0.005, 0.016]])
    Hd = np.diag([0.011, 0.014])
    lo_r = tuple(np.minimum(_h_range(H / 2)[0], _h_range(Hd / 2)[0]))
    hi_r = tuple(np.maximum(_h_range(H)[1], _h_range(Hd)[1]))
    rng = np.random.default_rng(1020)
    X = rng.random((N, d))
    y = np.sin(3 * X).sum(axis=1) + 0.2 * rng.standard_normal(N)
    plan = make_plan(d, order, M, lo_r, hi_r, 1e-10 if prec == "fp64" else 1e-6, prec, n_max=N, max_weights=2,
                     tprec=tprec)
    dt = torch.float64 if prec == "fp64" else torch.float32
    Xr = X.astype(np.float32).astype(np.float64) if prec == "fp32" else X
    plan.set_points(to_dev(X, dt))
    mh = plan.fit_full(H, to_dev(y[:, None], dt))[0, 0]
    gp = orc.grid_points(M, (0,) * d, (1,) * d)
    flat = np.arange(0, gp.shape[0], 7)
    out = plan.interval(None, 0.3, mhat=mh, alpha=0.05, H=H)
    ref = orc.fit_variance(Xr, 0.3, None, order, gp[flat], H=H)
    s2_grid = 0.1 + gp[:, 0] ** 2
    out_g = plan.interval(None, to_dev(s2_grid), H=H)
    ref_g = orc.fit_variance(Xr, orc.interp(s2_grid, M, (0,) * d, (1,) * d, Xr), None, order, gp[flat], H=H)
    got = out["Sigma"].cpu().numpy()[flat]
    ok = np.isfinite(ref) & np.isfinite(got)
    bar = 1e-8 if prec == "fp64" else 1e-5
    e_c = rel_err(got, ref, ok)
    e_g = rel_err(out_g["Sigma"].cpu().numpy()[flat], ref_g, ok)
    half = 0.5 * (out["upper"] - out["lower"]).cpu().numpy()[flat]
    e_b = rel_err(half, 1.959963984540054 * np.sqrt(np.maximum(ref, 0.0)), ok)
    print(f"full-H interval {prec}: Sigma {e_c:.2e}, gridded sigma^2 {e_g:.2e}, band {e_b:.2e}")
    assert e_c < bar and e_g < bar and e_b < bar
    d1 = plan.interval(None, 0.3, H=Hd)["Sigma"].cpu().numpy()
    d2 = plan.interval(tuple(np.sqrt(np.diag(Hd))), 0.3)["Sigma"].cpu().numpy()
    fin = np.isfinite(d2)
    assert rel_err(d1, d2, fin) < (1e-10 if prec == "fp64" else 1e-5)


def test_full_h_variance_pass_matches_oracle(orc):
    """The conditional-variance pass (Sec. 3, eq. 23-26) with the second fit
    at a full bandwidth matrix, after the fit at that matrix: against the
    oracle's pass (the same residuals from the GPU fit)."""
    d, order, M, N = 2, 1, (26, 24), 4000
    H = np.array([[0.012, 0.005], [0.005, 0.016]])
    hmin, hmax = _h_range(H)
    rng = np.random.default_rng(1030)
    X = rng.random((N, d))
    y = X[:, 0] ** 2 + (0.2 + 0.5 * X[:, 1]) * rng.standard_normal(N)
    plan = make_plan(d, order, M, hmin, hmax, 1e-10, "fp64", n_max=N, max_weights=2)
    plan.set_points(to_dev(X))
    Y = to_dev(y[:, None])
    mh = plan.fit_full(H, Y)[0, 0]
    lo, hi = (0.0,) * d, (1.0,) * d
    yhat = orc.interp(mh.cpu().numpy(), M, lo, hi, X)
    gp = orc.grid_points(M, lo, hi)
    fin = np.isfinite(orc.fit_full(X, y, H, order, gp)[0][:, 0])
    for mode in ("log", "direct"):
        s2 = plan.variance(None, Y, mh, mode=mode, H=H)[0].cpu().numpy()
        ref, _ = orc.variance(X, y, yhat, None, order, M, lo, hi, mode=mode, H=H)
        ok = fin & np.isfinite(ref) & np.isfinite(s2)
        err = rel_err(s2, ref, ok)
        print(f"full-H variance pass {mode}: rel err {err:.2e} over {ok.sum()} points")
        assert ok.sum() > 0.9 * fin.sum() and err < 1e-8


def test_full_h_argument_errors():
    """The full-H calls refuse what they cannot serve before enqueuing work:
    a non-symmetric or indefinite H, an H outside the plan's bandwidth range,
    more matrices than the plan holds (FKR_E_ARG); a compact kernel
    (FKR_E_UNSUPPORTED)."""
    from paper_2204_07716_amd._lib import FKR_E_ARG, FKR_E_UNSUPPORTED, FkrError
    N = 500
    X = np.random.default_rng(5).random((N, 2))
    H = np.array([[0.010, 0.004], [0.004, 0.012]])
    hmin, hmax = _h_range(H / 2)[0], _h_range(H)[1]
    plan = make_plan(2, 1, (24, 24), hmin, hmax, 1e-6, "fp64", n_max=N, max_weights=4, max_h=1)
    plan.set_points(to_dev(X))
    Y = to_dev(np.sin(X[:, 0])[:, None])
    bad = [np.array([[0.010, 0.004], [0.001, 0.012]]),            # not symmetric
           np.array([[0.010, 0.012], [0.012, 0.012]]),            # not positive definite
           4.0 * H]                                               # wider than the plan's h_max
    for B in bad:
        for call in (lambda: plan.cv_full(B, Y, 2), lambda: plan.interval(None, 0.1, H=B),
                     lambda: plan.fit_full(B, Y)):
            with pytest.raises(FkrError) as e:
                call()
            assert e.value.status == FKR_E_ARG
    with pytest.raises(FkrError) as e:
        plan.cv_full(np.stack([H, H]), Y, 2)                      # max_h = 1
    assert e.value.status == FKR_E_ARG
    pc = make_plan(2, 1, (24, 24), hmin, hmax, 1e-6, "fp64", n_max=N, max_weights=4, reg_kernel="epanechnikov")
    pc.set_points(to_dev(X))
    mh = torch.zeros(24 * 24, dtype=torch.float64, device="cuda")
    for call in (lambda: pc.cv_full(H, Y, 2), lambda: pc.interval(None, 0.1, H=H),
                 lambda: pc.variance(None, Y, mh, H=H)):
        with pytest.raises(FkrError) as e:
            call()
        assert e.value.status == FKR_E_UNSUPPORTED


def test_full_h_gcv_grad_matches_oracle(orc):
    """GCV gradient in the entries of a full bandwidth matrix (the derivative
    of the multivariate Hermite multipliers, the Gaussian factor and the
    equilibration, then the derivative of the solve and the sums): against
    central differences of the oracle's GCV with the same Philox probes; at a
    diagonal H, the log-h gradient of fkr_gcv_grad over 2 H_jj."""
    d, order, M, N, Np, seed = 2, 1, (28, 26), 2000, 4, 91
    H = np.array([[0.012, 0.005], [0.005, 0.016]])
    Hd = np.diag([0.011, 0.015])
    lo_r = tuple(np.minimum(_h_range(H)[0], _h_range(Hd)[0]) * 0.99)
    hi_r = tuple(np.maximum(_h_range(H)[1], _h_range(Hd)[1]) * 1.01)
    rng = np.random.default_rng(1040)
    X = rng.random((N, d))
    y = np.sin(3 * (X[:, 0] + 0.5 * X[:, 1])) + 0.3 * rng.standard_normal(N)
    plan = make_plan(d, order, M, lo_r, hi_r, 1e-10, "fp64", n_max=N, max_weights=16)
    plan.set_points(to_dev(X))
    Y = to_dev(y[:, None])
    out = plan.gcv_grad_full(H, Y, Np, seed)
    Wp = orc.probes(seed, N, Np)
    lo, hi = (0.0,) * d, (1.0,) * d
    inc = orc.support(X, None, order, M, lo, hi, H=H)[0]
    assert inc.all()
    ref_g = orc.gcv_criterion(X, y, None, order, M, lo, hi, Wp, inc, H=H)
    ref = orc.gcv_H_gradient(X, y, H, order, M, lo, hi, Wp, include=inc, step=1e-4)
    got = out["dH"].cpu().numpy()
    err = np.abs(got - ref).max() / np.abs(ref).max()
    print(f"full-H gradient: gcv {out['gcv'].item():.10e} / {ref_g:.10e}; dGCV/dH {got} / {ref}; rel err {err:.2e}")
    assert out["gcv"].item() == pytest.approx(ref_g, rel=1e-9)
    assert err < 1e-6
    # the diagonal matrix against the log-h gradient
    gd = plan.gcv_grad_full(Hd, Y, Np, seed)["dH"].cpu().numpy()
    gl = plan.gcv_grad(tuple(np.sqrt(np.diag(Hd))), Y, Np, seed, want_dy=False)["dlogh"].cpu().numpy()
    np.testing.assert_allclose([2 * Hd[0, 0] * gd[0], 2 * Hd[1, 1] * gd[2]], gl, rtol=1e-8,
                               atol=1e-10 * np.abs(gl).max())


@pytest.mark.parametrize("cplx", [False, True])
def test_full_h_gcv_y_gradient_matches_oracle(orc, cplx):
    """GCV gradient in y at a full bandwidth matrix (the adjoint of the
    smoother: residuals scattered to the grid, the full-H multipliers with
    the conjugate phase, the type-2 transform to the samples) against the
    oracle's explicit smoother of the full-H fits; real and complex y.  At a
    diagonal H it is fkr_gcv_grad's y gradient at h = sqrt(diag H)."""
    d, order, M, N, Np, seed = 2, 1, (26, 24), 500, 4, 93
    H = np.array([[0.014, 0.006], [0.006, 0.018]])
    Hd = np.diag([0.013, 0.017])
    lo_r = tuple(np.minimum(_h_range(H)[0], _h_range(Hd)[0]) * 0.99)
    hi_r = tuple(np.maximum(_h_range(H)[1], _h_range(Hd)[1]) * 1.01)
    rng = np.random.default_rng(1045 + cplx)
    X = rng.random((N, d))
    y = np.sin(3 * (X[:, 0] + 0.5 * X[:, 1])) + 0.3 * rng.standard_normal(N)
    if cplx:
        y = y + 1j * (np.cos(2 * X[:, 1]) + 0.3 * rng.standard_normal(N))
    plan = make_plan(d, order, M, lo_r, hi_r, 1e-10, "fp64", n_max=N, max_weights=16)
    plan.set_points(to_dev(X))
    Y = torch.as_tensor(y[:, None]).to("cuda")
    out = plan.gcv_grad_full(H, Y, Np, seed)
    Wp = orc.probes(seed, N, Np)
    lo, hi = (0.0,) * d, (1.0,) * d
    inc = orc.support(X, None, order, M, lo, hi, H=H)[0]
    assert inc.all()
    ref = orc.gcv_y_gradient(X, y, None, order, M, lo, hi, Wp, include=inc, H=H)
    got = out["dy"].cpu().numpy().reshape(-1)
    err = np.abs(got - ref).max() / np.abs(ref).max()
    print(f"full-H d GCV / dy ({'complex' if cplx else 'real'} y): rel err {err:.2e}")
    assert err < 1e-9
    gd = plan.gcv_grad_full(Hd, Y, Np, seed)["dy"].cpu().numpy()
    gh = plan.gcv_grad(tuple(np.sqrt(np.diag(Hd))), Y, Np, seed)["dy"].cpu().numpy()
    assert np.abs(gd - gh).max() <= 1e-10 * np.abs(gh).max()
    if cplx:   # GCV of a complex y is that of its real part plus that of its imaginary part
        parts = [plan.gcv_grad_full(H, to_dev(v[:, None]), Np, seed, want_dy=False) for v in (y.real, y.imag)]
        assert out["gcv"].item() == pytest.approx(sum(q["gcv"].item() for q in parts), rel=1e-12)
        np.testing.assert_allclose(out["dH"].cpu().numpy(), sum(q["dH"].cpu().numpy() for q in parts),
                                   rtol=1e-10, atol=1e-12 * np.abs(out["dH"].cpu().numpy()).max())
    # dy is optional: the same GCV and H gradient without it
    nody = plan.gcv_grad_full(H, Y, Np, seed, want_dy=False)
    assert nody["dy"] is None
    assert nody["gcv"].item() == pytest.approx(out["gcv"].item(), rel=1e-13)   # atomic sums: rounding order
    np.testing.assert_allclose(nody["dH"].cpu().numpy(), out["dH"].cpu().numpy(), rtol=1e-9)


def test_full_h_gcv_gradients_3d(orc):
    """Both GCV gradients at a 3-D full bandwidth matrix with three nonzero
    off-diagonal entries (six directions of the Hermite recurrence's
    derivative; the adjoint with the 3-D multipliers): in H against central
    differences of the oracle's GCV, in y against its explicit smoother."""
    d, order, M, N, Np, seed = 3, 1, (14, 13, 12), 700, 3, 95
    H = np.array([[0.030, 0.010, -0.008], [0.010, 0.025, 0.006], [-0.008, 0.006, 0.028]])
    lo_r, hi_r = _h_range(H)
    rng = np.random.default_rng(1047)
    X = rng.random((N, d))
    y = np.sin(2 * (X[:, 0] + X[:, 1] - X[:, 2])) + 0.3 * rng.standard_normal(N)
    plan = make_plan(d, order, M, lo_r, hi_r, 1e-10, "fp64", n_max=N, max_weights=16)
    plan.set_points(to_dev(X))
    out = plan.gcv_grad_full(H, to_dev(y[:, None]), Np, seed)
    Wp = orc.probes(seed, N, Np)
    lo, hi = (0.0,) * d, (1.0,) * d
    inc = orc.support(X, None, order, M, lo, hi, H=H)[0]
    ref_g = orc.gcv_criterion(X, y, None, order, M, lo, hi, Wp, inc, H=H)
    ref_H = orc.gcv_H_gradient(X, y, H, order, M, lo, hi, Wp, include=inc, step=1e-4)
    ref_y = orc.gcv_y_gradient(X, y, None, order, M, lo, hi, Wp, include=inc, H=H)
    got_H = out["dH"].cpu().numpy()
    got_y = out["dy"].cpu().numpy()
    e_H = np.abs(got_H - ref_H).max() / np.abs(ref_H).max()
    e_y = np.abs(got_y - ref_y).max() / np.abs(ref_y).max()
    print(f"3-D full H ({inc.sum()} of {N} supported): gcv {out['gcv'].item():.10e} / {ref_g:.10e}; "
          f"dGCV/dH rel err {e_H:.2e}; dGCV/dy rel err {e_y:.2e}")
    assert out["gcv"].item() == pytest.approx(ref_g, rel=1e-9)
    assert e_H < 1e-6 and e_y < 1e-9


def test_full_h_autograd():
    """GCVFullH through torch.autograd: the gradient of GCV(H(t)) for a
    symmetric path H(t) = H0 + t D equals sum(G * D), checked against central
    differences of the GPU's own GCV along D."""
    from paper_2204_07716_amd import GCVFullH
    d, M, N, Np, seed = 2, (24, 22), 1500, 4, 5
    H0 = np.array([[0.012, 0.004], [0.004, 0.015]])
    D = np.array([[0.3, -0.5], [-0.5, 0.8]]) * 1e-3
    lo_r = tuple(np.array(_h_range(H0)[0]) * 0.9)
    hi_r = tuple(np.array(_h_range(H0)[1]) * 1.1)
    rng = np.random.default_rng(1050)
    X = rng.random((N, d))
    y = np.cos(2 * X[:, 0] * X[:, 1] + X[:, 0]) + 0.3 * rng.standard_normal(N)
    plan = make_plan(d, 1, M, lo_r, hi_r, 1e-10, "fp64", n_max=N, max_weights=16)
    plan.set_points(to_dev(X))
    Y = to_dev(y[:, None])
    t = torch.zeros((), dtype=torch.float64, requires_grad=True)
    H = torch.as_tensor(H0) + t * torch.as_tensor(D)
    g = GCVFullH.apply(H, Y, plan, Np, seed)
    g.backward()
    e = 1e-2
    up = plan.cv_full(H0 + e * D, Y, Np, seed=seed)["gcv"][0, 0].item()
    dn = plan.cv_full(H0 - e * D, Y, Np, seed=seed)["gcv"][0, 0].item()
    fd = (up - dn) / (2 * e)
    print(f"autograd dGCV/dt {t.grad.item():.8e}, central differences {fd:.8e}")
    assert t.grad.item() == pytest.approx(fd, rel=1e-5)
    # the response: GCV is quadratic in y, so central differences along a
    # direction v are exact up to rounding
    Yg = Y[:, 0].clone().requires_grad_(True)
    GCVFullH.apply(torch.as_tensor(H0), Yg, plan, Np, seed).backward()
    v = to_dev(np.random.default_rng(7).standard_normal(N))
    e = 1e-2
    up = plan.cv_full(H0, (Y[:, 0] + e * v)[:, None], Np, seed=seed)["gcv"][0, 0].item()
    dn = plan.cv_full(H0, (Y[:, 0] - e * v)[:, None], Np, seed=seed)["gcv"][0, 0].item()
    fd_y = (up - dn) / (2 * e)
    dd = float((Yg.grad * v).sum())
    print(f"autograd dGCV/dy . v {dd:.8e}, central differences {fd_y:.8e}")
    assert dd == pytest.approx(fd_y, rel=1e-7)
