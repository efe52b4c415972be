"""GPU parity of the GCV gradient in log h (eq. 22, Sec. 2.1): the library's
hand-written derivative (derivative moment multipliers, the derivative of
the normal-equation solve, sums over the supported samples) against central
differences of the GPU's own GCV and fits, against the oracle's gradient, and
through torch.autograd."""
import numpy as np
import pytest

from gpu_common import make_plan, to_dev

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _setup(d, N, seed):
    rng = np.random.default_rng(seed)
    X = rng.random((N, d))
    y = np.sin(3 * X).sum(axis=1) + 0.3 * rng.standard_normal(N)
    M, h = {1: ((60,), (0.06,)), 2: ((30, 26), (0.1, 0.12)), 3: ((12, 11, 10), (0.17, 0.16, 0.18))}[d]
    return X, y, M, np.array(h)


def _plan(d, M, h, N, Np, prec, tprec, order=1):
    n_s = {1: 3, 2: 6, 3: 10}[d] if order == 1 else None
    n_t = d + 1
    mw = 2 * (2 + Np) + n_s // n_t + 2
    return make_plan(d, order, M, tuple(0.9 * h), tuple(1.1 * h), 1e-10 if prec == "fp64" else 1e-6, prec,
                     n_max=N, max_weights=mw, max_h=1, tprec=tprec)


@pytest.mark.parametrize("d", [1, 2, 3])
def test_gcv_grad_matches_finite_differences(d):
    """FP64 path: the gradient and the derivative grids d m_hat / d log h_j
    against central differences (step 1e-4 in log h) of the GPU's own GCV
    and fits; the supported set does not change across the steps."""
    N, Np, seed = 3000, 6, 21
    X, y, M, h = _setup(d, N, 500 + d)
    plan = _plan(d, M, h, N, Np, "fp64", "same")
    plan.set_points(to_dev(X))
    Y = to_dev(y[:, None])
    out = plan.gcv_grad(h, Y, Np, seed)
    g = out["dlogh"].cpu().numpy()
    dfit = out["dfit"].cpu().numpy()
    base = plan.cv(h, Y, Np, seed=seed)
    assert out["gcv"].item() == pytest.approx(base["gcv"].item(), rel=1e-10)
    st = 1e-4
    for j in range(d):
        e = np.zeros(d)
        e[j] = st
        up = plan.cv(h * np.exp(e), Y, Np, seed=seed)
        dn = plan.cv(h * np.exp(-e), Y, Np, seed=seed)
        assert up["nused"].item() == dn["nused"].item() == base["nused"].item()
        fd = (up["gcv"].item() - dn["gcv"].item()) / (2 * st)
        print(f"d={d} j={j}: grad {g[j]:.8e} fd {fd:.8e}")
        assert g[j] == pytest.approx(fd, rel=1e-6, abs=1e-9 * abs(base["gcv"].item()))
        fdm = (up["mhat"].cpu().numpy()[0, 0] - dn["mhat"].cpu().numpy()[0, 0]) / (2 * st)
        fin = np.isfinite(dfit[j, 0])
        scale = np.abs(fdm[fin]).max()
        assert np.abs(dfit[j, 0][fin] - fdm[fin]).max() < 1e-6 * scale


@pytest.mark.parametrize("d,prec,tprec", [(1, "fp64", "same"), (2, "fp32", "fp64"), (3, "fp32", "fp64")])
def test_gcv_grad_matches_oracle(orc, d, prec, tprec):
    """Against the oracle's gradient (central differences of the plain GCV
    with the same Philox probes and the supported set of h)."""
    N, Np, seed = 2500, 6, 33
    X, y, M, h = _setup(d, N, 600 + d)
    plan = _plan(d, M, h, N, Np, prec, tprec)
    dt = torch.float64 if prec == "fp64" else torch.float32
    plan.set_points(to_dev(X, dt))
    out = plan.gcv_grad(h, to_dev(y[:, None], dt), Np, seed)
    g = out["dlogh"].cpu().numpy()
    Xr = X.astype(np.float32).astype(np.float64) if prec == "fp32" else X
    yr = y.astype(np.float32).astype(np.float64) if prec == "fp32" else y
    Wp = orc.probes(seed, N, Np)
    if prec == "fp32":
        Wp = Wp.astype(np.float32).astype(np.float64)
    lo, hi = (0.0,) * d, (1.0,) * d
    inc = orc.support(Xr, h, 1, M, lo, hi)[0]
    assert inc.all()
    ref_g = orc.gcv_criterion(Xr, yr, h, 1, M, lo, hi, Wp, inc)
    ref = orc.gcv_log_h_gradient(Xr, yr, h, 1, M, lo, hi, Wp, include=inc, step=1e-4)
    err = np.abs(g - ref).max() / np.abs(ref).max()
    print(f"d={d} {prec}: gcv {out['gcv'].item():.10e} / {ref_g:.10e}; grad {g} / {ref}; rel err {err:.2e}")
    assert out["gcv"].item() == pytest.approx(ref_g, rel=1e-9 if prec == "fp64" else 1e-5)
    assert err < (1e-6 if prec == "fp64" else 1e-5)   # FP64: the oracle's central differences (step 1e-4)


@pytest.mark.parametrize("d", [1, 2, 3])
def test_gcv_y_grad_matches_finite_differences(d):
    """FP64 path: GCV is quadratic in y, so central differences in y_i are
    exact up to rounding; the gradient of the adjoint (type-2) path must
    match them at every checked sample."""
    N, Np, seed = 2000, 4, 8
    X, y, M, h = _setup(d, N, 800 + d)
    plan = _plan(d, M, h, N, Np, "fp64", "same")
    plan.set_points(to_dev(X))
    out = plan.gcv_grad(h, to_dev(y[:, None]), Np, seed)
    dy = out["dy"].cpu().numpy()
    scale = np.abs(dy).max()
    for i in range(0, N, 97):
        e = np.zeros(N)
        e[i] = 0.05
        up = plan.cv(h, to_dev((y + e)[:, None]), Np, seed=seed)["gcv"].item()
        dn = plan.cv(h, to_dev((y - e)[:, None]), Np, seed=seed)["gcv"].item()
        fd = (up - dn) / 0.1
        assert abs(dy[i] - fd) < 1e-7 * scale, (i, dy[i], fd)


@pytest.mark.parametrize("d,prec,tprec", [(1, "fp64", "same"), (2, "fp64", "same"), (2, "fp32", "fp64"),
                                          (3, "fp32", "fp64")])
def test_gcv_y_grad_matches_oracle(orc, d, prec, tprec):
    """Against the oracle's gradient from the explicit smoother (fits of the
    unit responses), same Philox probes."""
    N, Np, seed = {1: 400, 2: 500, 3: 600}[d], 4, 12
    X, y, M, h = _setup(d, N, 900 + d)
    plan = _plan(d, M, h, N, Np, prec, tprec)
    dt = torch.float64 if prec == "fp64" else torch.float32
    plan.set_points(to_dev(X, dt))
    out = plan.gcv_grad(h, to_dev(y[:, None], dt), Np, seed)
    dy = out["dy"].cpu().numpy()
    Xr = X.astype(np.float32).astype(np.float64) if prec == "fp32" else X
    yr = y.astype(np.float32).astype(np.float64) if prec == "fp32" else y
    Wp = orc.probes(seed, N, Np)
    if prec == "fp32":
        Wp = Wp.astype(np.float32).astype(np.float64)
    lo, hi = (0.0,) * d, (1.0,) * d
    inc = orc.support(Xr, h, 1, M, lo, hi)[0]
    ref = orc.gcv_y_gradient(Xr, yr, h, 1, M, lo, hi, Wp, include=inc)
    err = np.abs(dy - ref).max() / np.abs(ref).max()
    print(f"d={d} {prec}: dy rel err {err:.2e} ({inc.sum()} of {N} supported)")
    assert err < (1e-8 if prec == "fp64" else 1e-5)


def test_gcv_autograd_backward():
    from paper_2204_07716_amd import GCVLogH
    N, Np, seed, d = 2000, 4, 5, 2
    X, y, M, h = _setup(d, N, 700)
    plan = _plan(d, M, h, N, Np, "fp32", "fp64")
    plan.set_points(to_dev(X, torch.float32))
    Y = to_dev(y[:, None], torch.float32).requires_grad_(True)
    log_h = torch.tensor(np.log(h), dtype=torch.float64, requires_grad=True)
    gcv = GCVLogH.apply(log_h, Y, plan, Np, seed)
    gcv.backward()
    ref = plan.gcv_grad(h, Y.detach(), Np, seed)
    # two calls with FP32 spreading: the subgrids' FP32 stores may differ in
    # the last bit (their FP64 tile sums are added in a varying order)
    assert gcv.item() == pytest.approx(ref["gcv"].item(), rel=1e-6)
    np.testing.assert_allclose(log_h.grad.numpy(), ref["dlogh"].cpu().numpy(), rtol=1e-5)
    np.testing.assert_allclose(Y.grad.cpu().numpy()[:, 0], ref["dy"].cpu().numpy(), rtol=1e-6,
                               atol=1e-6 * ref["dy"].abs().max().item())


def test_gcv_grad_complex_local_quadratic_matches_oracle(orc):
    """Complex y (the differentiated workload's kind of response), local
    quadratic in 2-D, FP32 spreading: GCV, its gradient in log h and its
    gradient d/dRe y + i d/dIm y against the oracle."""
    N, Np, seed, d = 600, 4, 19, 2
    rng = np.random.default_rng(950)
    X = rng.random((N, d))
    y = (np.exp(3j * X[:, 0]) * (1 + X[:, 1]) + 0.2 * (rng.standard_normal(N) + 1j * rng.standard_normal(N)))
    M, h = (24, 20), np.array([0.12, 0.14])
    plan = make_plan(2, 2, M, tuple(0.9 * h), tuple(1.1 * h), 1e-6, "fp32", n_max=N, max_weights=16, tprec="fp64")
    plan.set_points(to_dev(X, torch.float32))
    yc = y.astype(np.complex64)
    out = plan.gcv_grad(h, torch.as_tensor(yc, device="cuda"), Np, seed)
    Xr = X.astype(np.float32).astype(np.float64)
    yr = yc.astype(np.complex128)
    Wp = orc.probes(seed, N, Np).astype(np.float32).astype(np.float64)
    lo, hi = (0.0, 0.0), (1.0, 1.0)
    inc = orc.support(Xr, h, 2, M, lo, hi)[0]
    g_ref = orc.gcv_criterion(Xr, yr, h, 2, M, lo, hi, Wp, inc)
    dl_ref = orc.gcv_log_h_gradient(Xr, yr, h, 2, M, lo, hi, Wp, include=inc)
    dy_ref = orc.gcv_y_gradient(Xr, yr, h, 2, M, lo, hi, Wp, include=inc)
    dl = out["dlogh"].cpu().numpy()
    dy = out["dy"].cpu().numpy()
    e_l = np.abs(dl - dl_ref).max() / np.abs(dl_ref).max()
    e_y = np.abs(dy - dy_ref).max() / np.abs(dy_ref).max()
    print(f"complex l=2: gcv {out['gcv'].item():.8e}/{g_ref:.8e}; dlogh err {e_l:.2e}; dy err {e_y:.2e}; "
          f"{inc.sum()} of {N} supported")
    assert out["gcv"].item() == pytest.approx(g_ref, rel=1e-5)
    assert e_l < 1e-5 and e_y < 1e-5


def test_cplx2d_full_size_gradients():
    """The differentiated workload at full size (complex Lorentzian peaks,
    N = 4e6, M = 512^2, local quadratic, h = 0.02, 10 probes, FP32
    spreading) through GCVLogH: GCV is quadratic in y, so its central
    difference along the gradient's own direction equals the directional
    derivative (checked to 1e-4, the FP32 noise of GCV over the step); the
    log-h gradient against central differences of GCV (step 1e-3, to 1e-3)."""
    import workloads
    from paper_2204_07716_amd import GCVLogH
    w = workloads.make("cplx2d")
    h = np.asarray(w.h[0])
    Np, seed = w.n_probes, w.probe_seed
    plan = make_plan(2, 2, w.M, tuple(0.99 * h), tuple(1.01 * h), w.eps, "fp32", n_max=w.N, max_weights=28,
                     tprec="fp64")
    plan.set_points(to_dev(w.X, torch.float32))
    Y = torch.as_tensor(w.Y[:, 0].astype(np.complex64), device="cuda").requires_grad_(True)
    log_h = torch.tensor(np.log(h), dtype=torch.float64, requires_grad=True)
    G = GCVLogH.apply(log_h, Y, plan, Np, seed)
    G.backward()
    G = G.item()
    dy = Y.grad.detach().to(torch.complex128)
    assert np.isfinite(G) and torch.isfinite(torch.view_as_real(dy)).all()
    v = dy / torch.linalg.vector_norm(dy)
    eps = 0.1 * G / torch.linalg.vector_norm(dy).item()            # about a 10% change of GCV
    Yd = Y.detach().to(torch.complex128)
    up = plan.cv(h, (Yd + eps * v).to(torch.complex64), Np, seed=seed)["gcv"].item()
    dn = plan.cv(h, (Yd - eps * v).to(torch.complex64), Np, seed=seed)["gcv"].item()
    dirv = torch.linalg.vector_norm(dy).item()                    # <dy, v> for v along dy
    fd = (up - dn) / (2 * eps)
    print(f"cplx2d: GCV {G:.6e}; directional derivative {dirv:.6e} vs central difference {fd:.6e}")
    assert fd == pytest.approx(dirv, rel=1e-4)
    dl = log_h.grad.numpy()
    Yc = Y.detach()
    for j in range(2):
        e = np.zeros(2)
        e[j] = 1e-3
        gp = plan.cv(h * np.exp(e), Yc, Np, seed=seed)["gcv"].item()
        gm = plan.cv(h * np.exp(-e), Yc, Np, seed=seed)["gcv"].item()
        fdl = (gp - gm) / 2e-3
        print(f"cplx2d: d GCV / d log h_{j} {dl[j]:.6e} vs central difference {fdl:.6e}")
        assert dl[j] == pytest.approx(fdl, rel=1e-3, abs=1e-3 * G)
