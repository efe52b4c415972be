"""GPU parity of the compact regression kernels of Table 1 (box, triangle,
Epanechnikov, biweight, triweight): the moments are the binned
approximation of eq. (11)-(13) (the kernel sampled at the grid offsets, its
discrete transform over every mode of the period), checked against the
oracle's definition of that approximation; its distance to the exact kernel
sums is the method's error, reported per kernel."""
import numpy as np
import pytest

from gpu_common import compare_fit, make_plan, rel_err, sample_flat, to_dev

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

KERNELS = ["box", "triangle", "epanechnikov", "biweight", "triweight"]


@pytest.mark.parametrize("name", KERNELS)
@pytest.mark.parametrize("d,order,prec,tprec", [(1, 2, "fp64", "same"), (2, 1, "fp32", "fp64")])
def test_compact_moments_and_fit_match_binned_oracle(orc, name, d, order, prec, tprec):
    N = 3000 if d == 1 else 5000
    M, h = {1: ((200,), (0.05,)), 2: ((48, 40), (0.12, 0.14))}[d]
    rng = np.random.default_rng(1100 + d + KERNELS.index(name))
    X = rng.random((N, d))
    y = np.sin(3 * X).sum(axis=1) + 0.2 * rng.standard_normal(N)
    plan = make_plan(d, order, M, h, h, 1e-10 if prec == "fp64" else 1e-6, prec, n_max=N, tprec=tprec,
                     reg_kernel=name)
    dt = torch.float64 if prec == "fp64" else torch.float32
    Xr = X.astype(np.float32).astype(np.float64) if prec == "fp32" else X
    yr = y.astype(np.float32).astype(np.float64) if prec == "fp32" else y
    plan.set_points(to_dev(X, dt))
    S_eq, T_eq = plan.moments(h, to_dev(y[:, None], dt))
    mh = plan.fit(h, to_dev(y[:, None], dt)).cpu().numpy()[0, 0]
    g = plan.geometry
    L = [g.L[j] for j in range(d)]
    delta = [g.delta[j] for j in range(d)]
    flat = sample_flat(np.random.default_rng(5), M, 40)
    gp = orc.grid_points(M, (0,) * d, (1,) * d)[flat]
    S, T = orc.moments_binned(Xr, yr[:, None], h, order, gp, name, delta, L)
    es = orc.multi_indices(d, 2 * order)
    et = orc.multi_indices(d, order)
    hh = np.asarray(h)
    Sg = S_eq.cpu().numpy()[0][:, flat].T * np.array([np.prod(hh ** np.array(a)) for a in es])[None, :]
    Tg = T_eq.cpu().numpy()[0, 0][:, flat].T * np.array([np.prod(hh ** np.array(b)) for b in et])[None, :]
    bar = 1e-8 if prec == "fp64" else 1e-5
    es_err = max(rel_err(Sg[:, a], S[:, a]) for a in range(len(es)))
    et_err = max(rel_err(Tg[:, b], T[:, 0, b]) for b in range(len(et)))
    Sx, _ = orc.moments_compact(Xr, None, h, order, gp, name)
    method = max(rel_err(S[:, a], Sx[:, a]) for a in range(len(es)))
    print(f"{name} d={d} l={order} {prec}: S err {es_err:.2e} T err {et_err:.2e}; "
          f"binned vs exact sums {method:.2e} (h / delta = {h[0] / delta[0]:.1f})")
    assert es_err < bar and et_err < bar
    mref, _, _ = orc.solve(S, T, h, order, d)
    compare_fit(mh[flat], mref[:, 0], S, h, order, d, bar)


def test_compact_kernel_unsupported_calls():
    from paper_2204_07716_amd._lib import FKR_E_UNSUPPORTED, FkrError
    N = 500
    X = np.random.default_rng(4).random((N, 2))
    plan = make_plan(2, 1, (32, 32), (0.05, 0.05), (0.15, 0.15), 1e-6, "fp32", n_max=N, max_weights=16,
                     tprec="fp64", reg_kernel="epanechnikov")
    plan.set_points(to_dev(X, torch.float32))
    Y = to_dev(np.zeros((N, 1)), torch.float32)
    for call in (lambda: plan.interval((0.1, 0.1), 0.1), lambda: plan.gcv_grad((0.1, 0.1), Y, 2),
                 lambda: plan.fit_full(np.diag([0.01, 0.01]), Y)):
        with pytest.raises(FkrError) as e:
            call()
        assert e.value.status == FKR_E_UNSUPPORTED
