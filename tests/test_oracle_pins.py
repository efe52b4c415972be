"""Pins for the FP64 oracle against what the paper and the mathematics fix.

None of these tests re-types the oracle's own formula.  Each one checks it
against an independent fact:  Gaussian moment integrals (Poisson summation on
a dense lattice), weighted least squares by ``numpy.linalg.lstsq`` on the
explicit design matrix of eq. (3)-(5), polynomial reproduction, the OLS limit,
``numpy.fft`` on lattice samples, ``numpy.random.Philox``, exact smoother traces
and the Girard moments (Sec. 2.1), the printed ``get_hList`` values (Sec. 4.1),
and the closed-form invariants of the variance estimator (Sec. 3).
"""
import itertools
import json
import math
import os

import numpy as np
import pytest
from scipy import stats

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _gauss_moment(a: int, h: float) -> float:
    """E[Z^a] for Z ~ N(0, h^2): 0 for odd a, h^a (a-1)!! for even a."""
    if a % 2:
        return 0.0
    return h ** a * float(np.prod(np.arange(a - 1, 0, -2))) if a else 1.0


# ---------------------------------------------------------------------------
# eq. (9) moments
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("d,order", [(1, 0), (1, 2), (2, 1), (2, 2), (3, 1)])
def test_moments_match_gaussian_integrals_on_dense_lattice(orc, d, order):
    """A unit-weight lattice with spacing delta << h turns s_a(g) delta^d into
    the Gaussian moment integral, exactly up to exp(-2 pi^2 h^2/delta^2)."""
    h = np.array([0.11, 0.07, 0.09][:d])
    delta = h / 3.0
    g = np.array([0.013, -0.021, 0.004][:d])  # off-lattice evaluation point
    axes = [np.arange(-14 * 3, 14 * 3 + 1) * delta[j] for j in range(d)]
    mesh = np.meshgrid(*axes, indexing="ij")
    X = np.stack([m.ravel() for m in mesh], axis=1)
    S, _ = orc.moments(X, None, h, order, g[None, :], cutoff=False)
    exps = orc.multi_indices(d, 2 * order)
    vol = float(np.prod(delta))
    for m, a in enumerate(exps):
        expect = np.prod([_gauss_moment(a[j], h[j]) for j in range(d)])
        scale = np.prod([h[j] ** a[j] for j in range(d)])
        assert abs(S[0, m] * vol - expect) <= 1e-12 * scale, (a, S[0, m] * vol, expect)


def test_moments_sign_and_index_convention_single_sample(orc):
    """One sample: s_a / s_0 = (x - g)^a (z = x_i - g, eq. 2-4), with each
    exponent attached to its own dimension."""
    h = np.array([0.2, 0.3, 0.25])
    x = np.array([[0.31, 0.47, 0.52]])
    g = np.array([[0.25, 0.55, 0.50]])
    S, T = orc.moments(x, np.array([[2.5]]), h, 1, g, cutoff=False)
    z = (x - g)[0]
    for m, a in enumerate(orc.multi_indices(3, 2)):
        assert np.isclose(S[0, m] / S[0, 0], np.prod(z ** np.array(a)), rtol=1e-13, atol=0)
    for m, a in enumerate(orc.multi_indices(3, 1)):
        assert np.isclose(T[0, 0, m] / S[0, 0], 2.5 * np.prod(z ** np.array(a)), rtol=1e-13)
    assert S[0, 1] > 0 and S[0, 2] < 0  # x0 > g0, x1 < g1


def test_moment_cutoff_changes_nothing_at_fp64(orc):
    rng = np.random.default_rng(7)
    X = rng.random((300, 2))
    W = rng.standard_normal((300, 2))
    gp = orc.grid_points((9, 7), (0, 0), (1, 1))
    S1, T1 = orc.moments(X, W, [0.03, 0.05], 1, gp, cutoff=True)
    S2, T2 = orc.moments(X, W, [0.03, 0.05], 1, gp, cutoff=False)
    assert np.allclose(S1, S2, rtol=1e-14, atol=1e-300)
    assert np.allclose(T1, T2, rtol=1e-13, atol=1e-14 * np.abs(T2).max())


def test_kde_integrates_to_n(orc):
    """sum_g s_0(g) Delta^d -> N (eq. 8: the KDE integrates to one) when the
    grid is much finer than h and covers the kernel's support."""
    rng = np.random.default_rng(3)
    X = 0.35 + 0.3 * rng.random((50, 2))
    M = (161, 161)
    gp = orc.grid_points(M, (0, 0), (1, 1))
    S, _ = orc.moments(X, None, [0.03, 0.04], 0, gp)
    assert abs(S[:, 0].sum() * (1 / 160) ** 2 - 50) < 1e-9


# ---------------------------------------------------------------------------
# eq. (3) solve
# ---------------------------------------------------------------------------

def _wls_intercept(X, y, g, h, order):
    """m(g) of eq. (3) from the explicit design matrix D (eq. 4) and kernel
    weights (eq. 5), solved by lstsq on sqrt(W) D."""
    d = X.shape[1]
    exps = [a for a in itertools.product(range(order + 1), repeat=d) if sum(a) <= order]
    exps.sort(key=lambda a: (sum(a), [-v for v in a]))
    Z = X - g
    D = np.stack([np.prod(Z ** np.array(a), axis=1) for a in exps], axis=1)
    w = np.exp(-0.5 * ((Z / h) ** 2).sum(axis=1))
    sw = np.sqrt(w)
    coef, *_ = np.linalg.lstsq(sw[:, None] * D, sw * y, rcond=None)
    return coef[0]


@pytest.mark.parametrize("d,order", [(1, 0), (1, 1), (1, 2), (2, 1), (2, 2), (3, 1)])
def test_fit_equals_weighted_least_squares(orc, d, order):
    rng = np.random.default_rng(10 + d * 3 + order)
    N = 80
    X = rng.random((N, d))
    y = np.sin(3 * X).sum(axis=1) + 0.1 * rng.standard_normal(N)
    h = np.array([0.3, 0.25, 0.35][:d])
    gp = rng.random((6, d))
    mh = orc.fit(X, y, h, order, gp)[:, 0]
    ref = np.array([_wls_intercept(X, y, g, h, order) for g in gp])
    assert np.allclose(mh, ref, rtol=1e-9, atol=1e-11)


@pytest.mark.parametrize("d,order", [(1, 0), (1, 1), (1, 2), (2, 1), (2, 2), (3, 1), (3, 2)])
def test_polynomial_reproduction(orc, d, order):
    """A polynomial response of degree <= l is reproduced exactly."""
    rng = np.random.default_rng(100 + 7 * d + order)
    X = rng.random((120, d))
    coef = {a: rng.standard_normal() for a in orc.multi_indices(d, order)}

    def p(P):
        return sum(c * np.prod(P ** np.array(a), axis=1) for a, c in coef.items())

    gp = rng.random((10, d))
    mh = orc.fit(X, p(X), [0.2] * d, order, gp)[:, 0]
    assert np.allclose(mh, p(gp), rtol=1e-8, atol=1e-9)


def test_nw_of_constant_is_constant(orc):
    rng = np.random.default_rng(4)
    X = rng.random((200, 2))
    gp = orc.grid_points((5, 5), (0, 0), (1, 1))
    mh = orc.fit(X, np.ones(200), [0.05, 0.08], 0, gp)[:, 0]
    assert np.allclose(mh, 1.0, rtol=1e-14)


def test_local_linear_1d_closed_form(orc):
    """1-D local linear: m = (s2 t0 - s1 t1) / (s0 s2 - s1^2)."""
    rng = np.random.default_rng(5)
    X = rng.random((150, 1))
    y = np.cos(4 * X[:, 0]) + 0.2 * rng.standard_normal(150)
    gp = np.linspace(0, 1, 11)[:, None]
    mh, S, T, _, _ = orc.fit(X, y, [0.1], 1, gp, return_all=True)
    s0, s1, s2 = S[:, 0], S[:, 1], S[:, 2]
    t0, t1 = T[:, 0, 0], T[:, 0, 1]
    assert np.allclose(mh[:, 0], (s2 * t0 - s1 * t1) / (s0 * s2 - s1 ** 2), rtol=1e-10)


@pytest.mark.parametrize("d", [1, 2])
def test_large_bandwidth_tends_to_global_ols(orc, d):
    rng = np.random.default_rng(11 + d)
    X = rng.random((90, d))
    y = rng.standard_normal(90)
    D = np.concatenate([np.ones((90, 1)), X], axis=1)
    beta, *_ = np.linalg.lstsq(D, y, rcond=None)
    gp = rng.random((4, d))
    mh = orc.fit(X, y, [1e3] * d, 1, gp)[:, 0]
    assert np.allclose(mh, beta[0] + gp @ beta[1:], rtol=1e-5, atol=1e-6)


def test_complex_response_is_real_plus_imaginary(orc):
    rng = np.random.default_rng(6)
    X = rng.random((100, 2))
    yr, yi = rng.standard_normal(100), rng.standard_normal(100)
    gp = rng.random((5, 2))
    mc = orc.fit(X, yr + 1j * yi, [0.2, 0.2], 2, gp)[:, 0]
    assert np.allclose(mc.real, orc.fit(X, yr, [0.2, 0.2], 2, gp)[:, 0], rtol=1e-12)
    assert np.allclose(mc.imag, orc.fit(X, yi, [0.2, 0.2], 2, gp)[:, 0], rtol=1e-12)


def test_empty_region_is_ill_posed(orc):
    X = np.array([[0.1], [0.12], [0.15]])
    gp = np.array([[0.13], [0.9]])
    mh, S, T, r0, ill = orc.fit(X, np.ones(3), [0.005], 1, gp, return_all=True)
    assert not ill[0] and ill[1] and np.isnan(mh[1, 0])


# ---------------------------------------------------------------------------
# Type-1 NUDFT stage oracle (Sec. 1.2)
# ---------------------------------------------------------------------------

def test_nudft_on_lattice_equals_fft(orc):
    """Samples on a lattice of the period turn the NUDFT into numpy's FFT."""
    rng = np.random.default_rng(8)
    L0, L1 = 24, 20
    T = np.array([1.3, 1.1])
    m = np.stack([rng.integers(0, L0, 60), rng.integers(0, L1, 60)], axis=1)
    X = m * (T / np.array([L0, L1]))
    w = rng.standard_normal(60) + 1j * rng.standard_normal(60)
    grid = np.zeros((L1, L0), dtype=complex)
    np.add.at(grid, (m[:, 1], m[:, 0]), w)
    F = np.fft.fft2(grid)
    K = np.array([5, 4])
    c = orc.nudft(X, w, [0, 0], T, K)[..., 0]
    for n1 in range(-K[1], K[1] + 1):
        for n0 in range(-K[0], K[0] + 1):
            assert np.isclose(c[n1 + K[1], n0 + K[0]], F[n1 % L1, n0 % L0], rtol=1e-12, atol=1e-12)


# ---------------------------------------------------------------------------
# Interpolation
# ---------------------------------------------------------------------------

def test_interp_exact_on_multilinear_functions(orc):
    rng = np.random.default_rng(9)
    M, lo, hi = (7, 6, 5), (0, -1, 2), (1, 1, 3)
    c = rng.standard_normal(8)

    def f(P):
        x, y, z = P[:, 0], P[:, 1], P[:, 2]
        return (c[0] + c[1] * x + c[2] * y + c[3] * z + c[4] * x * y + c[5] * y * z
                + c[6] * x * z + c[7] * x * y * z)

    gp = orc.grid_points(M, lo, hi)
    Xq = np.stack([rng.uniform(lo[j], hi[j], 50) for j in range(3)], axis=1)
    Xq[0] = hi
    Xq[1] = lo
    assert np.allclose(orc.interp(f(gp), M, lo, hi, Xq), f(Xq), rtol=1e-12, atol=1e-12)
    assert np.allclose(orc.interp(f(gp), M, lo, hi, gp), f(gp), rtol=1e-13, atol=1e-13)


# ---------------------------------------------------------------------------
# Probes
# ---------------------------------------------------------------------------

def test_philox_known_answers(orc):
    """Philox4x32-10 against the generator's published known-answer vectors."""
    with open(os.path.join(GOLD, "philox4x32_10_kat.json")) as f:
        kat = json.load(f)
    for case in kat["cases"]:
        ctr = np.array([[int(v, 16) for v in case["ctr"]]], dtype=np.uint64)
        key = [int(v, 16) for v in case["key"]]
        got = orc.philox4x32(ctr, key)[0]
        assert [int(v) for v in got] == [int(v, 16) for v in case["out"]]


def test_philox_counter_and_key_layout(orc):
    """probes() feeds (i mod 2^32, i / 2^32, block, 0) and (seed mod 2^32,
    seed / 2^32): sample indices and seeds above 2^32 reach the high words."""
    i = np.array([5, 5 + 2**32], dtype=np.uint64)
    P = orc.probes(7, 0, 4, index=i)
    assert not np.array_equal(P[0], P[1])
    assert not np.array_equal(orc.probes(7, 3, 4), orc.probes(7 + 2**32, 3, 4))
    x = orc.philox4x32(np.array([[5, 0, 0, 0]], dtype=np.uint64), [7, 0])[0]
    u = ((x >> np.uint64(8)).astype(np.float64) + 0.5) * 2.0 ** -24
    assert np.isclose(P[0, 0], np.sqrt(-2 * np.log(u[0])) * np.cos(2 * np.pi * u[1]), rtol=1e-15)
    assert np.isclose(P[0, 3], np.sqrt(-2 * np.log(u[2])) * np.sin(2 * np.pi * u[3]), rtol=1e-15)


def test_probes_are_standard_normal_and_reproducible(orc):
    P = orc.probes(1234, 50_000, 6)
    assert P.shape == (50_000, 6)
    for p in range(6):
        assert stats.kstest(P[:, p], "norm").pvalue > 1e-4
    C = np.corrcoef(P.T)
    assert np.abs(C - np.eye(6)).max() < 0.03
    sub = orc.probes(1234, 0, 6, index=np.array([17, 49_999]))
    assert np.array_equal(sub, P[[17, 49_999]])
    assert not np.array_equal(orc.probes(1235, 10, 6), P[:10])


# ---------------------------------------------------------------------------
# DF (Sec. 2.1) and GCV (eq. 22)
# ---------------------------------------------------------------------------

def _smoother_matrix(orc, X, h, order, M, lo, hi):
    gp = orc.grid_points(M, lo, hi)
    N = X.shape[0]
    mh = orc.fit(X, np.eye(N), h, order, gp)
    return orc.interp(mh, M, lo, hi, X)  # column j = S e_j


def test_dof_identity_smoother_gives_zero(orc):
    """Samples on the grid nodes, tiny h: the smoother is the identity, so
    every Girard ratio is 0 and DF = N."""
    M = (33,)
    X = orc.grid_points(M, (0,), (1,))
    Wp = orc.probes(5, 33, 8)
    rho, m, df, inc = orc.dof(X, [1.0 / 32 / 20], 0, M, (0,), (1,), Wp)
    assert inc.all()
    assert np.all(np.abs(rho) < 1e-12) and abs(df - 33) < 1e-9


@pytest.mark.parametrize("d", [1, 2])
def test_dof_large_bandwidth_is_ols_projection(orc, d):
    """h -> infinity with l = 1: the smoother projects onto linear functions,
    so rho_p = ||(I - H) w_p||^2 / ||w_p||^2 with H the OLS hat matrix."""
    rng = np.random.default_rng(20 + d)
    N = 60
    X = rng.random((N, d))
    M, lo, hi = (9,) * d, (0,) * d, (1,) * d
    Wp = orc.probes(77, N, 5)
    rho, m, df, inc = orc.dof(X, [1e3] * d, 1, M, lo, hi, Wp)
    assert inc.all()
    D = np.concatenate([np.ones((N, 1)), X], axis=1)
    res = Wp - D @ np.linalg.lstsq(D, Wp, rcond=None)[0]
    assert np.allclose(rho, (res ** 2).sum(0) / (Wp ** 2).sum(0), rtol=1e-5)


def test_girard_estimator_mean_matches_exact_trace(orc):
    """E rho_p = tr(I - S)/N exactly for Gaussian probes, with
    Var rho_p = 2 (tr B^2 - (tr B)^2/N) / (N (N + 2)), B = sym(I - S)."""
    rng = np.random.default_rng(31)
    N, M = 40, (16,)
    X = rng.random((N, 1))
    S = _smoother_matrix(orc, X, [0.08], 1, M, (0,), (1,))
    B = np.eye(N) - S
    Bs = 0.5 * (B + B.T)
    exact = np.trace(B) / N
    var = 2 * (np.trace(Bs @ Bs) - np.trace(Bs) ** 2 / N) / (N * (N + 2))
    Np = 3000
    Wp = orc.probes(99, N, Np)
    rho, m, df, inc = orc.dof(X, [0.08], 1, M, (0,), (1,), Wp)
    assert inc.all()
    assert abs(m - exact) < 4 * math.sqrt(var / Np)
    assert abs(np.var(rho, ddof=1) / var - 1) < 0.15


def test_girard_estimator_over_a_subset_matches_restricted_trace(orc):
    """Over a sample subset I the ratio sum_I w (w - S w) / sum_I w^2 has
    mean tr(B_II) / N_I exactly (B = I - S; the probes off I enter linearly
    with zero mean), with the variance formula applied to sym(B_II)."""
    rng = np.random.default_rng(32)
    N, M = 40, (16,)
    X = rng.random((N, 1))
    S = _smoother_matrix(orc, X, [0.08], 1, M, (0,), (1,))
    inc = rng.random(N) < 0.6
    B = (np.eye(N) - S)[np.ix_(inc, inc)]
    Bs = 0.5 * (B + B.T)
    n = int(inc.sum())
    exact = np.trace(B) / n
    Np = 4000
    Wp = orc.probes(98, N, Np)
    # the variance of the subset ratio also carries the off-subset probe
    # terms; bound the mean with the full conditional variance by simulation
    rho, m, df, got = orc.dof(X, [0.08], 1, M, (0,), (1,), Wp, include=inc)
    assert np.array_equal(got, inc) and abs(df - n * (1 - m)) < 1e-9
    assert abs(m - exact) < 4 * np.std(rho, ddof=1) / math.sqrt(Np)
    assert np.std(rho, ddof=1) > math.sqrt(2 * (np.trace(Bs @ Bs) - np.trace(Bs) ** 2 / n) / (n * (n + 2))) * 0.8


def test_gcv_of_ols_fit(orc):
    """With the exact trace of the OLS hat matrix, eq. (22) is the classical
    GCV: (RSS/N) / (1 - P/N)^2."""
    rng = np.random.default_rng(40)
    N = 50
    X = rng.random((N, 1))
    y = 2 + 3 * X[:, 0] + rng.standard_normal(N)
    D = np.concatenate([np.ones((N, 1)), X], axis=1)
    beta, rss, *_ = np.linalg.lstsq(D, y, rcond=None)
    g = orc.gcv(y, D @ beta, 1 - 2 / N)
    assert np.isclose(g[0], rss[0] / N / (1 - 2 / N) ** 2, rtol=1e-12)


def test_rgcv_selection_rule(orc):
    g = [5.0, 3.0, 2.0, 2.05, 2.5, 4.0]
    assert orc.rgcv_select(g, 0.0) == 2
    assert orc.rgcv_select([3.0, 1.0, 1.0, 2.0], 0.0) == 2  # tie -> larger h
    sd = np.std(g, ddof=1)
    assert orc.rgcv_select(g, 0.5 / sd) == 4  # threshold 2.5 includes index 4
    assert orc.rgcv_select(g, 0.01 / sd) == 2


def test_get_hlist_printed_values():
    from oracle import oracle as orc
    with open(os.path.join(GOLD, "get_hlist_paper.json")) as f:
        gold = json.load(f)
    hl = orc.get_hlist(gold["n"], gold["range"], gold["kind"])[:, 0]
    for item in gold["printed"]:
        v = hl[item["position_1based"] - 1]
        assert float(f"{v:.{item['digits']}g}") == item["value"]
    assert hl[0] == 0.01 and np.isclose(hl[-1], 1.0)
    h2 = orc.get_hlist([3, 2], [[0.1, 0.3], [1, 2]], "lin")
    assert h2.shape == (6, 2) and np.allclose(h2[:3, 0], [0.1, 0.2, 0.3])


# ---------------------------------------------------------------------------
# Variance (Sec. 3)
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("order", [0, 1])
def test_variance_constant_residuals(orc, order):
    """|y - yhat|^2 = c everywhere: v = log(c + 1/N) exactly, kappa =
    (c + 1/N)/c, so sigma^2 = c on every grid point (eq. 24-26); the direct
    fit of eq. (23) also gives c."""
    rng = np.random.default_rng(50)
    N, c = 200, 0.37
    X = rng.random((N, 2))
    yhat = rng.standard_normal(N)
    y = yhat + np.sqrt(c) * np.where(rng.random(N) < 0.5, -1, 1)
    M = (6, 5)
    s2, ex = orc.variance(X, y, yhat, [0.2, 0.2], order, M, (0, 0), (1, 1))
    assert np.allclose(s2, c, rtol=1e-10)
    assert np.isclose(ex["kappa"], (c + 1 / N) / c, rtol=1e-12)
    s2d, _ = orc.variance(X, y, yhat, [0.2, 0.2], order, M, (0, 0), (1, 1), mode="direct")
    assert np.allclose(s2d, c, rtol=1e-10)


def test_variance_full_h_diagonal_equals_product_kernel(orc):
    """The second pass with a diagonal full bandwidth matrix equals the
    product-kernel pass at h = sqrt(diag H) (both modes)."""
    rng = np.random.default_rng(31)
    N = 400
    X = rng.random((N, 2))
    y = X[:, 0] + (0.2 + 0.5 * X[:, 1]) * rng.standard_normal(N)
    M, lo, hi = (9, 8), (0.0, 0.0), (1.0, 1.0)
    h = np.array([0.15, 0.2])
    yhat = orc.interp(orc.fit(X, y, h, 1, orc.grid_points(M, lo, hi))[:, 0], M, lo, hi, X)
    for mode in ("log", "direct"):
        a, _ = orc.variance(X, y, yhat, h, 1, M, lo, hi, mode=mode)
        b, _ = orc.variance(X, y, yhat, None, 1, M, lo, hi, mode=mode, H=np.diag(h ** 2))
        np.testing.assert_allclose(b, a, rtol=1e-10)


def test_variance_log_linear_reproduction(orc):
    """If log(r + 1/N) is linear in x, the local-linear v reproduces it."""
    rng = np.random.default_rng(51)
    N = 300
    X = rng.random((N, 1))
    v_true = -1.0 + 2.0 * X[:, 0]
    r = np.exp(v_true) - 1.0 / N
    yhat = np.zeros(N)
    y = np.sqrt(r)
    M = (11,)
    s2, ex = orc.variance(X, y, yhat, [0.15], 1, M, (0,), (1,))
    g = np.linspace(0, 1, 11)
    assert np.allclose(ex["v"], -1.0 + 2.0 * g, rtol=1e-9, atol=1e-9)
    kappa = 1.0 / np.mean(r * np.exp(-v_true))
    assert np.allclose(s2, np.exp(-1.0 + 2.0 * g) / kappa, rtol=1e-9)


def test_pivots_equal_squared_cholesky_diagonal(orc):
    """The minor-ratio pivots are the squares of the diagonal of numpy's
    Cholesky factor (a different algorithm for the same quantity)."""
    rng = np.random.default_rng(70)
    for P in (1, 3, 6, 10):
        B = rng.standard_normal((20, P, P))
        A = B @ np.transpose(B, (0, 2, 1)) + 0.1 * np.eye(P) * rng.random((20, 1, 1))
        A *= 10.0 ** rng.uniform(-3, 5, (20, 1, 1))
        L = np.linalg.cholesky(A)
        ref = np.diagonal(L, axis1=1, axis2=2) ** 2
        assert np.allclose(orc.pivots(A), ref, rtol=1e-8)


def test_collinear_design_is_ill_posed(orc):
    """Samples on the line x1 = 0.5: the local-linear system is singular at
    every grid point; a generic design is not."""
    rng = np.random.default_rng(71)
    X = np.stack([rng.random(300), np.full(300, 0.5)], axis=1)
    gp = rng.random((10, 2))
    mh, S, T, r0, ill = orc.fit(X, rng.standard_normal(300), [0.1, 0.1], 1, gp, return_all=True)
    assert ill.all() and np.isnan(mh).all()
    X2 = rng.random((300, 2))
    gp2 = 0.2 + 0.6 * rng.random((10, 2))
    mh, S, T, r0, ill = orc.fit(X2, rng.standard_normal(300), [0.1, 0.1], 1, gp2, return_all=True)
    assert not ill.any()


def test_relative_pivots_are_one_minus_r_squared(orc):
    """pivot_c / A_cc of the weighted Gram matrix of a design equals one minus
    the uncentred R^2 of column c regressed (weighted least squares, numpy
    lstsq) on the columns before it, and does not change under diagonal
    scaling of the columns (the bandwidth equilibration)."""
    rng = np.random.default_rng(73)
    for P in (2, 3, 6):
        D = rng.standard_normal((50, P))
        D[:, -1] = D[:, 0] * 0.9 + 0.1 * rng.standard_normal(50)   # a nearly collinear column
        wgt = rng.random(50)
        A = (D * wgt[:, None]).T @ D
        rp = orc.relative_pivots(A[None])[0]
        sq = np.sqrt(wgt)[:, None]
        assert abs(rp[0] - 1) < 1e-12
        for c in range(1, P):
            coef = np.linalg.lstsq(D[:, :c] * sq, D[:, c] * sq[:, 0], rcond=None)[0]
            res = (D[:, c] - D[:, :c] @ coef) * sq[:, 0]
            r2 = 1 - (res @ res) / ((D[:, c] * sq[:, 0]) @ (D[:, c] * sq[:, 0]))
            assert abs(rp[c] - (1 - r2)) < 1e-10
        sc = 10.0 ** rng.uniform(-3, 3, P)
        assert np.allclose(orc.relative_pivots((A * sc[:, None] * sc[None, :])[None])[0], rp, rtol=1e-9)


def test_resolved_points_follow_the_local_design(orc):
    """1-D local linear: the relative pivot is 1 - s_1^2 / (s_0 s_2) (closed
    form).  Samples piled on one point x = 0.26 between grid points leave the
    grid points near it unresolved (their local design is a single point),
    while a spread cloud resolves every point it covers."""
    rng = np.random.default_rng(74)
    X = np.concatenate([np.full(300, 0.26), 0.6 + 0.4 * rng.random(300)])[:, None]
    gp = np.linspace(0, 1, 41)[:, None]
    h = [0.04]
    S, _ = orc.moments(X, None, h, 1, gp)
    s0, s1, s2 = S[:, 0], S[:, 1], S[:, 2]
    closed = 1 - s1 ** 2 / (s0 * s2)
    A = orc.assemble(S, h, 1, 1)
    assert np.allclose(orc.relative_pivots(A)[:, 1], closed, rtol=1e-6, atol=1e-13)
    ok = orc.resolved(S, h, 1, 1)
    assert np.array_equal(ok, closed > orc.RESOLVE)
    assert not ok[10] and not ok[11] and ok[32]    # g = 0.25, 0.275 (the pile) and 0.8 (the cloud)


def test_supported_samples_by_brute_force(orc):
    """A sample is supported when every corner of its interpolation cell
    (floor clamped to [0, M - 2]) is in the resolved set: checked against
    explicit loops over samples and corners."""
    rng = np.random.default_rng(75)
    M, lo, hi = (7, 6), (0.0, -1.0), (1.0, 2.0)
    X = np.stack([rng.random(300), -1 + 3 * rng.random(300)], axis=1)
    X[:5] = [[1.0, 2.0], [0.0, -1.0], [1.0, -1.0], [0.5, 2.0], [0.0, 0.5]]
    ok = rng.random(M[0] * M[1]) < 0.8
    got = orc.supported(ok, M, lo, hi, X)
    for i in range(X.shape[0]):
        cell = []
        for j in range(2):
            dlt = (hi[j] - lo[j]) / (M[j] - 1)
            cell.append(min(max(int(math.floor((X[i, j] - lo[j]) / dlt)), 0), M[j] - 2))
        want = all(ok[(cell[0] + a) + M[0] * (cell[1] + b)] for a in (0, 1) for b in (0, 1))
        assert got[i] == want, i


def test_variance_skips_undefined_residuals(orc):
    """Residuals that are undefined (NaN mean fit) are left out: with the
    rest constant, sigma^2 is still that constant (eq. 24-26 invariant)."""
    rng = np.random.default_rng(76)
    N, M = 3000, (15, 14)
    X = rng.random((N, 2))
    c = 0.37
    yhat = rng.standard_normal(N)
    y = yhat + math.sqrt(c)
    yhat[:200] = np.nan
    s2, ex = orc.variance(X, y, yhat, [0.2, 0.2], 1, M, (0, 0), (1, 1))
    assert np.isnan(ex["r"][:200]).all()
    kappa = (c + 1.0 / N) / c
    assert abs(ex["kappa"] / kappa - 1) < 1e-9
    assert np.allclose(s2, c, rtol=1e-8)


def test_rgcv_select_skips_nan(orc):
    g = np.array([np.nan, 3.0, 1.0, 1.05, np.nan, 2.0])
    assert orc.rgcv_select(g, 0.0) == 2
    f = g[np.isfinite(g)]
    thr = f.min() + 0.1 * np.std(f, ddof=1)
    assert orc.rgcv_select(g, 0.1) == max(k for k in range(6) if np.isfinite(g[k]) and g[k] <= thr)


# ---------------------------------------------------------------------------
# Prediction (Sec. 4 fkreg_predict; Table 1 y_grid_opt: 'spline', extrapolation
# 'linear') and the variance of the fit with its interval (Sec. 4.2, eq. 27-28)
# ---------------------------------------------------------------------------

def test_spline_1d_matches_scipy_not_a_knot(orc):
    """Inside: SciPy's CubicSpline with not-a-knot ends.  Outside: the
    tangent line at the nearer end, from CubicSpline's own derivative."""
    from scipy.interpolate import CubicSpline
    rng = np.random.default_rng(5)
    for n in (4, 5, 6, 11, 40):
        f = rng.standard_normal(n)
        cs = CubicSpline(np.arange(n, dtype=float), f, bc_type="not-a-knot")
        for t in np.concatenate([rng.uniform(0, n - 1, 20), [0.0, n - 1.0, 1.0, n - 2.0]]):
            assert orc.spline_eval_1d(f, t) == pytest.approx(cs(t), abs=1e-13)
        for t in (-2.5, -0.01):
            assert orc.spline_eval_1d(f, t) == pytest.approx(cs(0.0) + t * cs(0.0, 1), abs=1e-12)
        for t in (n - 1 + 0.01, n + 3.0):
            assert orc.spline_eval_1d(f, t) == pytest.approx(cs(n - 1.0) + (t - n + 1) * cs(n - 1.0, 1),
                                                             abs=1e-12)


def test_spline_few_nodes_parabola_and_line(orc):
    """Three nodes: the interpolating parabola (np.polyfit, exact); two: the
    line through them, also beyond the ends."""
    f3 = np.array([0.3, -1.2, 2.0])
    par = np.polyfit([0.0, 1.0, 2.0], f3, 2)
    for t in (0.0, 0.4, 1.7, 2.0):
        assert orc.spline_eval_1d(f3, t) == pytest.approx(np.polyval(par, t), abs=1e-14)
    f2 = np.array([1.5, -0.5])
    for t in (-1.0, 0.25, 1.0, 3.0):
        assert orc.spline_eval_1d(f2, t) == pytest.approx(1.5 - 2.0 * t, abs=1e-14)


def test_spline_tensor_product_matches_scipy_grid_cubic(orc):
    """Interior points: SciPy's RegularGridInterpolator 'cubic' (tensor
    product of not-a-knot B-splines) with an exact sparse solve."""
    from scipy.interpolate import RegularGridInterpolator
    from scipy.sparse.linalg import spsolve
    rng = np.random.default_rng(6)
    for M, lo, hi in (([7, 9, 6], [0.0, -1.0, 2.0], [1.0, 1.0, 3.0]), ([5, 4], [0.0, 0.0], [1.0, 2.0])):
        d = len(M)
        G = rng.standard_normal(int(np.prod(M)))
        Xq = np.stack([rng.uniform(lo[j], hi[j], 40) for j in range(d)], 1)
        V = G.reshape(M[::-1]).transpose(tuple(range(d - 1, -1, -1)))   # axis j = dimension j
        ref = RegularGridInterpolator(orc.grid_axes(M, lo, hi), V, method="cubic", solver=spsolve)(Xq)
        np.testing.assert_allclose(orc.spline_predict(G, M, lo, hi, Xq)[0], ref, atol=1e-12)


def test_spline_reproduces_separable_cubics_and_extends_linearly(orc):
    """A product of cubics is its own tensor spline (grid values in, the
    function out, at any interior point); beyond the box in one dimension the
    value is the function at the face plus its normal derivative times the
    distance; beyond a corner, the product of the per-dimension tangent
    lines."""
    cub = [np.poly1d([0.5, -1.0, 0.3, 2.0]), np.poly1d([-0.2, 0.7, 1.1, -0.4]), np.poly1d([1.3, 0.0, -0.6, 0.9])]
    M, lo, hi = [6, 5, 7], [0.0, -1.0, 0.5], [2.0, 1.0, 1.5]
    ax = orc.grid_axes(M, lo, hi)
    G = np.einsum("k,j,i->kji", cub[2](ax[2]), cub[1](ax[1]), cub[0](ax[0])).ravel()
    rng = np.random.default_rng(7)
    Xq = np.stack([rng.uniform(lo[j], hi[j], 30) for j in range(3)], 1)
    exact = cub[0](Xq[:, 0]) * cub[1](Xq[:, 1]) * cub[2](Xq[:, 2])
    np.testing.assert_allclose(orc.spline_predict(G, M, lo, hi, Xq)[0], exact, rtol=1e-11, atol=1e-11)

    def ext(p, x, a, b):
        if x < a:
            return p(a) + (x - a) * p.deriv()(a)
        if x > b:
            return p(b) + (x - b) * p.deriv()(b)
        return p(x)

    for x in ([-0.7, 0.2, 1.0], [1.0, 1.6, 0.9], [2.5, -1.4, 1.7]):
        want = np.prod([ext(cub[j], x[j], lo[j], hi[j]) for j in range(3)])
        got = orc.spline_predict(G, M, lo, hi, np.array([x]))[0, 0]
        assert got == pytest.approx(want, rel=1e-11, abs=1e-11)


def test_fit_variance_equals_explicit_smoother_rows(orc):
    """Sigma(g) = sum_i S_gi^2 sigma_i^2 with the rows S_g. of the smoother
    built column by column: the fit of each unit response e_i (eq. 3)."""
    rng = np.random.default_rng(8)
    for d, order, h in ((1, 0, [0.08]), (1, 2, [0.12]), (2, 1, [0.15, 0.2]), (3, 1, [0.25, 0.3, 0.2])):
        N = 150
        X = rng.uniform(0, 1, (N, d))
        M = [6, 5, 4][:d]
        gp = orc.grid_points(M, [0.0] * d, [1.0] * d)
        s2 = 0.1 + X[:, 0] ** 2
        rows = orc.fit(X, np.eye(N), h, order, gp)
        np.testing.assert_allclose(orc.fit_variance(X, s2, h, order, gp), (rows ** 2 * s2).sum(1), rtol=1e-10)


def test_fit_variance_full_h_equals_explicit_smoother_rows(orc):
    """With a full bandwidth matrix: Sigma from the smoother rows of the
    full-H fits of the unit responses, and a diagonal H gives the product
    kernel's Sigma at h = sqrt(diag H)."""
    rng = np.random.default_rng(30)
    N = 140
    X = rng.uniform(0, 1, (N, 2))
    gp = orc.grid_points([5, 4], [0.0, 0.0], [1.0, 1.0])
    s2 = 0.1 + X[:, 0] ** 2
    H = np.array([[0.03, 0.012], [0.012, 0.045]])
    rows, _, ill = orc.fit_full(X, np.eye(N), H, 1, gp)
    got = orc.fit_variance(X, s2, None, 1, gp, H=H)
    np.testing.assert_allclose(got[~ill], (rows ** 2 * s2).sum(1)[~ill], rtol=1e-10)
    h = np.array([0.17, 0.21])
    np.testing.assert_allclose(orc.fit_variance(X, s2, None, 1, gp, H=np.diag(h ** 2)),
                               orc.fit_variance(X, s2, h, 1, gp), rtol=1e-10)


def test_fit_variance_is_the_variance_of_the_fit(orc):
    """eq. (27): Sigma is var[m_hat(g)].  Simulated responses y = m + sigma eps
    (8000 replicas): the sample variance of the fits agrees within five
    standard errors, sqrt(2 / R) relative."""
    rng = np.random.default_rng(9)
    N, R = 200, 8000
    X = rng.uniform(0, 1, (N, 2))
    h, order = [0.15, 0.2], 1
    gp = orc.grid_points([5, 4], [0.0, 0.0], [1.0, 1.0])
    s2 = 0.1 + X[:, 0] ** 2
    Y = np.sin(3 * X[:, 0])[:, None] + np.sqrt(s2)[:, None] * rng.standard_normal((N, R))
    emp = orc.fit(X, Y, h, order, gp).var(axis=1, ddof=1)
    np.testing.assert_allclose(emp, orc.fit_variance(X, s2, h, order, gp), rtol=5 * np.sqrt(2.0 / R))


def test_fit_variance_nadaraya_watson_constant_noise(orc):
    """l = 0, constant sigma^2: Sigma = sigma^2 sum K^2 / (sum K)^2, the
    variance of a weighted mean (direct sums here)."""
    rng = np.random.default_rng(10)
    X = rng.uniform(0, 1, (120, 1))
    g = np.array([[0.0], [0.37], [1.0]])
    h = 0.07
    K = np.exp(-0.5 * ((X[:, 0][None, :] - g) / h) ** 2)
    want = 0.3 * (K ** 2).sum(1) / K.sum(1) ** 2
    np.testing.assert_allclose(orc.fit_variance(X, 0.3, [h], 0, g), want, rtol=1e-12)


def test_interval_quantile(orc):
    """z_{0.975} = 1.959963984540054 (the two-sided 95% point); the band is
    symmetric about m_hat with half-width z sqrt(Sigma)."""
    assert orc.normal_quantile(0.975) == pytest.approx(1.959963984540054, rel=1e-15)
    assert orc.normal_quantile(0.5) == 0.0
    lo, hi = orc.interval(np.array([1.0, -2.0]), np.array([4.0, 0.25]), alpha=0.05)
    np.testing.assert_allclose(hi - lo, 2 * 1.959963984540054 * np.array([2.0, 0.5]), rtol=1e-15)
    np.testing.assert_allclose((hi + lo) / 2, [1.0, -2.0], rtol=1e-15)


# ---------------------------------------------------------------------------
# The GCV criterion as a function of log h and its gradient (eq. 22, Sec. 2.1)
# ---------------------------------------------------------------------------

def test_gcv_gradient_step_independent_and_vanishes_in_ols_limit(orc):
    """The central-difference gradient agrees for two steps (an O(step^2)
    scheme: a dropped or mis-scaled term would not); at bandwidths far above
    the data span the local fit is the global OLS fit, independent of h, so
    the gradient vanishes."""
    rng = np.random.default_rng(12)
    N = 400
    X = rng.random((N, 2))
    y = np.sin(3 * X[:, 0]) + X[:, 1] + 0.3 * rng.standard_normal(N)
    Wp = rng.standard_normal((N, 4))
    M, lo, hi = (12, 10), (0.0, 0.0), (1.0, 1.0)
    h = np.array([0.15, 0.2])
    g1 = orc.gcv_log_h_gradient(X, y, h, 1, M, lo, hi, Wp, step=1e-3)
    g2 = orc.gcv_log_h_gradient(X, y, h, 1, M, lo, hi, Wp, step=5e-4)
    np.testing.assert_allclose(g1, g2, rtol=2e-5)
    # the approach to the OLS limit is O((span / h)^2): the gradient falls
    # about a hundredfold from h = 300 to h = 3000
    g300 = orc.gcv_log_h_gradient(X, y, np.array([300.0, 300.0]), 1, M, lo, hi, Wp, step=1e-3)
    g3000 = orc.gcv_log_h_gradient(X, y, np.array([3000.0, 3000.0]), 1, M, lo, hi, Wp, step=1e-3)
    G = orc.gcv_criterion(X, y, np.array([3000.0, 3000.0]), 1, M, lo, hi, Wp)
    assert np.abs(g3000).max() < 1e-7 * G
    assert 50 < abs(g300[0] / g3000[0]) < 200


def test_gcv_gradient_symmetric_design(orc):
    """A design and response symmetric under swapping the two coordinates
    (each sample also present with x_1 and x_2 exchanged) has equal partial
    derivatives at equal bandwidths."""
    rng = np.random.default_rng(13)
    X0 = rng.random((150, 2))
    X = np.concatenate([X0, X0[:, ::-1]])
    y = np.cos(2 * X[:, 0]) + np.cos(2 * X[:, 1])
    y = y + 0.2 * np.concatenate([e := rng.standard_normal(150), e])
    Wp0 = rng.standard_normal((150, 3))
    Wp = np.concatenate([Wp0, Wp0])
    g = orc.gcv_log_h_gradient(X, y, np.array([0.2, 0.2]), 1, (9, 9), (0.0, 0.0), (1.0, 1.0), Wp)
    assert g[0] == pytest.approx(g[1], rel=1e-8)


def test_gcv_y_gradient_matches_central_differences(orc):
    """GCV is quadratic in y (the smoother and the Girard ratios do not
    depend on y), so central differences in y_i are exact up to rounding;
    some samples are unsupported (a sparse corner of the box)."""
    rng = np.random.default_rng(14)
    N = 160
    X = rng.random((N, 2)) ** 1.5
    y = np.sin(4 * X[:, 0]) * np.cos(2 * X[:, 1]) + 0.2 * rng.standard_normal(N)
    Wp = rng.standard_normal((N, 3))
    M, lo, hi, h = (9, 8), (0.0, 0.0), (1.0, 1.0), np.array([0.12, 0.14])
    inc = orc.support(X, h, 1, M, lo, hi)[0]
    g = orc.gcv_y_gradient(X, y, h, 1, M, lo, hi, Wp, include=inc)
    for i in list(range(0, N, 23)) + [int(np.nonzero(~inc)[0][0])] if (~inc).any() else list(range(0, N, 23)):
        e = np.zeros(N)
        e[i] = 0.05
        fd = (orc.gcv_criterion(X, y + e, h, 1, M, lo, hi, Wp, inc)
              - orc.gcv_criterion(X, y - e, h, 1, M, lo, hi, Wp, inc)) / 0.1
        assert g[i] == pytest.approx(fd, rel=1e-7, abs=1e-12)


def test_gcv_gradients_binned_compact_kernel(orc):
    """Under the binned approximation of a compact kernel the GCV is still
    quadratic in y: the y gradient (explicit smoother of the binned fits)
    matches central differences; in log h, away from the bandwidths where a
    grid offset enters the support, the central-difference gradient does not
    depend on the step."""
    rng = np.random.default_rng(15)
    N = 150
    X = rng.random((N, 2))
    y = np.sin(4 * X[:, 0]) * np.cos(2 * X[:, 1]) + 0.2 * rng.standard_normal(N)
    Wp = rng.standard_normal((N, 3))
    M, lo, hi = (9, 8), (0.0, 0.0), (1.0, 1.0)
    delta = [1.0 / 8, 1.0 / 7]
    h = np.array([2.5 / 8, 2.5 / 7])
    binned = ("epanechnikov", delta, [24, 22])
    inc = orc.support(X, h, 1, M, lo, hi, binned=binned)[0]
    g = orc.gcv_y_gradient(X, y, h, 1, M, lo, hi, Wp, include=inc, binned=binned)
    for i in range(0, N, 19):
        e = np.zeros(N)
        e[i] = 0.05
        fd = (orc.gcv_criterion(X, y + e, h, 1, M, lo, hi, Wp, inc, binned=binned)
              - orc.gcv_criterion(X, y - e, h, 1, M, lo, hi, Wp, inc, binned=binned)) / 0.1
        assert g[i] == pytest.approx(fd, rel=1e-7, abs=1e-12)
    g1 = orc.gcv_log_h_gradient(X, y, h, 1, M, lo, hi, Wp, include=inc, step=1e-3, binned=binned)
    g2 = orc.gcv_log_h_gradient(X, y, h, 1, M, lo, hi, Wp, include=inc, step=5e-4, binned=binned)
    np.testing.assert_allclose(g1, g2, rtol=2e-5, atol=2e-5 * np.abs(g1).max())


def test_gcv_binned_box_is_flat_between_jumps(orc):
    """The binned box kernel weighs the grid offsets |m delta| <= h equally,
    and a local polynomial fit does not change when all its weights scale
    together or when its monomials are rescaled (the equilibration), so the
    GCV does not depend on h until an offset crosses the support's edge,
    where it jumps."""
    rng = np.random.default_rng(19)
    N = 150
    X = rng.random((N, 2))
    y = np.sin(4 * X[:, 0]) * np.cos(2 * X[:, 1]) + 0.2 * rng.standard_normal(N)
    Wp = rng.standard_normal((N, 3))
    M, lo, hi = (9, 8), (0.0, 0.0), (1.0, 1.0)
    delta = [1.0 / 8, 1.0 / 7]
    binned = ("box", delta, [24, 22])
    h = np.array([2.3 / 8, 2.4 / 7])
    inc = orc.support(X, h, 1, M, lo, hi, binned=binned)[0]
    g0 = orc.gcv_criterion(X, y, h, 1, M, lo, hi, Wp, inc, binned=binned)
    g1 = orc.gcv_criterion(X, y, h * 1.2, 1, M, lo, hi, Wp, inc, binned=binned)      # offsets 2 delta still inside
    g2 = orc.gcv_criterion(X, y, h * 1.35, 1, M, lo, hi, Wp, inc, binned=binned)     # 3 delta enters
    assert g1 == pytest.approx(g0, rel=1e-12)
    assert abs(g2 / g0 - 1) > 1e-4
    gl = orc.gcv_log_h_gradient(X, y, h, 1, M, lo, hi, Wp, include=inc, step=1e-3, binned=binned)
    assert np.abs(gl).max() <= 1e-9 * g0


def test_gcv_full_h_diagonal_reduces_to_product_kernel(orc):
    """A diagonal bandwidth matrix H = diag(h^2) gives the product-kernel
    GCV at h (the full-H moments by NumPy sums, the diagonal ones by the C
    sums), and a rotated H changes it."""
    rng = np.random.default_rng(16)
    N = 300
    X = rng.random((N, 2))
    y = np.sin(3 * X[:, 0]) + X[:, 1] ** 2 + 0.2 * rng.standard_normal(N)
    Wp = rng.standard_normal((N, 3))
    M, lo, hi = (10, 9), (0.0, 0.0), (1.0, 1.0)
    h = np.array([0.14, 0.17])
    g_diag = orc.gcv_criterion(X, y, h, 1, M, lo, hi, Wp)
    g_full = orc.gcv_criterion(X, y, None, 1, M, lo, hi, Wp, H=np.diag(h ** 2))
    assert g_full == pytest.approx(g_diag, rel=1e-10)
    g_rot = orc.gcv_criterion(X, y, None, 1, M, lo, hi, Wp, H=np.array([[0.02, 0.012], [0.012, 0.03]]))
    assert abs(g_rot / g_diag - 1) > 1e-4


def test_gcv_H_gradient_diagonal_matches_log_h_gradient(orc):
    """At a diagonal H = diag(h^2) the gradient in the diagonal entries is the
    log-h gradient over 2 H_jj (h_j = sqrt(H_jj)), by two different
    central-difference paths; the off-diagonal derivative does not vanish
    for a correlated response."""
    rng = np.random.default_rng(17)
    N = 300
    X = rng.random((N, 2))
    y = np.sin(3 * (X[:, 0] + X[:, 1])) + 0.2 * rng.standard_normal(N)
    Wp = rng.standard_normal((N, 3))
    M, lo, hi = (10, 9), (0.0, 0.0), (1.0, 1.0)
    h = np.array([0.15, 0.18])
    inc = orc.support(X, h, 1, M, lo, hi)[0]
    gH = orc.gcv_H_gradient(X, y, np.diag(h ** 2), 1, M, lo, hi, Wp, include=inc)
    gl = orc.gcv_log_h_gradient(X, y, h, 1, M, lo, hi, Wp, include=inc)
    np.testing.assert_allclose([gH[0] * 2 * h[0] ** 2, gH[2] * 2 * h[1] ** 2], gl, rtol=1e-5)
    assert abs(gH[1]) > 1e-3 * np.abs(gH).max()


def test_gcv_y_gradient_full_h(orc):
    """With a full bandwidth matrix GCV is still quadratic in y: the y
    gradient from the explicit smoother matches central differences; at a
    diagonal H = diag(h^2) it is the product kernel's y gradient at h."""
    rng = np.random.default_rng(18)
    N = 150
    X = rng.random((N, 2))
    y = np.sin(3 * (X[:, 0] + 0.5 * X[:, 1])) + 0.2 * rng.standard_normal(N)
    Wp = rng.standard_normal((N, 3))
    M, lo, hi = (9, 8), (0.0, 0.0), (1.0, 1.0)
    H = np.array([[0.03, 0.012], [0.012, 0.04]])
    inc = orc.support(X, None, 1, M, lo, hi, H=H)[0]
    g = orc.gcv_y_gradient(X, y, None, 1, M, lo, hi, Wp, include=inc, H=H)
    for i in range(0, N, 17):
        e = np.zeros(N)
        e[i] = 0.05
        fd = (orc.gcv_criterion(X, y + e, None, 1, M, lo, hi, Wp, inc, H=H)
              - orc.gcv_criterion(X, y - e, None, 1, M, lo, hi, Wp, inc, H=H)) / 0.1
        assert g[i] == pytest.approx(fd, rel=1e-7, abs=1e-12)
    h = np.array([0.16, 0.19])
    inc_d = orc.support(X, h, 1, M, lo, hi)[0]
    gd = orc.gcv_y_gradient(X, y, None, 1, M, lo, hi, Wp, include=inc_d, H=np.diag(h ** 2))
    gh = orc.gcv_y_gradient(X, y, h, 1, M, lo, hi, Wp, include=inc_d)
    np.testing.assert_allclose(gd, gh, rtol=1e-9, atol=1e-12 * np.abs(gh).max())


def test_gcv_gradients_complex_response(orc):
    """Complex y: GCV uses |y - yhat|^2; the gradient d/dRe y + i d/dIm y
    matches central differences along the real and the imaginary axis, and
    the log-h gradient is the sum of the two parts' contributions (the GCV
    of a complex response is that of its real part plus that of its
    imaginary part in the numerator)."""
    rng = np.random.default_rng(15)
    N = 150
    X = rng.random((N, 2))
    y = np.exp(2j * X[:, 0]) * X[:, 1] + 0.2 * (rng.standard_normal(N) + 1j * rng.standard_normal(N))
    Wp = rng.standard_normal((N, 3))
    M, lo, hi, h = (8, 8), (0.0, 0.0), (1.0, 1.0), np.array([0.15, 0.15])
    inc = orc.support(X, h, 1, M, lo, hi)[0]
    g = orc.gcv_y_gradient(X, y, h, 1, M, lo, hi, Wp, include=inc)
    for i in (3, 77, 140):
        for unit, part in ((1.0, g[i].real), (1j, g[i].imag)):
            e = np.zeros(N, dtype=complex)
            e[i] = 0.05 * unit
            fd = (orc.gcv_criterion(X, y + e, h, 1, M, lo, hi, Wp, inc)
                  - orc.gcv_criterion(X, y - e, h, 1, M, lo, hi, Wp, inc)) / 0.1
            assert part == pytest.approx(fd, rel=1e-7, abs=1e-12)
    G = orc.gcv_criterion(X, y, h, 1, M, lo, hi, Wp, inc)
    Gr = orc.gcv_criterion(X, y.real, h, 1, M, lo, hi, Wp, inc)
    Gi = orc.gcv_criterion(X, y.imag, h, 1, M, lo, hi, Wp, inc)
    assert G == pytest.approx(Gr + Gi, rel=1e-12)
    np.testing.assert_allclose(orc.gcv_log_h_gradient(X, y, h, 1, M, lo, hi, Wp, inc),
                               orc.gcv_log_h_gradient(X, y.real, h, 1, M, lo, hi, Wp, inc)
                               + orc.gcv_log_h_gradient(X, y.imag, h, 1, M, lo, hi, Wp, inc), rtol=1e-9)


# ---------------------------------------------------------------------------
# Full bandwidth matrix (eq. 2 with a general H)
# ---------------------------------------------------------------------------

def test_moments_full_diagonal_equals_product_kernel(orc):
    """A diagonal H = diag(h^2) is the product Gaussian of the C oracle."""
    rng = np.random.default_rng(16)
    X = rng.random((300, 3))
    W = rng.standard_normal((300, 2))
    h = np.array([0.11, 0.15, 0.09])
    g = rng.random((7, 3))
    S1, T1 = orc.moments_full(X, W, np.diag(h ** 2), 2, g)
    S2, T2 = orc.moments(X, W, h, 2, g)
    np.testing.assert_allclose(S1, S2, rtol=1e-11, atol=1e-13 * np.abs(S2).max())
    np.testing.assert_allclose(T1, T2, rtol=1e-11, atol=1e-13 * np.abs(T2).max())


def test_moments_full_lattice_integrals(orc):
    """On a dense unit-weight lattice s_a(g) Delta^d is the Gaussian moment
    E[Z^a] for Z ~ N(0, H): 1, 0 for odd orders, H for the second moments,
    and Isserlis' H_jj H_kk + 2 H_jk^2 for E[Z_j^2 Z_k^2]."""
    H = np.array([[0.010, 0.006], [0.006, 0.016]])
    delta = 0.012
    ax = np.arange(-1.2, 1.2 + 1e-12, delta)
    X = np.stack(np.meshgrid(ax, ax, indexing="ij"), -1).reshape(-1, 2)
    S, _ = orc.moments_full(X, None, H, 2, np.array([[0.003, -0.002]]))
    S = S[0] * delta ** 2
    es = orc.multi_indices(2, 4)
    want = {(0, 0): 1.0, (2, 0): H[0, 0], (1, 1): H[0, 1], (0, 2): H[1, 1],
            (2, 2): H[0, 0] * H[1, 1] + 2 * H[0, 1] ** 2, (4, 0): 3 * H[0, 0] ** 2,
            (3, 1): 3 * H[0, 0] * H[0, 1], (1, 3): 3 * H[1, 1] * H[0, 1], (0, 4): 3 * H[1, 1] ** 2,
            (1, 0): 0.0, (0, 1): 0.0, (3, 0): 0.0, (2, 1): 0.0, (1, 2): 0.0, (0, 3): 0.0}
    for a, e in enumerate(es):
        assert S[a] == pytest.approx(want[tuple(e)], abs=1e-9)


def test_fit_full_rotation_invariant(orc):
    """Rotating the samples, the evaluation point and H together (H -> R H
    R^T) leaves the local-linear fit unchanged."""
    rng = np.random.default_rng(17)
    X = rng.random((400, 2))
    y = np.sin(3 * X[:, 0]) + X[:, 1] ** 2 + 0.1 * rng.standard_normal(400)
    H = np.array([[0.02, -0.008], [-0.008, 0.012]])
    th = 0.7
    R = np.array([[np.cos(th), -np.sin(th)], [np.sin(th), np.cos(th)]])
    g = np.array([[0.4, 0.55], [0.2, 0.8]])
    m1 = orc.fit_full(X, y, H, 1, g)[0]
    m2 = orc.fit_full(X @ R.T, y, R @ H @ R.T, 1, g @ R.T)[0]
    np.testing.assert_allclose(m1, m2, rtol=1e-10)


# ---------------------------------------------------------------------------
# Compact kernels (Table 1 kernel_type) and the binned approximation (eq. 11-13)
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("name", ["box", "triangle", "epanechnikov", "biweight", "triweight"])
def test_compact_kernels_are_densities(orc, name):
    """Each kernel integrates to one, is symmetric and vanishes beyond |u| = 1
    (midpoint rule on a fine lattice)."""
    u = np.arange(-120000, 120001) * 1e-5                        # exactly symmetric lattice
    k = orc.compact_kernel(name, u)
    assert np.sum(k) * 1e-5 == pytest.approx(1.0, abs=2e-5)
    np.testing.assert_array_equal(k, k[::-1])
    assert (k[np.abs(u) > 1] == 0).all()


@pytest.mark.parametrize("name", ["box", "epanechnikov", "triweight"])
def test_binned_moments_exact_for_samples_on_grid_nodes(orc, name):
    """The trigonometric interpolant of the sampled kernel passes through its
    samples, so for samples on grid nodes the binned moments equal the exact
    sums (2-D, up to degree 4)."""
    rng = np.random.default_rng(18)
    delta = np.array([0.02, 0.025])
    L = np.array([90, 72])
    k = np.stack([rng.integers(10, 40, 300), rng.integers(8, 30, 300)], axis=1)
    X = k * delta
    W = rng.standard_normal((300, 1))
    g = np.array([[0.4, 0.3], [0.5, 0.45]])                       # grid nodes too
    h = np.array([0.13, 0.11])
    S1, T1 = orc.moments_binned(X, W, h, 2, g, name, delta, L)
    S2, T2 = orc.moments_compact(X, W, h, 2, g, name)
    np.testing.assert_allclose(S1, S2, rtol=1e-9, atol=1e-11 * np.abs(S2).max())
    np.testing.assert_allclose(T1, T2, rtol=1e-9, atol=1e-11 * np.abs(T2).max())


@pytest.mark.parametrize("name", ["box", "triangle", "epanechnikov", "triweight"])
def test_fit_variance_compact_equals_explicit_smoother_rows(orc, name):
    """For a compact kernel Sigma(g) = sum_i S_gi^2 sigma_i^2 with the rows
    of the smoother built from the fits of the unit responses e_i (exact
    kernel sums), and for l = 0 it is the variance of the weighted mean,
    sigma^2 sum K^2 / (sum K)^2."""
    rng = np.random.default_rng(28)
    N = 140
    X = rng.uniform(0, 1, (N, 2))
    h = [0.3, 0.35]
    gp = orc.grid_points([4, 3], [0.0, 0.0], [1.0, 1.0])
    s2 = 0.1 + X[:, 0] ** 2
    for order in (0, 1):
        S, T = orc.moments_compact(X, np.eye(N), h, order, gp, name)
        rows, _, ill = orc.solve(S, T, h, order, 2)
        want = (rows ** 2 * s2).sum(1)
        got = orc.fit_variance(X, s2, h, order, gp, kernel=name)
        np.testing.assert_allclose(got[~ill], want[~ill], rtol=1e-10)
    K = np.prod(orc.compact_kernel(name, (X[None, :, :] - gp[:, None, :]) / np.array(h)), axis=2)
    wm = 0.3 * (K ** 2).sum(1) / K.sum(1) ** 2
    got0 = orc.fit_variance(X, 0.3, h, 0, gp, kernel=name)
    ok = K.sum(1) > 0
    np.testing.assert_allclose(got0[ok], wm[ok], rtol=1e-12)


@pytest.mark.parametrize("name", ["box", "epanechnikov", "triweight"])
def test_fit_variance_binned_exact_for_samples_on_grid_nodes(orc, name):
    """Samples on grid nodes: the binned moments of K and of K^2 are the exact
    sums, so r^T Q r from them equals the variance of the fit from its
    definition (2-D, local linear, per-sample sigma^2)."""
    rng = np.random.default_rng(29)
    delta = np.array([0.02, 0.025])
    L = np.array([90, 72])
    k = np.stack([rng.integers(10, 40, 400), rng.integers(8, 30, 400)], axis=1)
    X = k * delta
    s2 = 0.05 + rng.random(400)
    g = np.array([[0.4, 0.3], [0.5, 0.45], [0.3, 0.5]])
    h = np.array([0.13, 0.11])
    got = orc.fit_variance_binned(X, s2, h, 1, g, name, delta, L)
    want = orc.fit_variance(X, s2, h, 1, g, kernel=name)
    assert np.isfinite(want).all()
    np.testing.assert_allclose(got, want, rtol=1e-9)


def test_binned_moments_converge_with_kernel_smoothness(orc):
    """Off the nodes the binned sums approach the exact ones as the grid
    refines, faster for smoother kernels: halving delta / h cuts the error
    of the triweight (two continuous derivatives) more than that of the box
    (discontinuous)."""
    rng = np.random.default_rng(19)
    X = rng.random((400, 1)) * 0.6 + 0.2
    g = np.array([[0.5]])
    h = np.array([0.1])

    def err(name, delta):
        L = int(round(1.5 / delta))
        S1, _ = orc.moments_binned(X, None, h, 0, g, name, [delta], [L])
        S2, _ = orc.moments_compact(X, None, h, 0, g, name)
        return abs(S1[0, 0] - S2[0, 0]) / S2[0, 0]

    rb = err("box", 0.01) / err("box", 0.005)
    rt = err("triweight", 0.01) / err("triweight", 0.005)
    assert err("triweight", 0.005) < 1e-3
    assert rt > rb
