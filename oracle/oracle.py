"""FP64 CPU oracle for fast multivariate kernel regression -- TEST INFRASTRUCTURE.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this module.  It shares no code with the HIP path and
never imports the product package.  It computes what the paper's method
computes, by the plain definitions, slowly and in FP64:

* ``grid_points``   the uniform grid of eq. (6), spacing (hi - lo)/(M - 1).
* ``moments``       the kernel-weighted moment sums of eq. (9) by direct
                    O(N * G) summation (C library ``fkr_oracle.c``).
* ``solve``         the local-polynomial normal equations of eq. (3)/(11):
                    A_bc = s_{b+c}, rhs_b = t_b, equilibrated by the bandwidth
                    and solved by LAPACK's pivoted LU (``numpy.linalg.solve``);
                    the fit is the intercept (e_1 of eq. 3).
* ``moments_compact`` exact moment sums for the compact kernels of Table 1,
                    ``moments_binned`` their binned approximation of eq. (11)-(13)
                    (sampled kernel, discrete transform over the whole period).
* ``moments_full``  the moment sums of eq. (9) for a Gaussian kernel with a full
                    bandwidth matrix H (eq. 2), and ``fit_full`` the fit.
* ``interp``        multilinear interpolation of a grid function (the linear
                    ``griddedInterpolant`` setting of Sec. 5).
* ``philox4x32``    the Philox4x32-10 counter-based generator (Salmon et al.,
                    SC'11) behind ``probes``, the Gaussian probe vectors.
* ``dof``           Girard's fast Monte-Carlo estimate of (1/N) tr(I - S_h),
                    Sec. 2.1 steps i-iii.
* ``gcv``           the GCV criterion of eq. (22); ``rgcv_select`` the relaxed
                    selection rule of Table 1 (``dstd``); ``gcv_criterion`` GCV
                    as a function of h and ``gcv_log_h_gradient`` its gradient
                    in log h by central differences; ``gcv_y_gradient`` its
                    gradient in y from the explicit smoother.
* ``variance``      the conditional-variance second pass of Sec. 3: the
                    log-residual fit of eq. (24)-(26) (default) or the direct
                    residual fit of eq. (23).
* ``get_hlist``     the bandwidth list helper of Sec. 4.
* ``spline_predict`` tensor-product not-a-knot cubic spline interpolation of a
                    grid function with linear extrapolation (Sec. 4
                    fkreg_predict; Table 1 y_grid_opt), one dimension at a
                    time from the dense spline system.
* ``fit_variance``  the variance of the fit, Sigma(g) = sum_i S_gi^2 sigma_i^2
                    (eq. 27), from the smoother weights of eq. (3); with
                    ``interval`` the confidence band of eq. (28).

Readings taken where the paper is silent or garbled: the bandwidth ``h_j`` is the per-dimension kernel standard
deviation (H = diag(h^2)); the kernel is the normalised Gaussian; the
displacement is z = x_i - g; the design row holds every monomial of total
degree <= l in graded order; the Girard estimate is the mean over probes of
per-probe ratios; a grid point is ill-posed (NaN) when some pivot of the
equilibrated moment matrix (s_0 is the first) is at most 1e-12 times its
diagonal entry (exact or near-exact singularity, nothing else).

DF, RSS and GCV are sums over the *supported* samples: those whose
interpolation cell has all 2^d corners *resolved*.  A grid point is resolved
when it is not ill-posed and every pivot of its moment matrix is more than
``RESOLVE`` = 1e-3 times the matching diagonal entry.  The ratio pivot_c / A_cc
is the part of the c-th design column's weighted second moment that the
earlier columns do not explain (one minus its uncentred R^2, the reciprocal
of its variance inflation factor), so the rule keeps the points whose local
design has VIF <= 1000 in every direction; it does not depend on the
bandwidth equilibration.  The Girard ratio, RSS and GCV of eq. (22) then use
N_I supported samples in place of N.  In the variance pass, samples whose
residual is undefined (the mean fit is NaN at a corner of their cell) are
left out of the second fit and of kappa.  ``rgcv_select`` skips NaN GCV values.

No part of this module is pinned to the fast path's arithmetic: every
threshold here is a fixed reading of the method, not a round-off model.

Parity pins for every function here live in ``tests/test_oracle_*.py``.
"""
from __future__ import annotations

import ctypes
import itertools
import os
import subprocess
from typing import Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "fkr_oracle.c")
_LIB = os.path.join(_HERE, "libfkr_oracle.so")
_lib = None

ILL_REL = 1e-12      # relative pivot at or below which a point is ill-posed
RESOLVE = 1e-3       # pivot / A_cc above which a point supports DF / RSS sums


def build(force: bool = True) -> str:
    """Compile the C part of the oracle with gcc (OpenMP, FP64, -O2)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-shared", "-fPIC", "-std=gnu11",
                               _SRC, "-o", tmp, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build(force=True)
        lib = ctypes.CDLL(_LIB)
        P = ctypes.c_void_p
        lib.orc_moments.argtypes = [ctypes.c_int, ctypes.c_int64, P, ctypes.c_int, P, P,
                                    ctypes.c_int, P, ctypes.c_int, P, ctypes.c_int64, P,
                                    P, P, ctypes.c_int]
        lib.orc_moments.restype = ctypes.c_int
        lib.orc_nudft.argtypes = [ctypes.c_int, ctypes.c_int64, P, P, P, ctypes.c_int, P, P, P]
        lib.orc_nudft.restype = ctypes.c_int
        lib.orc_threads.argtypes = []
        lib.orc_threads.restype = ctypes.c_int
        _lib = lib
    return _lib


def threads() -> int:
    """OpenMP threads used by the C loops."""
    return int(_load().orc_threads())


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


# ---------------------------------------------------------------------------
# Grid and monomials
# ---------------------------------------------------------------------------

def multi_indices(d: int, deg: int) -> list:
    """All exponent tuples of total degree <= deg: degree ascending; within a
    degree, the exponent of dimension 0 descending, then dimension 1, ...
    (eq. (4)/(14): the row [1, x^T, vech(x x^T), ...])."""
    out = []

    def rec(prefix, left, dims):
        if dims == 1:
            out.append(tuple(prefix + [left]))
            return
        for a in range(left, -1, -1):
            rec(prefix + [a], left - a, dims - 1)

    for t in range(deg + 1):
        rec([], t, d)
    return out


def grid_axes(M: Sequence[int], lo: Sequence[float], hi: Sequence[float]) -> list:
    """Per-dimension grid coordinates g_k = lo + k * (hi - lo) / (M - 1)
    (eq. (6) with the spacing of Sec. 1.1)."""
    return [lo[j] + np.arange(M[j]) * ((hi[j] - lo[j]) / (M[j] - 1)) for j in range(len(M))]


def grid_points(M, lo, hi) -> np.ndarray:
    """All grid points, flattened with the index of dimension 0 fastest."""
    ax = grid_axes(M, lo, hi)
    mesh = np.meshgrid(*ax[::-1], indexing="ij")
    return np.stack([m.ravel() for m in mesh[::-1]], axis=1)


def flat_index(k: Sequence[int], M: Sequence[int]) -> int:
    idx, stride = 0, 1
    for j in range(len(M)):
        idx += int(k[j]) * stride
        stride *= int(M[j])
    return idx


# ---------------------------------------------------------------------------
# Moments (eq. 9) and the normal-equation solve (eq. 3 / 11)
# ---------------------------------------------------------------------------

def moments(X: np.ndarray, W: Optional[np.ndarray], h: Sequence[float], order: int,
            gpts: np.ndarray, cutoff: bool = True):
    """s_a(g) for |a| <= 2 order and t_{w,b}(g) for |b| <= order, weights W
    (N x nw, real).  Returns S (G x n_s) and T (G x nw x n_t)."""
    lib = _load()
    X = np.ascontiguousarray(X, dtype=np.float64)
    N, d = X.shape
    if W is None:
        W = np.zeros((N, 0))
    W = np.ascontiguousarray(W, dtype=np.float64).reshape(N, -1)
    nw = W.shape[1]
    gpts = np.ascontiguousarray(gpts, dtype=np.float64).reshape(-1, d)
    G = gpts.shape[0]
    es = np.ascontiguousarray(multi_indices(d, 2 * order), dtype=np.int32)
    et = np.ascontiguousarray(multi_indices(d, order), dtype=np.int32)
    h = np.ascontiguousarray(h, dtype=np.float64)
    S = np.zeros((G, len(es)))
    T = np.zeros((G, nw, len(et)))
    rc = lib.orc_moments(d, N, _ptr(X), nw, _ptr(W), _ptr(h), len(es), _ptr(es), len(et),
                         _ptr(et), G, _ptr(gpts), _ptr(S), _ptr(T), 1 if cutoff else 0)
    if rc != 0:
        raise ValueError(f"orc_moments failed ({rc})")
    return S, T


def assemble(S: np.ndarray, h: Sequence[float], order: int, d: int) -> np.ndarray:
    """Equilibrated moment matrix A~_bc = s_{b+c} / h^{b+c} (G x P x P)."""
    es = multi_indices(d, 2 * order)
    et = multi_indices(d, order)
    pos = {a: i for i, a in enumerate(es)}
    h = np.asarray(h, dtype=np.float64)
    P = len(et)
    A = np.empty((S.shape[0], P, P))
    for b in range(P):
        for c in range(P):
            a = tuple(et[b][j] + et[c][j] for j in range(d))
            A[:, b, c] = S[:, pos[a]] / np.prod(h ** np.array(a))
    return A


def pivots(A: np.ndarray) -> np.ndarray:
    """Pivots of the triangular (Cholesky / LDL^T) factorisation of each
    symmetric matrix in A (G x P x P), from their definition as ratios of
    leading principal minors: pivot_c = det A[:c+1, :c+1] / det A[:c, :c].
    Each matrix is scaled by its (0, 0) entry first to keep the
    determinants in range; rows with A_00 <= 0 give NaN."""
    G, P, _ = A.shape
    a00 = A[:, 0, 0]
    with np.errstate(divide="ignore", invalid="ignore"):
        B = A / a00[:, None, None]
        minors = np.ones((G, P + 1))
        for c in range(1, P + 1):
            minors[:, c] = np.linalg.det(B[:, :c, :c])
        pv = minors[:, 1:] / minors[:, :-1] * a00[:, None]
    pv[~(a00 > 0)] = np.nan
    return pv


def relative_pivots(A: np.ndarray) -> np.ndarray:
    """pivot_c / A_cc for each symmetric matrix in A (G x P x P): one minus
    the uncentred R^2 of design column c on the columns before it (the
    reciprocal of its variance inflation factor).  Invariant to diagonal
    scaling, so the bandwidth equilibration does not change it."""
    with np.errstate(divide="ignore", invalid="ignore"):
        return pivots(A) / np.diagonal(A, axis1=1, axis2=2)


def resolved(S: np.ndarray, h: Sequence[float], order: int, d: int,
             kappa: float = RESOLVE) -> np.ndarray:
    """Grid points whose moment matrix is resolved: every relative pivot
    exceeds kappa (VIF <= 1 / kappa in every design direction)."""
    rp = relative_pivots(assemble(S, h, order, d))
    with np.errstate(invalid="ignore"):
        return np.all(rp > kappa, axis=1)


def solve(S: np.ndarray, T: np.ndarray, h: Sequence[float], order: int, d: int):
    """Per grid point: solve A c = t (eq. 3 / 11) and return
    mhat (G x nw) = c_0, r0 (G x P) = row 0 of the inverse of the
    equilibrated matrix, and the ill-posed mask (G,): some pivot of the
    equilibrated matrix is at most 1e-12 A_cc."""
    et = multi_indices(d, order)
    h = np.asarray(h, dtype=np.float64)
    scale = np.array([np.prod(h ** np.array(b)) for b in et])
    A = assemble(S, h, order, d)
    rhs = T / scale[None, None, :]
    G, nw, P = rhs.shape
    pv = pivots(A)
    thr = ILL_REL * np.diagonal(A, axis1=1, axis2=2)
    with np.errstate(invalid="ignore"):
        ill = ~np.all(pv > thr, axis=1)
    ok = ~ill
    mhat = np.full((G, nw), np.nan)
    r0 = np.full((G, P), np.nan)
    if ok.any():
        Ainv = np.linalg.inv(A[ok])
        r0[ok] = Ainv[:, 0, :]
        if nw:
            c = np.linalg.solve(A[ok], np.transpose(rhs[ok], (0, 2, 1)))
            mhat[ok] = c[:, 0, :]
    return mhat, r0, ill


def moments_full(X: np.ndarray, W: Optional[np.ndarray], H: np.ndarray, order: int, gpts: np.ndarray):
    """s_a(g) and t_{w,b}(g) of eq. (9) for the Gaussian kernel with a full
    bandwidth matrix H (eq. 2: K_H(u) = |H|^{-1/2} K(H^{-1/2} u), K the
    standard normal density, so K_H(u) = exp(-u^T H^{-1} u / 2) /
    ((2 pi)^{d/2} |H|^{1/2})), by direct summation in NumPy.  Returns S
    (G x n_s) and T (G x nw x n_t)."""
    X = np.asarray(X, dtype=np.float64)
    if X.ndim == 1:
        X = X[:, None]
    N, d = X.shape
    H = np.asarray(H, dtype=np.float64).reshape(d, d)
    Hi = np.linalg.inv(H)
    norm = 1.0 / np.sqrt((2.0 * np.pi) ** d * np.linalg.det(H))
    W = np.zeros((N, 0)) if W is None else np.asarray(W, dtype=np.float64).reshape(N, -1)
    gpts = np.asarray(gpts, dtype=np.float64).reshape(-1, d)
    es = np.array(multi_indices(d, 2 * order))
    et = np.array(multi_indices(d, order))
    S = np.zeros((len(gpts), len(es)))
    T = np.zeros((len(gpts), W.shape[1], len(et)))
    for g in range(len(gpts)):
        u = X - gpts[g]                                        # z = x_i - g
        K = norm * np.exp(-0.5 * np.einsum("ij,jk,ik->i", u, Hi, u))
        for a, e in enumerate(es):
            S[g, a] = np.sum(K * np.prod(u ** e, axis=1))
        for b, e in enumerate(et):
            T[g, :, b] = (K * np.prod(u ** e, axis=1)) @ W
    return S, T


def fit_full(X, Y, H, order, gpts):
    """m_hat(g) of eq. (3) with the full bandwidth matrix H (real Y, N x q),
    the moment matrix equilibrated by sqrt(diag H).  Returns (mhat, S, ill)."""
    X = np.asarray(X, dtype=np.float64)
    if X.ndim == 1:
        X = X[:, None]
    d = X.shape[1]
    W = np.asarray(Y, dtype=np.float64).reshape(X.shape[0], -1)
    S, T = moments_full(X, W, H, order, gpts)
    s = np.sqrt(np.diag(np.asarray(H, dtype=np.float64).reshape(d, d)))
    mhat, r0, ill = solve(S, T, s, order, d)
    return mhat, S, ill


COMPACT_KERNELS = ("box", "triangle", "epanechnikov", "biweight", "triweight")


def compact_kernel(name: str, u):
    """The compact kernels of Table 1 on |u| <= 1 (each integrates to one)."""
    u = np.asarray(u, dtype=np.float64)
    q = 1.0 - u * u
    inside = np.abs(u) <= 1.0
    v = {"box": np.full_like(u, 0.5), "triangle": 1.0 - np.abs(u), "epanechnikov": 0.75 * q,
         "biweight": 15.0 / 16.0 * q ** 2, "triweight": 35.0 / 32.0 * q ** 3}[name]
    return np.where(inside, v, 0.0)


def moments_compact(X, W, h, order, gpts, kernel: str):
    """The exact moment sums of eq. (9) for the product kernel
    K_h(u) = prod_j K(u_j / h_j) / h_j of a compact K, by direct summation."""
    X = np.asarray(X, dtype=np.float64)
    if X.ndim == 1:
        X = X[:, None]
    N, d = X.shape
    h = np.asarray(h, dtype=np.float64)
    W = np.zeros((N, 0)) if W is None else np.asarray(W, dtype=np.float64).reshape(N, -1)
    gpts = np.asarray(gpts, dtype=np.float64).reshape(-1, d)
    es, et = np.array(multi_indices(d, 2 * order)), np.array(multi_indices(d, order))
    S = np.zeros((len(gpts), len(es)))
    T = np.zeros((len(gpts), W.shape[1], len(et)))
    for g in range(len(gpts)):
        u = X - gpts[g]
        K = np.prod(compact_kernel(kernel, u / h) / h, axis=1)
        for a, e in enumerate(es):
            S[g, a] = np.sum(K * np.prod(u ** e, axis=1))
        for b, e in enumerate(et):
            T[g, :, b] = (K * np.prod(u ** e, axis=1)) @ W
    return S, T


def moments_binned(X, W, h, order, gpts, kernel: str, delta, L, square: bool = False, sw=None):
    """The binned approximation of the moment sums (eq. 11-13): the moment
    kernels k_a(z) = z^a K_h(z) sampled at the grid offsets m delta over one
    period T = L delta and convolved with the samples through their discrete
    transform, which makes each sample's contribution the trigonometric
    interpolant of the sampled kernel (the Fourier series of the periodised
    samples over every mode |n| <= L / 2, the modes +-L/2 of an even L with
    half the Nyquist coefficient each) at x_i - g.  Per dimension the
    transform is NumPy's FFT of the samples; the series is summed directly.
    square: the sampled kernel is K(z / h)^2 / h per dimension (the squared
    kernel of the variance of the fit, up to prod_j 1 / h_j); sw: weights of
    the samples in S (default one)."""
    X = np.asarray(X, dtype=np.float64)
    if X.ndim == 1:
        X = X[:, None]
    N, d = X.shape
    h = np.asarray(h, dtype=np.float64)
    delta = np.asarray(delta, dtype=np.float64).reshape(d)
    L = np.asarray(L, dtype=np.int64).reshape(d)
    W = np.zeros((N, 0)) if W is None else np.asarray(W, dtype=np.float64).reshape(N, -1)
    gpts = np.asarray(gpts, dtype=np.float64).reshape(-1, d)
    es, et = np.array(multi_indices(d, 2 * order)), np.array(multi_indices(d, order))
    deg = 2 * order
    # per dimension: coefficients c_{j,a}(n) of the interpolant of z^a K_h(z)
    coef, freq = [], []
    for j in range(d):
        m = np.arange(L[j])
        z = np.where(m <= L[j] // 2, m, m - L[j]) * delta[j]            # periodised offsets
        kz = compact_kernel(kernel, z / h[j]) ** (2 if square else 1) / h[j]
        K = L[j] // 2
        n = np.arange(-K, K + 1)
        half = np.where(2 * np.abs(n) == L[j], 0.5, 1.0)                # even L: +-L/2 share the Nyquist term
        cj = []
        for a in range(deg + 1):
            F = np.fft.fft(z ** a * kz) * delta[j]                      # sum_m k(z_m) e^{-2 pi i n m / L} delta
            cj.append(half * F[n % L[j]] / (L[j] * delta[j]))
        coef.append(np.array(cj))
        freq.append(2.0 * np.pi * n / (L[j] * delta[j]))
    S = np.zeros((len(gpts), len(es)))
    T = np.zeros((len(gpts), W.shape[1], len(et)))
    sw = np.ones(N) if sw is None else np.asarray(sw, dtype=np.float64).reshape(N)
    for g in range(len(gpts)):
        u = X - gpts[g]
        # interpolant values per dimension and degree: [d][deg+1][N]
        vals = [np.real(np.exp(1j * np.outer(u[:, j], freq[j])) @ coef[j].T).T for j in range(d)]
        for a, e in enumerate(es):
            S[g, a] = np.sum(sw * np.prod([vals[j][e[j]] for j in range(d)], axis=0))
        for b, e in enumerate(et):
            T[g, :, b] = np.prod([vals[j][e[j]] for j in range(d)], axis=0) @ W
    return S, T


def _split_complex(Y: np.ndarray):
    Y = np.asarray(Y)
    if Y.ndim == 1:
        Y = Y[:, None]
    if np.iscomplexobj(Y):
        return np.concatenate([Y.real, Y.imag], axis=1), True
    return Y.astype(np.float64), False


def _moments_of(X, W, h, order, gpts, binned, H=None):
    """The Gaussian moment sums (``moments``), with binned = (kernel, delta,
    L) those of the binned approximation of a compact kernel
    (``moments_binned``), or with H those of the Gaussian with the full
    bandwidth matrix H (``moments_full``)."""
    if H is not None:
        return moments_full(X, W, H, order, gpts)
    if binned is None:
        return moments(X, W, h, order, gpts)
    name, delta, L = binned
    return moments_binned(X, W, h, order, gpts, name, delta, L)


def _equilibration(h, H, d):
    """The equilibration of the moment matrix: h, or sqrt(diag H) for a full
    bandwidth matrix."""
    if H is None:
        return h
    return np.sqrt(np.diag(np.asarray(H, dtype=np.float64).reshape(d, d)))


def fit(X, Y, h, order, gpts, return_all: bool = False, binned=None, H=None):
    """m_hat(g; l) of eq. (11) at the given grid points, for each response
    column (complex responses: real and imaginary parts share the real moment
    matrix).  Returns mhat (G x q) [, S, T, r0, ill]."""
    X = np.asarray(X, dtype=np.float64)
    if X.ndim == 1:
        X = X[:, None]
    d = X.shape[1]
    W, cplx = _split_complex(Y)
    S, T = _moments_of(X, W, h, order, gpts, binned, H)
    mhat, r0, ill = solve(S, T, _equilibration(h, H, d), order, d)
    if cplx:
        q = W.shape[1] // 2
        mhat = mhat[:, :q] + 1j * mhat[:, q:]
    if return_all:
        return mhat, S, T, r0, ill
    return mhat


# ---------------------------------------------------------------------------
# Interpolation (Sec. 1.1 end, Sec. 5: linear griddedInterpolant)
# ---------------------------------------------------------------------------

def cell_corners(M, lo, hi, Xq: np.ndarray) -> np.ndarray:
    """Flat grid indices (n x 2^d) of the corners of each point's
    interpolation cell, floor((x - lo)/Delta) clamped to [0, M - 2]."""
    Xq = np.asarray(Xq, dtype=np.float64)
    if Xq.ndim == 1:
        Xq = Xq[:, None]
    d = Xq.shape[1]
    cell = []
    for j in range(d):
        delta = (hi[j] - lo[j]) / (M[j] - 1)
        cell.append(np.clip(np.floor((Xq[:, j] - lo[j]) / delta).astype(np.int64), 0, M[j] - 2))
    out = np.zeros((Xq.shape[0], 1 << d), dtype=np.int64)
    for q, corner in enumerate(itertools.product((0, 1), repeat=d)):
        stride = 1
        for j in range(d):
            out[:, q] += (cell[j] + corner[j]) * stride
            stride *= M[j]
    return out


def supported(ok_grid: np.ndarray, M, lo, hi, X: np.ndarray) -> np.ndarray:
    """Samples whose interpolation cell has every corner in ok_grid."""
    return np.all(np.asarray(ok_grid, dtype=bool)[cell_corners(M, lo, hi, X)], axis=1)


def interp(values: np.ndarray, M, lo, hi, Xq: np.ndarray) -> np.ndarray:
    """Multilinear interpolation of grid values (G x k, or G) at Xq (n x d).
    The cell of x is floor((x - lo)/Delta) clamped to [0, M - 2], so a point on
    hi uses the last cell with weight 1 on its upper corner."""
    Xq = np.asarray(Xq, dtype=np.float64)
    if Xq.ndim == 1:
        Xq = Xq[:, None]
    d = Xq.shape[1]
    vals = np.asarray(values)
    squeeze = vals.ndim == 1
    vals = vals.reshape(int(np.prod(M)), -1)
    cell, frac = [], []
    for j in range(d):
        delta = (hi[j] - lo[j]) / (M[j] - 1)
        t = (Xq[:, j] - lo[j]) / delta
        k = np.clip(np.floor(t).astype(np.int64), 0, M[j] - 2)
        cell.append(k)
        frac.append(t - k)
    out = np.zeros((Xq.shape[0], vals.shape[1]), dtype=vals.dtype)
    for corner in itertools.product((0, 1), repeat=d):
        wgt = np.ones(Xq.shape[0])
        idx = np.zeros(Xq.shape[0], dtype=np.int64)
        stride = 1
        for j in range(d):
            wgt = wgt * (frac[j] if corner[j] else (1.0 - frac[j]))
            idx += (cell[j] + corner[j]) * stride
            stride *= M[j]
        out += wgt[:, None] * vals[idx]
    return out[:, 0] if squeeze else out


# ---------------------------------------------------------------------------
# Probes: Philox4x32-10 + Box-Muller (Sec. 2.1 step i)
# ---------------------------------------------------------------------------

_PH_M0, _PH_M1 = np.uint64(0xD2511F53), np.uint64(0xCD9E8D57)   # round multipliers
_PH_W0, _PH_W1 = np.uint64(0x9E3779B9), np.uint64(0xBB67AE85)   # key increments
_LO32 = np.uint64(0xFFFFFFFF)
_S32 = np.uint64(32)


def philox4x32(ctr: np.ndarray, key: Sequence[int], rounds: int = 10) -> np.ndarray:
    """Philox4x32 (Salmon, Moraes, Dror, Shaw, SC'11), 10 rounds by default.
    ctr: (n, 4) words < 2^32; key: two words.  Products are formed exactly in
    uint64.  Returns (n, 4) uint64 holding 32-bit words."""
    c = [np.array(ctr[:, i], dtype=np.uint64) & _LO32 for i in range(4)]
    k0, k1 = np.uint64(key[0]) & _LO32, np.uint64(key[1]) & _LO32
    for _ in range(rounds):
        p0 = c[0] * _PH_M0
        p1 = c[2] * _PH_M1
        c = [(p1 >> _S32) ^ c[1] ^ k0, p1 & _LO32, (p0 >> _S32) ^ c[3] ^ k1, p0 & _LO32]
        k0 = (k0 + _PH_W0) & _LO32
        k1 = (k1 + _PH_W1) & _LO32
    return np.stack(c, axis=1)


def probes(seed: int, N: int, Np: int, index: Optional[np.ndarray] = None) -> np.ndarray:
    """N x Np standard normal probes.  Sample i, probe p = 4 g + r uses the
    Philox4x32-10 block with counter (i mod 2^32, floor(i / 2^32), g, 0) and
    key (seed mod 2^32, floor(seed / 2^32) mod 2^32); each of its words x_k
    gives the uniform u_k = (floor(x_k / 2^8) + 1/2) 2^-24 in (0, 1) (exact in
    single and double precision), and Box-Muller gives
    sqrt(-2 ln u0) (cos, sin)(2 pi u1) for r = 0, 1 and
    sqrt(-2 ln u2) (cos, sin)(2 pi u3) for r = 2, 3."""
    idx = np.arange(N, dtype=np.uint64) if index is None else np.asarray(index, dtype=np.uint64)
    out = np.empty((idx.size, Np))
    key = (int(seed) & 0xFFFFFFFF, (int(seed) >> 32) & 0xFFFFFFFF)
    for g in range((Np + 3) // 4):
        ctr = np.zeros((idx.size, 4), dtype=np.uint64)
        ctr[:, 0] = idx & _LO32
        ctr[:, 1] = idx >> _S32
        ctr[:, 2] = g
        x = philox4x32(ctr, key)
        u = ((x >> np.uint64(8)).astype(np.float64) + 0.5) * 2.0 ** -24
        r0 = np.sqrt(-2.0 * np.log(u[:, 0]))
        r1 = np.sqrt(-2.0 * np.log(u[:, 2]))
        z = [r0 * np.cos(2 * np.pi * u[:, 1]), r0 * np.sin(2 * np.pi * u[:, 1]),
             r1 * np.cos(2 * np.pi * u[:, 3]), r1 * np.sin(2 * np.pi * u[:, 3])]
        for r in range(4):
            p = 4 * g + r
            if p < Np:
                out[:, p] = z[r]
    return out


# ---------------------------------------------------------------------------
# DF (Sec. 2.1), GCV (eq. 22), relaxed selection (Table 1, dstd)
# ---------------------------------------------------------------------------

def girard_ratios(Wp: np.ndarray, What: np.ndarray) -> np.ndarray:
    """rho_p = w_p^T (w_p - w_hat_p) / (w_p^T w_p) for each probe column."""
    return np.einsum("ip,ip->p", Wp, Wp - What) / np.einsum("ip,ip->p", Wp, Wp)


def support(X, h, order, M, lo, hi, kappa: float = RESOLVE, binned=None, H=None):
    """Supported samples at bandwidth h (see the module docstring): the grid
    fit of the density moments, the resolved points, and the samples whose
    cell corners are all resolved.  Returns (supported samples, resolved
    grid points)."""
    X = np.asarray(X, dtype=np.float64)
    if X.ndim == 1:
        X = X[:, None]
    d = X.shape[1]
    S, _ = _moments_of(X, None, h, order, grid_points(M, lo, hi), binned, H)
    ok = resolved(S, _equilibration(h, H, d), order, d, kappa)
    return supported(ok, M, lo, hi, X), ok


def dof(X, h, order, M, lo, hi, Wp, kappa: float = RESOLVE, include=None):
    """Fast Monte-Carlo DF (Sec. 2.1): each probe is pushed through the grid
    smoother (moments -> solve -> interpolation back to the samples), and the
    Girard ratio is taken over the supported samples I (``include``, or the
    rule of ``support`` with ``kappa``; kappa = 0 keeps every sample whose
    cell has no ill-posed corner):
        rho_p = sum_I w_ip (w_ip - w_hat_ip) / sum_I w_ip^2.
    Returns (rho per probe, mean rho ~ (1/N_I) tr((I - S)_II),
    DF = N_I (1 - mean), supported-sample mask)."""
    X = np.asarray(X, dtype=np.float64).reshape(len(Wp), -1)
    d = X.shape[1]
    gp = grid_points(M, lo, hi)
    mh, S, T, r0, ill = fit(X, Wp, h, order, gp, return_all=True)
    if include is None:
        ok = ~ill & (resolved(S, h, order, d, kappa) if kappa > 0 else True)
        include = supported(ok, M, lo, hi, X)
    include = np.asarray(include, dtype=bool)
    What = interp(mh, M, lo, hi, X)
    rho = girard_ratios(Wp[include], What[include])
    m = float(np.mean(rho))
    return rho, m, int(include.sum()) * (1.0 - m), include


def gcv(y: np.ndarray, yhat: np.ndarray, rho_mean: float, include=None) -> np.ndarray:
    """eq. (22): (1/N_I) sum_I |y - yhat|^2 / [(1/N_I) tr((I - S)_II)]^2 per
    response column over the supported samples I (all when include is
    None); |.|^2 for complex responses."""
    r = np.asarray(y) - np.asarray(yhat)
    r = r.reshape(r.shape[0], -1)
    if include is not None:
        r = r[np.asarray(include, dtype=bool)]
    return np.mean(np.abs(r) ** 2, axis=0) / rho_mean ** 2


def gcv_criterion(X, y, h, order, M, lo, hi, Wp, include=None, binned=None, H=None) -> float:
    """GCV of eq. (22) at bandwidth h for one real response y, with the DF
    from the probes Wp (``dof``), over the supported samples I (``include``,
    else the support rule at h).  binned: a compact kernel's binned moments;
    H: a full bandwidth matrix in place of h (see ``fit``)."""
    y = np.asarray(y).reshape(-1)
    X = np.asarray(X, dtype=np.float64).reshape(len(y), -1)
    Yr, cplx = _split_complex(y)          # complex y: real and imaginary parts
    ny = Yr.shape[1]
    W = np.concatenate([Yr, Wp], axis=1)
    gp = grid_points(M, lo, hi)
    mh, S, T, r0, ill = fit(X, W, h, order, gp, return_all=True, binned=binned, H=H)
    d = X.shape[1]
    if include is None:
        include = supported(~ill & resolved(S, _equilibration(h, H, d), order, d), M, lo, hi, X)
    include = np.asarray(include, dtype=bool)
    F = interp(mh, M, lo, hi, X)
    rho = girard_ratios(Wp[include], F[include, ny:])
    yhat = F[:, 0] + 1j * F[:, 1] if cplx else F[:, 0]
    return float(gcv(y, yhat, float(np.mean(rho)), include=include)[0])


def gcv_log_h_gradient(X, y, h, order, M, lo, hi, Wp, include=None, step: float = 1e-4,
                       binned=None) -> np.ndarray:
    """d GCV / d log h_j by central differences of ``gcv_criterion`` (step
    in log h), with the supported set held at that of h."""
    h = np.asarray(h, dtype=np.float64)
    X = np.asarray(X, dtype=np.float64).reshape(len(y), -1)
    if include is None:
        include = support(X, h, order, M, lo, hi, binned=binned)[0]
    out = np.empty(len(h))
    for j in range(len(h)):
        e = np.zeros(len(h))
        e[j] = step
        gp_ = gcv_criterion(X, y, h * np.exp(e), order, M, lo, hi, Wp, include, binned)
        gm_ = gcv_criterion(X, y, h * np.exp(-e), order, M, lo, hi, Wp, include, binned)
        out[j] = (gp_ - gm_) / (2.0 * step)
    return out


def gcv_H_gradient(X, y, H, order, M, lo, hi, Wp, include=None, step: float = 1e-4) -> np.ndarray:
    """d GCV / d H_pq (p <= q, row-major upper triangle; an off-diagonal
    entry moves H_pq and H_qp together) at a full bandwidth matrix, by
    central differences of ``gcv_criterion`` with step * H_pq' where
    H_pq' = sqrt(H_pp H_qq), with the supported set held at that of H."""
    X = np.asarray(X, dtype=np.float64).reshape(len(y), -1)
    d = X.shape[1]
    H = np.asarray(H, dtype=np.float64).reshape(d, d)
    if include is None:
        include = support(X, None, order, M, lo, hi, H=H)[0]
    out = []
    for p in range(d):
        for q in range(p, d):
            E = np.zeros((d, d))
            E[p, q] = E[q, p] = 1.0
            eps = step * np.sqrt(H[p, p] * H[q, q])
            gp_ = gcv_criterion(X, y, None, order, M, lo, hi, Wp, include, H=H + eps * E)
            gm_ = gcv_criterion(X, y, None, order, M, lo, hi, Wp, include, H=H - eps * E)
            out.append((gp_ - gm_) / (2.0 * eps))
    return np.array(out)


def gcv_y_gradient(X, y, h, order, M, lo, hi, Wp, include=None, binned=None, H=None) -> np.ndarray:
    """d GCV / dy of ``gcv_criterion`` from its definition: the fitted
    values are yhat = S y with the smoother S (samples to samples through the
    grid fit and the interpolation) built column by column from the fits of
    the unit responses; the Girard ratios do not depend on y, so with
    r = (y - S y) on the supported samples I,
    d GCV / dy = 2 / (N_I rho_bar^2) (r - S_I^T r_I).  H: a full bandwidth
    matrix in place of h (see ``fit``)."""
    y = np.asarray(y).reshape(-1)
    N = len(y)
    X = np.asarray(X, dtype=np.float64).reshape(N, -1)
    d = X.shape[1]
    gp = grid_points(M, lo, hi)
    mh, S, T, r0, ill = fit(X, np.concatenate([np.eye(N), Wp], axis=1), h, order, gp, return_all=True,
                            binned=binned, H=H)
    if include is None:
        include = supported(~ill & resolved(S, _equilibration(h, H, d), order, d), M, lo, hi, X)
    include = np.asarray(include, dtype=bool)
    F = interp(mh, M, lo, hi, X)
    Smat = F[include, :N]                       # rows of the supported samples
    rho = girard_ratios(Wp[include], F[include, N:])
    m = float(np.mean(rho))
    # S is real: for complex y the same formula holds for the real and the
    # imaginary part, d/dRe y + i d/dIm y
    r = y[include] - Smat @ y
    g = np.zeros(N, dtype=r.dtype)
    g[include] = r
    return 2.0 / (include.sum() * m * m) * (g - Smat.T @ r)


def rgcv_select(gcv_values: Sequence[float], dstd: float = 0.0) -> int:
    """Index of the selected bandwidth: the last (largest, for an ascending
    list) h whose GCV is within dstd * std(GCV) of the minimum; dstd = 0 is
    the plain argmin with ties going to the larger h.  std uses N - 1 and,
    like the minimum, only the finite entries."""
    g = np.asarray(gcv_values, dtype=np.float64)
    f = g[np.isfinite(g)]
    if f.size == 0:
        raise ValueError("no finite GCV value")
    thr = np.min(f) + (dstd * np.std(f, ddof=1) if dstd > 0 and f.size > 1 else 0.0)
    return int(np.nonzero(np.isfinite(g) & (g <= thr))[0][-1])


def get_hlist(n, rng, kind: str = "log") -> np.ndarray:
    """Bandwidth candidates (Sec. 4, get_hList).  1-D: n values over rng =
    [a, b], inclusive of both ends, log- or linearly spaced.  d-D: n and rng
    per dimension; the result is every combination (dimension 0 fastest),
    one row per candidate."""
    n = np.atleast_1d(n).astype(int)
    rng = np.atleast_2d(np.asarray(rng, dtype=np.float64))
    axes = []
    for j in range(len(n)):
        a, b = rng[j]
        if kind == "log":
            axes.append(np.logspace(np.log10(a), np.log10(b), n[j]))
        elif kind == "lin":
            axes.append(np.linspace(a, b, n[j]))
        else:
            raise ValueError(kind)
    if len(axes) == 1:
        return axes[0][:, None]
    mesh = np.meshgrid(*axes[::-1], indexing="ij")
    return np.stack([m.ravel() for m in mesh[::-1]], axis=1)


# ---------------------------------------------------------------------------
# Conditional variance (Sec. 3)
# ---------------------------------------------------------------------------

def variance(X, y, yhat_at_samples, h, order, M, lo, hi, mode: str = "log",
             gpts: Optional[np.ndarray] = None, H=None):
    """Second pass on squared residuals r_i = |y_i - yhat(x_i)|^2.

    Samples whose residual is undefined (NaN mean fit at their cell) are left
    out of the second fit and of kappa.
    mode "log" (eq. 24-26): v = local fit of log(r_i + 1/N); kappa =
    [mean_i r_i exp(-v(x_i))]^-1 with v(x_i) interpolated from the full grid,
    over the samples where that term is defined; sigma^2(g) = exp(v(g)) / kappa.
    mode "direct" (eq. 23): sigma^2(g) = local fit of r_i.  H: the second
    fit with that full bandwidth matrix (h unused).
    Returns (sigma2 at gpts (or the full grid), extras dict)."""
    X = np.asarray(X, dtype=np.float64).reshape(len(yhat_at_samples), -1)
    N = X.shape[0]
    r = np.abs(np.asarray(y).reshape(N) - np.asarray(yhat_at_samples).reshape(N)) ** 2
    keep = np.isfinite(r)
    full = grid_points(M, lo, hi)
    if mode == "direct":
        s2 = fit(X[keep], r[keep], h, order, full if gpts is None else gpts, H=H)[:, 0]
        return s2, {"r": r}
    z = np.log(r + 1.0 / N)
    v_full = fit(X[keep], z[keep], h, order, full, H=H)[:, 0]
    v_i = interp(v_full, M, lo, hi, X)
    term = r * np.exp(-v_i)
    kappa = 1.0 / np.mean(term[np.isfinite(term)])
    v = v_full if gpts is None else fit(X[keep], z[keep], h, order, gpts, H=H)[:, 0]
    return np.exp(v) / kappa, {"r": r, "z": z, "v": v_full, "kappa": kappa}


# ---------------------------------------------------------------------------
# Stage oracle for the NUFFT (type-1 definition, Sec. 1.2)
# ---------------------------------------------------------------------------

def nudft(X, W, lo, period, K) -> np.ndarray:
    """c(n) = sum_i w_i exp(-i sum_j 2 pi n_j (x_ij - lo_j)/T_j) for
    n_j = -K_j..K_j.  W: N x nw (complex allowed).  Returns an array of shape
    (2K_{d-1}+1, ..., 2K_0+1, nw) (n_0 fastest before the weight index)."""
    lib = _load()
    X = np.ascontiguousarray(X, dtype=np.float64)
    if X.ndim == 1:
        X = X[:, None]
    N, d = X.shape
    Wc = np.asarray(W).reshape(N, -1).astype(np.complex128)
    nw = Wc.shape[1]
    Wri = np.ascontiguousarray(Wc.view(np.float64).reshape(N, nw, 2))
    K = np.ascontiguousarray(K, dtype=np.int32)
    B = int(np.prod(2 * K + 1))
    out = np.zeros((B, nw, 2))
    rc = lib.orc_nudft(d, N, _ptr(X), _ptr(np.ascontiguousarray(lo, dtype=np.float64)),
                       _ptr(np.ascontiguousarray(period, dtype=np.float64)), nw, _ptr(Wri),
                       _ptr(K), _ptr(out))
    if rc != 0:
        raise ValueError("orc_nudft failed")
    c = out[..., 0] + 1j * out[..., 1]
    return c.reshape(tuple((2 * K + 1)[::-1]) + (nw,))


# ---------------------------------------------------------------------------
# Prediction and pointwise inference (Sec. 4 fkreg_predict and
# fkreg_interval, Table 1 y_grid_opt; Sec. 4.2 eq. 27-28)
# ---------------------------------------------------------------------------

def spline_second_derivatives(f: np.ndarray) -> np.ndarray:
    """Second derivatives (in index units, spacing 1) of the not-a-knot cubic
    interpolating spline through f[0], ..., f[n-1] at consecutive integer
    nodes, along axis 0 (any trailing shape: one spline per column).

    The spline is C^2 at every interior node, which gives
    m_{k-1} + 4 m_k + m_{k+1} = 6 (f_{k-1} - 2 f_k + f_{k+1}) for k = 1..n-2,
    and its third derivative is continuous at nodes 1 and n-2 (the
    not-a-knot ends): m_0 - 2 m_1 + m_2 = 0 and m_{n-3} - 2 m_{n-2} + m_{n-1}
    = 0.  Three nodes: the interpolating parabola (constant m); two: the
    line (m = 0).  Solved as one dense linear system."""
    f = np.asarray(f, dtype=np.float64)
    n = f.shape[0]
    rest = f.shape[1:]
    F = f.reshape(n, -1)
    if n <= 2:
        return np.zeros_like(f)
    A = np.zeros((n, n))
    R = np.zeros((n, F.shape[1]))
    for k in range(1, n - 1):
        A[k, k - 1:k + 2] = (1.0, 4.0, 1.0)
        R[k] = 6.0 * (F[k - 1] - 2.0 * F[k] + F[k + 1])
    if n == 3:
        A[0, :] = (1.0, -1.0, 0.0)
        A[2, :] = (0.0, 1.0, -1.0)
    else:
        A[0, 0:3] = (1.0, -2.0, 1.0)
        A[n - 1, n - 3:n] = (1.0, -2.0, 1.0)
    return np.linalg.solve(A, R).reshape((n,) + rest)


def spline_eval_1d(f: np.ndarray, t: float) -> np.ndarray:
    """Value at index coordinate t of the not-a-knot spline through f along
    axis 0 (node k at t = k).  Inside [0, n-1] the cubic piece of t's
    interval; outside, the tangent line at the nearer end (linear
    extrapolation).  Returns an array of f's trailing shape."""
    f = np.asarray(f, dtype=np.float64)
    n = f.shape[0]
    m = spline_second_derivatives(f)

    def piece(k, u):   # cubic on [k, k+1] at k + u
        a, b = 1.0 - u, u
        return a * f[k] + b * f[k + 1] + ((a ** 3 - a) * m[k] + (b ** 3 - b) * m[k + 1]) / 6.0

    def slope(k, u):   # its derivative
        return f[k + 1] - f[k] + ((1.0 - 3.0 * (1.0 - u) ** 2) * m[k] + (3.0 * u ** 2 - 1.0) * m[k + 1]) / 6.0

    if t < 0.0:
        return piece(0, 0.0) + t * slope(0, 0.0)
    if t > n - 1:
        return piece(n - 2, 1.0) + (t - (n - 1)) * slope(n - 2, 1.0)
    k = min(int(np.floor(t)), n - 2)
    return piece(k, t - k)


def spline_predict(values: np.ndarray, M, lo, hi, Xq: np.ndarray) -> np.ndarray:
    """Tensor-product not-a-knot cubic spline interpolation of a grid function
    (the 'spline' method of griddedInterpolant named by Table 1 y_grid_opt,
    with its 'linear' extrapolation) at the query points Xq (n x d):
    interpolate along one dimension at a time, every grid line of the
    remaining dimensions, down to one value.  values: flat grid, dimension 0
    fastest, optionally with a leading axis of several grid functions."""
    M = [int(m) for m in M]
    d = len(M)
    Xq = np.asarray(Xq, dtype=np.float64).reshape(-1, d)
    V = np.asarray(values, dtype=np.float64).reshape((-1,) + tuple(M[::-1]))   # [nv][M_{d-1}]..[M_0]
    nv = V.shape[0]
    delta = [(hi[j] - lo[j]) / (M[j] - 1) for j in range(d)]
    out = np.empty((nv, Xq.shape[0]))
    for i, x in enumerate(Xq):
        for v in range(nv):
            A = V[v]
            for j in range(d):                      # axis -1 is dimension j now
                t = (x[j] - lo[j]) / delta[j]
                A = spline_eval_1d(np.moveaxis(A, -1, 0), t)
            out[v, i] = float(A)
    return out


def fit_variance(X, sigma2_i, h, order, gpts, kernel: str = "gauss", H=None) -> np.ndarray:
    """Variance of the linear fit m_hat(g) = sum_i S_gi y_i for independent
    errors of variance sigma2_i (the Sigma of eq. 27):
    Sigma(g) = sum_i S_gi^2 sigma2_i, with the smoother weights of eq. (3),
    S_gi = e_1^T A(g)^{-1} K_h(x_i - g) d(x_i - g), d the monomial row of
    eq. (4)/(14).  Computed from its definition: row 0 of the inverse of the
    (equilibrated) moment matrix, then every weight S_gi.  NaN where the fit
    is ill-posed; samples with undefined sigma2_i are left out.  kernel: the
    Gaussian, or a compact kernel of Table 1 (exact sums); H: the Gaussian
    with a full bandwidth matrix (h unused), equilibrated by sqrt(diag H)."""
    X = np.asarray(X, dtype=np.float64)
    if X.ndim == 1:
        X = X[:, None]
    N, d = X.shape
    gpts = np.asarray(gpts, dtype=np.float64).reshape(-1, d)
    if H is not None:
        H = np.asarray(H, dtype=np.float64).reshape(d, d)
        h = np.sqrt(np.diag(H))
        Hi = np.linalg.inv(H)
        hnorm = 1.0 / np.sqrt((2.0 * np.pi) ** d * np.linalg.det(H))
    h = np.asarray(h, dtype=np.float64)
    s2 = np.broadcast_to(np.asarray(sigma2_i, dtype=np.float64), (N,))
    keep = np.isfinite(s2)
    if H is not None:
        S, _ = moments_full(X, None, H, order, gpts)
    elif kernel == "gauss":
        S, _ = moments(X, None, h, order, gpts)
    else:
        S, _ = moments_compact(X, None, h, order, gpts, kernel)
    _, r0, ill = solve(S, np.zeros((len(gpts), 0, len(multi_indices(d, order)))), h, order, d)
    et = np.array(multi_indices(d, order))
    norm = 1.0 / np.prod(h * np.sqrt(2.0 * np.pi))
    out = np.full(len(gpts), np.nan)
    Xk, sk = X[keep], s2[keep]
    chunk = 1 << 20
    for g in range(len(gpts)):
        if ill[g]:
            continue
        acc = 0.0
        for c0 in range(0, len(Xk), chunk):                     # the sum over samples, in pieces
            u = (Xk[c0:c0 + chunk] - gpts[g]) / h               # (x_i - g) / h per dimension
            if H is not None:
                z = Xk[c0:c0 + chunk] - gpts[g]
                K = hnorm * np.exp(-0.5 * np.einsum("ij,jk,ik->i", z, Hi, z))
            elif kernel == "gauss":
                K = norm * np.exp(-0.5 * np.sum(u * u, axis=1))
            else:
                K = np.prod(compact_kernel(kernel, u) / h, axis=1)
            pw = [[np.ones(len(u))] for _ in range(d)]          # powers u_j^a, a <= order
            for j in range(d):
                for a in range(order):
                    pw[j].append(pw[j][-1] * u[:, j])
            row = np.zeros(len(u))
            for b, e in enumerate(et):                          # e_1^T A~^{-1} d~(x_i - g)
                mono = pw[0][e[0]]
                for j in range(1, d):
                    mono = mono * pw[j][e[j]]
                row += r0[g, b] * mono
            w = row * K
            acc += float(np.sum(w * w * sk[c0:c0 + chunk]))
        out[g] = acc
    return out


def fit_variance_binned(X, sigma2_i, h, order, gpts, kernel: str, delta, L) -> np.ndarray:
    """Sigma(g) = r^T Q r (eq. 27) under the binned approximation of a
    compact kernel (eq. 11-13): r = row 0 of the inverse of the equilibrated
    binned moment matrix of K_h, Q_bc the sigma_i^2-weighted binned moment of
    degree b + c of the squared kernel K_h^2 = prod_j (K(z_j / h_j)^2 / h_j)
    / h_j, brought to the same equilibration.  NaN where the fit is
    ill-posed."""
    X = np.asarray(X, dtype=np.float64)
    if X.ndim == 1:
        X = X[:, None]
    N, d = X.shape
    h = np.asarray(h, dtype=np.float64)
    gpts = np.asarray(gpts, dtype=np.float64).reshape(-1, d)
    s2 = np.broadcast_to(np.asarray(sigma2_i, dtype=np.float64), (N,))
    keep = np.isfinite(s2)
    S, _ = moments_binned(X, None, h, order, gpts, kernel, delta, L)
    _, r0, ill = solve(S, np.zeros((len(gpts), 0, len(multi_indices(d, order)))), h, order, d)
    Q, _ = moments_binned(X[keep], None, h, order, gpts, kernel, delta, L, square=True, sw=s2[keep])
    A = assemble(Q, h, order, d)                                # Q_bc / h^{b+c}
    out = np.einsum("gb,gbc,gc->g", r0, A, r0) / np.prod(h)
    out[ill] = np.nan
    return out


def normal_quantile(p: float) -> float:
    """z with Phi(z) = p (the quantile of eq. 28), SciPy's ndtri."""
    from scipy.special import ndtri
    return float(ndtri(p))


def interval(mhat: np.ndarray, Sigma: np.ndarray, alpha: float = 0.05):
    """Pointwise confidence interval of eq. (28): m_hat -/+ z_{1-alpha/2}
    sqrt(Sigma)."""
    z = normal_quantile(1.0 - alpha / 2.0)
    half = z * np.sqrt(np.maximum(Sigma, 0.0))
    return mhat - half, mhat + half
