"""Seeded synthetic inputs for the five kernel-regression workloads.

This module is shared by the tests, the benchmark and the oracle's checks.
It only draws random numbers and evaluates the test functions that define the
synthetic responses; it holds none of the regression method's arithmetic.

Draws use NumPy's PCG64 generator (``numpy.random.default_rng(seed)``) in the
order listed for each workload, so every consumer sees the same arrays.

Workloads (all on the unit cube, both ends of the grid on the cube's faces):

* ``nw1d``      d=1 Nadaraya-Watson, x ~ U[0,1], y = sin(2 pi x) + 0.3 e,
                N=1e5, h=0.02, M=1024, FP64, eps=1e-9.
* ``ll2d``      d=2 local linear, x from a 4-component Gaussian mixture
                clipped to [0,1]^2, y = sin(4 x1) cos(3 x2) + 0.2 e,
                N=1e6, h=(0.03,0.05), M=256^2, FP32 spread/FFT, FP64 solve.
* ``ll3d``      d=3 local linear plus the log-variance second pass,
                x ~ U[0,1]^3, y = |x|^2 + (0.1 + 0.5 x1) e, N=1e7, h=0.05,
                M=128^3.
* ``batch2d``   d=2 shared-grid DF sweep: the ll2d mixture with N=2e6,
                32 log-spaced bandwidths in [0.01, 0.2], 64 Gaussian probes,
                plus 256 independent regressions with log-uniform N in
                [1e3, 1e6].
* ``cplx2d``    d=2 complex response: 8 Lorentzian peaks with complex
                amplitudes plus complex Gaussian noise at SNR 10,
                N=4e6, M=512^2, local quadratic, h=0.02, 10 probes.
"""
from __future__ import annotations

import dataclasses
from typing import Optional

import numpy as np

__all__ = ["Workload", "make", "NAMES", "mixture_points", "probe_seed"]

NAMES = ("nw1d", "ll2d", "ll3d", "batch2d", "cplx2d")

# Mixture used by ll2d / batch2d.
_MIX_W = np.array([0.35, 0.25, 0.25, 0.15])
_MIX_MU = np.array([[0.25, 0.30], [0.70, 0.25], [0.55, 0.75], [0.20, 0.80]])
_MIX_SD = np.array([0.10, 0.08, 0.12, 0.06])


@dataclasses.dataclass
class Workload:
    name: str
    d: int
    order: int
    X: np.ndarray                 # N x d, float64, row-major
    Y: np.ndarray                 # N x q, float64 or complex128
    h: np.ndarray                 # nh x d bandwidths (kernel std per dimension)
    M: tuple                      # grid points per dimension
    lo: tuple
    hi: tuple
    eps: float
    precision: str                # "fp64" | "fp32" (spread/FFT; solves are FP64)
    n_probes: int = 0
    probe_seed: int = 0
    extra: Optional[dict] = None

    @property
    def N(self) -> int:
        return int(self.X.shape[0])


def probe_seed(name: str) -> int:
    """Seed of the counter-based probe generator for a workload."""
    return {"nw1d": 1001, "ll2d": 1002, "ll3d": 1003, "batch2d": 1004,
            "cplx2d": 1005}[name]


def mixture_points(rng: np.random.Generator, n: int) -> np.ndarray:
    comp = rng.choice(4, size=n, p=_MIX_W)
    z = rng.standard_normal((n, 2))
    x = _MIX_MU[comp] + _MIX_SD[comp, None] * z
    return np.clip(x, 0.0, 1.0)


def _ll2d_response(x: np.ndarray, noise: np.ndarray) -> np.ndarray:
    return np.sin(4.0 * x[:, 0]) * np.cos(3.0 * x[:, 1]) + 0.2 * noise


def make(name: str, N: Optional[int] = None, M: Optional[tuple] = None,
         seed: Optional[int] = None) -> Workload:
    """Build a workload.  ``N`` / ``M`` override the sizes for small test
    variants; the recipe (distributions, draw order) stays the same."""
    if name == "nw1d":
        n = int(N or 100_000)
        rng = np.random.default_rng(1 if seed is None else seed)
        x = rng.random(n)
        e = rng.standard_normal(n)
        y = np.sin(2.0 * np.pi * x) + 0.3 * e
        return Workload(name, 1, 0, x[:, None].copy(), y[:, None].copy(),
                        np.array([[0.02]]), tuple(M or (1024,)), (0.0,), (1.0,),
                        1e-9, "fp64", n_probes=10, probe_seed=probe_seed(name))
    if name == "ll2d":
        n = int(N or 1_000_000)
        rng = np.random.default_rng(2 if seed is None else seed)
        x = mixture_points(rng, n)
        y = _ll2d_response(x, rng.standard_normal(n))
        return Workload(name, 2, 1, x, y[:, None].copy(), np.array([[0.03, 0.05]]),
                        tuple(M or (256, 256)), (0.0, 0.0), (1.0, 1.0), 1e-6,
                        "fp32", n_probes=10, probe_seed=probe_seed(name))
    if name == "ll3d":
        n = int(N or 10_000_000)
        rng = np.random.default_rng(3 if seed is None else seed)
        x = rng.random((n, 3))
        e = rng.standard_normal(n)
        y = (x * x).sum(axis=1) + (0.1 + 0.5 * x[:, 0]) * e
        return Workload(name, 3, 1, x, y[:, None].copy(), np.array([[0.05, 0.05, 0.05]]),
                        tuple(M or (128, 128, 128)), (0.0,) * 3, (1.0,) * 3, 1e-6,
                        "fp32", n_probes=10, probe_seed=probe_seed(name))
    if name == "batch2d":
        n = int(N or 2_000_000)
        rng = np.random.default_rng(4 if seed is None else seed)
        x = mixture_points(rng, n)
        y = _ll2d_response(x, rng.standard_normal(n))
        hs = np.logspace(np.log10(0.01), np.log10(0.2), 32)
        # 256 independent regressions with log-uniform sizes in [1e3, 1e6].
        sizes = np.rint(10.0 ** rng.uniform(3.0, 6.0, 256)).astype(np.int64)
        return Workload(name, 2, 1, x, y[:, None].copy(), np.stack([hs, hs], axis=1),
                        tuple(M or (256, 256)), (0.0, 0.0), (1.0, 1.0), 1e-6, "fp32",
                        n_probes=64, probe_seed=probe_seed(name),
                        extra={"regression_sizes": sizes, "regression_h": 0.05,
                               "regression_seed_base": 40_000})
    if name == "cplx2d":
        n = int(N or 4_000_000)
        rng = np.random.default_rng(5 if seed is None else seed)
        x = rng.random((n, 2))
        c = rng.uniform(0.1, 0.9, (8, 2))
        gam = rng.uniform(0.02, 0.08, 8)
        amp = rng.uniform(0.5, 1.5, 8)
        phi = rng.uniform(0.0, 2.0 * np.pi, 8)
        f = np.zeros(n, dtype=np.complex128)
        for k in range(8):
            r2 = ((x - c[k]) ** 2).sum(axis=1)
            f += amp[k] * np.exp(1j * phi[k]) / (1.0 + r2 / gam[k] ** 2)
        sig2 = np.mean(np.abs(f) ** 2) / 10.0
        noise = rng.standard_normal((n, 2)) * np.sqrt(sig2 / 2.0)
        y = f + noise[:, 0] + 1j * noise[:, 1]
        return Workload(name, 2, 2, x, y[:, None].copy(), np.array([[0.02, 0.02]]),
                        tuple(M or (512, 512)), (0.0, 0.0), (1.0, 1.0), 1e-6, "fp32",
                        n_probes=10, probe_seed=probe_seed(name))
    raise KeyError(name)


def independent_regression(w: Workload, k: int):
    """The k-th of batch2d's independent regressions: (X, Y)."""
    assert w.name == "batch2d"
    n = int(w.extra["regression_sizes"][k])
    rng = np.random.default_rng(w.extra["regression_seed_base"] + k)
    x = rng.random((n, 2))
    y = _ll2d_response(x, rng.standard_normal(n))
    return x, y[:, None].copy()
