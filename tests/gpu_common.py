"""Helpers shared by the GPU parity tests (not collected by pytest)."""
import numpy as np
import torch

from oracle import oracle as orc


def rel_err(gpu, ref, mask=None) -> float:
    """max |gpu - ref| / max |ref| over the mask: FFT errors are relative to a
    channel's global magnitude, so the error is measured against it."""
    gpu = np.asarray(gpu)
    ref = np.asarray(ref)
    if mask is not None:
        gpu = gpu[mask]
        ref = ref[mask]
    scale = np.abs(ref).max()
    if scale == 0:
        return float(np.abs(gpu).max())
    return float(np.abs(gpu - ref).max() / scale)


def density_mask(s0: np.ndarray, rho: float = 1e-3) -> np.ndarray:
    return s0 >= rho * s0.max()


U32, U64 = 2.0 ** -24, 2.0 ** -53


def noise_floor(N, h, eps, precision="fp32", tprec="same") -> float:
    """The library's documented absolute pivot floor e N K_h(0), with
    e = max(eps, round-off of the transforms, 30 round-offs of the spreading);
    handed to the oracle so both sides apply the same ill-posedness rule."""
    us = U64 if precision == "fp64" else U32
    tp = precision if tprec == "same" else tprec
    ut = U64 if tp == "fp64" else U32
    k0 = float(np.prod(1.0 / (np.asarray(h, dtype=np.float64) * np.sqrt(2.0 * np.pi))))
    return max(eps, ut, 30.0 * us) * max(N, 1) * k0


def nan_close(gpu, ref, bar, mask=None, scale=None) -> float:
    """NaN positions must agree; returns max |gpu - ref| / scale over the
    finite entries (scale defaults to max |ref| there)."""
    gpu = np.asarray(gpu)
    ref = np.asarray(ref)
    if mask is not None:
        gpu, ref = gpu[mask], ref[mask]
    gn, rn = np.isnan(gpu), np.isnan(ref)
    assert (gn == rn).all(), f"NaN sets differ: gpu {gn.sum()} oracle {rn.sum()} ({(gn != rn).sum()} mismatched)"
    f = ~gn
    if not f.any():
        return 0.0
    sc = np.abs(ref[f]).max() if scale is None else scale
    err = float(np.abs(gpu[f] - ref[f]).max() / sc) if sc > 0 else float(np.abs(gpu[f]).max())
    assert err < bar, err
    return err


def make_plan(d, order, M, h_min, h_max, eps, precision, n_max, max_weights=2, max_h=1,
              kernel="es", lo=None, hi=None, sigma=0.0, tprec="same"):
    from paper_2204_07716_amd import Plan
    lo = lo or (0.0,) * d
    hi = hi or (1.0,) * d
    return Plan(d, order, M, lo, hi, h_min, h_max, eps, precision=precision, kernel=kernel,
                sigma=sigma, n_max=n_max, max_weights=max_weights, max_h=max_h,
                transform_precision=tprec)


def to_dev(a, dtype=torch.float64):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=dtype, device="cuda")


def equilibrate_oracle(S, T, h, order, d):
    """Oracle moments divided by h^a (the library returns equilibrated channels)."""
    es = orc.multi_indices(d, 2 * order)
    et = orc.multi_indices(d, order)
    h = np.asarray(h, dtype=np.float64)
    Se = S / np.array([np.prod(h ** np.array(a)) for a in es])[None, :]
    Te = T / np.array([np.prod(h ** np.array(b)) for b in et])[None, None, :]
    return Se, Te
