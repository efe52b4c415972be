"""Python binding of the fast kernel-regression library (include/fkr.h).

Argument marshalling only: torch supplies device memory and the current HIP
stream; every step of the method runs in the HIP kernels of ``libfkr.so``.
Grid outputs are flat with the index of dimension 0 fastest (shape ``(..., M_tot)``);
``grid_shape`` gives the C-order shape ``(M_{d-1}, ..., M_0)`` to reshape them.
"""
from __future__ import annotations

import ctypes
from typing import Optional, Sequence

import numpy as np
import torch

from . import _lib
from ._lib import check

__all__ = ["Plan", "get_hlist", "select_bandwidth"]


def _dtype_code(t: torch.Tensor) -> int:
    if t.dtype == torch.float64:
        return _lib.FKR_F64
    if t.dtype == torch.float32:
        return _lib.FKR_F32
    raise TypeError(f"unsupported dtype {t.dtype}")


def _stream() -> ctypes.c_void_p:
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _ptr(t: Optional[torch.Tensor]) -> Optional[int]:
    if t is None:
        return None
    if not t.is_cuda:
        raise ValueError("device tensor expected")
    if not t.is_contiguous():
        raise ValueError("contiguous tensor expected")
    return t.data_ptr()


def _real_view(Y: torch.Tensor):
    """(tensor of reals, q, y_complex)."""
    if Y.dim() == 1:
        Y = Y[:, None]
    if Y.is_complex():
        q = Y.shape[1]
        return torch.view_as_real(Y.contiguous()).contiguous(), q, 1
    return Y.contiguous(), Y.shape[1], 0


def _hbuf(h, d: int) -> np.ndarray:
    a = np.ascontiguousarray(np.asarray(h, dtype=np.float64).reshape(-1, d))
    return a


def _hptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def get_hlist(n: int, lo: float, hi: float, kind: str = "log") -> np.ndarray:
    """Bandwidth candidates (Sec. 4 get_hList), both ends included."""
    out = np.zeros(n)
    check(_lib.load().fkr_hlist(n, lo, hi, 0 if kind == "log" else 1, _hptr(out)), "fkr_hlist")
    return out


def select_bandwidth(gcv: Sequence[float], dstd: float = 0.0) -> int:
    """Relaxed GCV selection (Table 1, dstd)."""
    g = np.ascontiguousarray(np.asarray(gcv, dtype=np.float64).ravel())
    idx = ctypes.c_int(-1)
    check(_lib.load().fkr_select_bandwidth(g.size, _hptr(g), float(dstd), ctypes.byref(idx)),
          "fkr_select_bandwidth")
    return idx.value


class GCVLogH(torch.autograd.Function):
    """GCV (eq. 22) of one real response as a function of log h and of the
    response y, with the library's hand-written gradients as its backward:
    ``GCVLogH.apply(log_h, Y, plan, Np, seed)`` with log_h a tensor of d
    entries and Y of N (either may require grad)."""

    @staticmethod
    def forward(ctx, log_h, Y, plan, Np, seed):
        h = torch.exp(log_h.detach().to(torch.float64)).cpu().numpy()
        out = plan.gcv_grad(h, Y.detach(), Np, seed, want_dy=Y.requires_grad)
        dy = out["dy"].to(Y.dtype).reshape(Y.shape) if out["dy"] is not None else None   # complex: dRe + i dIm
        ctx.save_for_backward(out["dlogh"].to(log_h.device, log_h.dtype), dy)
        return out["gcv"][0].to(log_h.device, log_h.dtype)

    @staticmethod
    def backward(ctx, grad_out):
        dl, dy = ctx.saved_tensors
        g_y = grad_out.to(dy.device, dy.dtype) * dy if dy is not None else None
        return grad_out * dl, g_y, None, None, None


class GCVFullH(torch.autograd.Function):
    """GCV (eq. 22) of one real response as a function of a full bandwidth
    matrix H (d x d, symmetric) and of the response y, with the library's
    hand-written gradients as its backward: ``GCVFullH.apply(H, Y, plan, Np,
    seed)`` (either may require grad).  The gradient in H is
    returned as a symmetric matrix G with G_pq = dGCV/dH_pq for H_pq and H_qp
    taken as separate entries (half the symmetric derivative off the
    diagonal), so that a symmetric step dH changes GCV by sum(G * dH)."""

    @staticmethod
    def forward(ctx, H, Y, plan, Np, seed):
        Hn = H.detach().to(torch.float64).cpu().numpy()
        out = plan.gcv_grad_full(Hn, Y.detach(), Np, seed, want_dy=Y.requires_grad)
        dy = out["dy"].to(Y.dtype).reshape(Y.shape) if out["dy"] is not None else None   # complex: dRe + i dIm
        d = Hn.shape[0]
        g = torch.zeros((d, d), dtype=torch.float64)
        k = 0
        dH = out["dH"].cpu()
        for p in range(d):
            for q in range(p, d):
                g[p, q] = dH[k] if p == q else 0.5 * dH[k]
                g[q, p] = g[p, q]
                k += 1
        ctx.save_for_backward(g.to(H.device, H.dtype), dy)
        return out["gcv"][0].to(H.device, H.dtype)

    @staticmethod
    def backward(ctx, grad_out):
        g, dy = ctx.saved_tensors
        g_y = grad_out.to(dy.device, dy.dtype) * dy if dy is not None else None
        return grad_out * g, g_y, None, None, None


def _plan_desc(d, order, M, lo, hi, h_min, h_max, eps, precision, kernel, sigma, n_max, max_weights,
               max_h, transform_precision):
    desc = _lib.PlanDesc()
    desc.d, desc.order = d, order
    for j in range(d):
        desc.M[j] = int(M[j])
        desc.lo[j], desc.hi[j] = float(lo[j]), float(hi[j])
        desc.h_min[j], desc.h_max[j] = float(h_min[j]), float(h_max[j])
    desc.eps = float(eps)
    desc.precision = _lib.FKR_F64 if precision == "fp64" else _lib.FKR_F32
    desc.spread_kernel = _lib.FKR_KERNEL_ES if kernel == "es" else _lib.FKR_KERNEL_GAUSS
    desc.sigma = float(sigma)
    desc.n_max = int(n_max)
    desc.max_weights = int(max_weights)
    desc.max_h = int(max_h)
    desc.transform_precision = {"same": _lib.FKR_TP_SAME, "fp32": _lib.FKR_TP_F32,
                                "fp64": _lib.FKR_TP_F64}[transform_precision]
    return desc


class Batch:
    """Independent regressions of uneven size on one plan geometry, run over
    n_lanes plans and streams (fkr_batch_*)."""

    def __init__(self, d: int, order: int, M: Sequence[int], lo: Sequence[float],
                 hi: Sequence[float], h_min: Sequence[float], h_max: Sequence[float],
                 eps: float, precision: str = "fp32", kernel: str = "es", sigma: float = 0.0,
                 n_max: int = 0, max_weights: int = 2, max_h: int = 1, n_lanes: int = 4,
                 device="cuda", transform_precision: str = "same"):
        self.lib = _lib.load()
        self.desc = _plan_desc(d, order, M, lo, hi, h_min, h_max, eps, precision, kernel, sigma, n_max,
                               max_weights, max_h, transform_precision)
        self.d = d
        self.Mtot = int(np.prod([int(m) for m in M]))
        self._b = ctypes.c_void_p()
        check(self.lib.fkr_batch_create(ctypes.byref(self.desc), int(n_lanes), ctypes.byref(self._b)),
              "fkr_batch_create")
        size = ctypes.c_size_t()
        check(self.lib.fkr_batch_workspace_size(self._b, ctypes.byref(size)), "fkr_batch_workspace_size")
        self.workspace = torch.empty(int(size.value) + 256, dtype=torch.uint8, device=device)
        base = self.workspace.data_ptr()
        check(self.lib.fkr_batch_set_workspace(self._b, ctypes.c_void_p(base + (-base) % 256), size),
              "fkr_batch_set_workspace")
        self.device = self.workspace.device

    def __del__(self):
        try:
            if getattr(self, "_b", None) and self._b.value:
                torch.cuda.synchronize(self.device)   # the lanes' streams may still run
                self.lib.fkr_batch_destroy(self._b)
                self._b = ctypes.c_void_p()
        except Exception:
            pass

    def _args(self, offsets, X, h, Y):
        off = np.ascontiguousarray(offsets, dtype=np.int64)
        X = X.contiguous()
        Yr, q, cplx = _real_view(Y)
        hb = _hbuf(h, self.d)
        self._keep = (off, X, Yr, hb)
        return off, X, Yr, q, cplx, hb

    def cv(self, offsets, X: torch.Tensor, h, Y: torch.Tensor, Np: int, seed: int = 0,
           want_mhat: bool = True) -> dict:
        off, X, Yr, q, cplx, hb = self._args(offsets, X, h, Y)
        R, nh = len(off) - 1, hb.shape[0]
        dev = self.device
        mhat = (torch.empty((R, nh, q, self.Mtot) + ((2,) if cplx else ()), dtype=torch.float64, device=dev)
                if want_mhat else None)
        rho = torch.empty((R, nh, Np), dtype=torch.float64, device=dev)
        rss = torch.empty((R, nh, q), dtype=torch.float64, device=dev)
        gcv = torch.empty((R, nh, q), dtype=torch.float64, device=dev)
        nused = torch.empty((R, nh), dtype=torch.float64, device=dev)
        check(self.lib.fkr_batch_cv(self._b, R, off.ctypes.data_as(ctypes.c_void_p), _ptr(X), _dtype_code(X), nh,
                                    _hptr(hb), q, cplx, _ptr(Yr), _dtype_code(Yr), Np, ctypes.c_uint64(seed),
                                    _ptr(mhat), _ptr(rho), _ptr(rss), _ptr(gcv), _ptr(nused), _stream()),
              "fkr_batch_cv")
        if mhat is not None and cplx:
            mhat = torch.view_as_complex(mhat)
        return {"mhat": mhat, "rho": rho, "rss": rss, "gcv": gcv, "nused": nused}

    def tune(self, offsets, X: torch.Tensor, h, Y: torch.Tensor, Np: int, seed: int = 0, reps: int = 2) -> dict:
        off, X, Yr, q, cplx, hb = self._args(offsets, X, h, Y)
        lanes, chunk, ms = ctypes.c_int(), ctypes.c_int64(), ctypes.c_double()
        check(self.lib.fkr_batch_tune(self._b, len(off) - 1, off.ctypes.data_as(ctypes.c_void_p), _ptr(X),
                                      _dtype_code(X), hb.shape[0], _hptr(hb), q, cplx, _ptr(Yr), _dtype_code(Yr),
                                      Np, ctypes.c_uint64(seed), int(reps), ctypes.byref(lanes),
                                      ctypes.byref(chunk), ctypes.byref(ms), _stream()), "fkr_batch_tune")
        return {"lanes": lanes.value, "chunk": chunk.value, "ms": ms.value}

    def config(self, lanes: int, chunk: int = 0) -> None:
        check(self.lib.fkr_batch_config(self._b, int(lanes), ctypes.c_int64(chunk)), "fkr_batch_config")


class Plan:
    """A plan bound to one device workspace (fkr_plan_create + fkr_set_workspace)."""

    def __init__(self, d: int, order: int, M: Sequence[int], lo: Sequence[float],
                 hi: Sequence[float], h_min: Sequence[float], h_max: Sequence[float],
                 eps: float, precision: str = "fp32", kernel: str = "es", sigma: float = 0.0,
                 n_max: int = 0, max_weights: int = 2, max_h: int = 1, device="cuda",
                 transform_precision: str = "same", reg_kernel: str = "gauss"):
        self.lib = _lib.load()
        desc = _lib.PlanDesc()
        desc.reg_kernel = _lib.FKR_REG[reg_kernel]
        desc.d, desc.order = d, order
        for j in range(d):
            desc.M[j] = int(M[j])
            desc.lo[j], desc.hi[j] = float(lo[j]), float(hi[j])
            desc.h_min[j], desc.h_max[j] = float(h_min[j]), float(h_max[j])
        desc.eps = float(eps)
        desc.precision = _lib.FKR_F64 if precision == "fp64" else _lib.FKR_F32
        desc.spread_kernel = _lib.FKR_KERNEL_ES if kernel == "es" else _lib.FKR_KERNEL_GAUSS
        desc.sigma = float(sigma)
        desc.n_max = int(n_max)
        desc.max_weights = int(max_weights)
        desc.max_h = int(max_h)
        desc.transform_precision = {"same": _lib.FKR_TP_SAME, "fp32": _lib.FKR_TP_F32,
                                    "fp64": _lib.FKR_TP_F64}[transform_precision]
        self.desc = desc
        self.d, self.order = d, order
        self.M = tuple(int(m) for m in M)
        self.Mtot = int(np.prod(self.M))
        self.grid_shape = tuple(reversed(self.M))
        self._plan = ctypes.c_void_p()
        check(self.lib.fkr_plan_create(ctypes.byref(desc), ctypes.byref(self._plan)), "fkr_plan_create")
        g = _lib.Geometry()
        check(self.lib.fkr_plan_geometry(self._plan, ctypes.byref(g)), "fkr_plan_geometry")
        self.geometry = g
        self.n_s, self.n_t = g.n_s, g.n_t
        self.workspace = torch.empty(int(g.workspace_bytes) + 256, dtype=torch.uint8, device=device)
        base = self.workspace.data_ptr()
        off = (-base) % 256
        self._ws_ptr = base + off
        check(self.lib.fkr_set_workspace(self._plan, ctypes.c_void_p(self._ws_ptr),
                                         ctypes.c_size_t(int(g.workspace_bytes))), "fkr_set_workspace")
        self.device = self.workspace.device
        self.N = None

    def __del__(self):
        try:
            if getattr(self, "_plan", None) and self._plan.value:
                self.lib.fkr_plan_destroy(self._plan)
                self._plan = ctypes.c_void_p()
        except Exception:
            pass

    @property
    def band(self):
        return tuple(2 * self.geometry.K[j] + 1 for j in range(self.d))

    # -- a2 -------------------------------------------------------------
    def set_points(self, X: torch.Tensor) -> None:
        X = X.contiguous()
        if X.dim() == 1:
            X = X[:, None]
        assert X.shape[1] == self.d
        self._X = X  # keep alive for the async kernels
        check(self.lib.fkr_set_points(self._plan, X.shape[0], _ptr(X), _dtype_code(X), _stream()),
              "fkr_set_points")
        self.N = X.shape[0]

    # -- a3-a5 ----------------------------------------------------------
    def spectrum(self, W: Optional[torch.Tensor] = None) -> torch.Tensor:
        nw = 1 if W is None else (W.shape[1] if W.dim() == 2 else 1)
        if W is not None:
            W = W.reshape(W.shape[0], nw).contiguous()
        out = torch.empty((nw,) + tuple(reversed(self.band)) + (2,), dtype=torch.float64,
                          device=self.device)
        check(self.lib.fkr_spectrum(self._plan, nw, _ptr(W), _dtype_code(W) if W is not None else 1,
                                    _ptr(out), _stream()), "fkr_spectrum")
        return torch.view_as_complex(out)

    # -- a3-a6 ----------------------------------------------------------
    def moments(self, h, W: Optional[torch.Tensor] = None):
        hb = _hbuf(h, self.d)
        nh = hb.shape[0]
        nw = 0 if W is None else (W.shape[1] if W.dim() == 2 else 1)
        if W is not None:
            W = W.reshape(W.shape[0], nw).contiguous()
        S = torch.empty((nh, self.n_s, self.Mtot), dtype=torch.float64, device=self.device)
        T = torch.empty((nh, max(nw, 1), self.n_t, self.Mtot), dtype=torch.float64, device=self.device)
        check(self.lib.fkr_moments(self._plan, nh, _hptr(hb), nw, _ptr(W),
                                   _dtype_code(W) if W is not None else 1, _ptr(S),
                                   _ptr(T) if nw else None, _stream()), "fkr_moments")
        return S, (T if nw else None)

    # -- a3-a7 ----------------------------------------------------------
    def fit(self, h, Y: torch.Tensor, want_s0: bool = False):
        hb = _hbuf(h, self.d)
        nh = hb.shape[0]
        Yr, q, cplx = _real_view(Y)
        shape = (nh, q, self.Mtot) + ((2,) if cplx else ())
        mhat = torch.empty(shape, dtype=torch.float64, device=self.device)
        s0 = torch.empty((nh, self.Mtot), dtype=torch.float64, device=self.device) if want_s0 else None
        check(self.lib.fkr_fit(self._plan, nh, _hptr(hb), q, cplx, _ptr(Yr), _dtype_code(Yr),
                               _ptr(mhat), _ptr(s0), _stream()), "fkr_fit")
        if cplx:
            mhat = torch.view_as_complex(mhat)
        return (mhat, s0) if want_s0 else mhat

    # -- a8 -------------------------------------------------------------
    def interp(self, G: torch.Tensor, Xq: torch.Tensor) -> torch.Tensor:
        G = G.reshape(-1, self.Mtot).contiguous()
        Xq = Xq.contiguous()
        if Xq.dim() == 1:
            Xq = Xq[:, None]
        out = torch.empty((G.shape[0], Xq.shape[0]), dtype=torch.float64, device=self.device)
        check(self.lib.fkr_interp(self._plan, G.shape[0], _ptr(G), Xq.shape[0], _ptr(Xq),
                                  _dtype_code(Xq), _ptr(out), _stream()), "fkr_interp")
        return out

    # -- a9 -------------------------------------------------------------
    def dof(self, h, Np: int, seed: int = 0, probes: Optional[torch.Tensor] = None,
            want_nused: bool = False):
        """Girard ratios [nh][Np] over the supported samples (and N_I [nh])."""
        hb = _hbuf(h, self.d)
        nh = hb.shape[0]
        rho = torch.empty((nh, Np), dtype=torch.float64, device=self.device)
        nused = torch.empty(nh, dtype=torch.float64, device=self.device)
        if probes is not None:
            probes = probes.contiguous()
        check(self.lib.fkr_dof(self._plan, nh, _hptr(hb), Np, ctypes.c_uint64(seed), _ptr(probes),
                               _dtype_code(probes) if probes is not None else 1, _ptr(rho), _ptr(nused),
                               _stream()), "fkr_dof")
        return (rho, nused) if want_nused else rho

    # -- a10 ------------------------------------------------------------
    def gcv(self, h, Y: torch.Tensor, rho: torch.Tensor, want_mhat: bool = False):
        """GCV (eq. 22) of responses Y against Girard ratios from dof()."""
        hb = _hbuf(h, self.d)
        nh = hb.shape[0]
        Yr, q, cplx = _real_view(Y)
        rho = rho.to(torch.float64).contiguous()
        Np = rho.shape[-1]
        mhat = (torch.empty((nh, q, self.Mtot) + ((2,) if cplx else ()), dtype=torch.float64,
                            device=self.device) if want_mhat else None)
        rss = torch.empty((nh, q), dtype=torch.float64, device=self.device)
        gcv = torch.empty((nh, q), dtype=torch.float64, device=self.device)
        nused = torch.empty(nh, dtype=torch.float64, device=self.device)
        check(self.lib.fkr_gcv(self._plan, nh, _hptr(hb), q, cplx, _ptr(Yr), _dtype_code(Yr), Np, _ptr(rho),
                               _ptr(mhat), _ptr(rss), _ptr(gcv), _ptr(nused), _stream()), "fkr_gcv")
        if mhat is not None and cplx:
            mhat = torch.view_as_complex(mhat)
        return {"mhat": mhat, "rss": rss, "gcv": gcv, "nused": nused}

    # -- a7-a10 batched -------------------------------------------------
    def cv(self, h, Y: torch.Tensor, Np: int, seed: int = 0,
           probes: Optional[torch.Tensor] = None, want_mhat: bool = True):
        hb = _hbuf(h, self.d)
        nh = hb.shape[0]
        Yr, q, cplx = _real_view(Y)
        if probes is not None:
            probes = probes.to(Yr.dtype).contiguous()
        mhat = (torch.empty((nh, q, self.Mtot) + ((2,) if cplx else ()), dtype=torch.float64,
                            device=self.device) if want_mhat else None)
        rho = torch.empty((nh, Np), dtype=torch.float64, device=self.device) if Np else None
        rss = torch.empty((nh, q), dtype=torch.float64, device=self.device)
        gcv = torch.empty((nh, q), dtype=torch.float64, device=self.device) if Np else None
        nused = torch.empty(nh, dtype=torch.float64, device=self.device)
        check(self.lib.fkr_cv(self._plan, nh, _hptr(hb), q, cplx, _ptr(Yr), _dtype_code(Yr), Np,
                              ctypes.c_uint64(seed), _ptr(probes), _ptr(mhat), _ptr(rho), _ptr(rss),
                              _ptr(gcv), _ptr(nused), _stream()), "fkr_cv")
        if mhat is not None and cplx:
            mhat = torch.view_as_complex(mhat)
        return {"mhat": mhat, "rho": rho, "rss": rss, "gcv": gcv, "nused": nused}

    # -- a11 ------------------------------------------------------------
    def variance(self, h, Y: torch.Tensor, mhat: torch.Tensor, mode: str = "log", H=None):
        """The second pass (Sec. 3) at h, or with H (d x d) at that full bandwidth matrix."""
        if H is not None:
            hb = np.ascontiguousarray(np.asarray(H, dtype=np.float64).reshape(self.d, self.d))
        else:
            hb = _hbuf(h, self.d)
        Yr, q, cplx = _real_view(Y)
        assert q == 1, "one response column"
        m = torch.view_as_real(mhat).contiguous() if mhat.is_complex() else mhat.contiguous()
        sigma2 = torch.empty(self.Mtot, dtype=torch.float64, device=self.device)
        vhat = torch.empty(self.Mtot, dtype=torch.float64, device=self.device)
        kappa = torch.empty(1, dtype=torch.float64, device=self.device)
        md = _lib.FKR_VAR_LOG if mode == "log" else _lib.FKR_VAR_DIRECT
        fn = self.lib.fkr_variance_full if H is not None else self.lib.fkr_variance
        check(fn(self._plan, _hptr(hb), cplx, _ptr(Yr), _dtype_code(Yr), _ptr(m), md, _ptr(sigma2), _ptr(vhat),
                 _ptr(kappa), _stream()), "fkr_variance_full" if H is not None else "fkr_variance")
        return sigma2, (vhat if mode == "log" else None), (kappa if mode == "log" else None)

    # -- full bandwidth matrices ----------------------------------------
    def fit_full(self, H, Y: torch.Tensor, want_s0: bool = False):
        """Fits with full bandwidth matrices H ([nh] x d x d)."""
        Hb = np.ascontiguousarray(np.asarray(H, dtype=np.float64).reshape(-1, self.d, self.d))
        nh = Hb.shape[0]
        Yr, q, cplx = _real_view(Y)
        mhat = torch.empty((nh, q, self.Mtot) + ((2,) if cplx else ()), dtype=torch.float64, device=self.device)
        s0 = torch.empty((nh, self.Mtot), dtype=torch.float64, device=self.device) if want_s0 else None
        check(self.lib.fkr_fit_full(self._plan, nh, Hb.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), q, cplx,
                                    _ptr(Yr), _dtype_code(Yr), _ptr(mhat), _ptr(s0), _stream()), "fkr_fit_full")
        if cplx:
            mhat = torch.view_as_complex(mhat)
        return (mhat, s0) if want_s0 else mhat

    def cv_full(self, H, Y: torch.Tensor, Np: int, seed: int = 0,
                probes: Optional[torch.Tensor] = None, want_mhat: bool = True):
        """fkr_cv over full bandwidth matrices H ([nh] x d x d): fits, DF, RSS, GCV."""
        Hb = np.ascontiguousarray(np.asarray(H, dtype=np.float64).reshape(-1, self.d, self.d))
        nh = Hb.shape[0]
        Yr, q, cplx = _real_view(Y)
        if probes is not None:
            probes = probes.to(Yr.dtype).contiguous()
        mhat = (torch.empty((nh, q, self.Mtot) + ((2,) if cplx else ()), dtype=torch.float64,
                            device=self.device) if want_mhat else None)
        rho = torch.empty((nh, Np), dtype=torch.float64, device=self.device) if Np else None
        rss = torch.empty((nh, q), dtype=torch.float64, device=self.device)
        gcv = torch.empty((nh, q), dtype=torch.float64, device=self.device) if Np else None
        nused = torch.empty(nh, dtype=torch.float64, device=self.device)
        check(self.lib.fkr_cv_full(self._plan, nh, Hb.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), q, cplx,
                                   _ptr(Yr), _dtype_code(Yr), Np, ctypes.c_uint64(seed), _ptr(probes),
                                   _ptr(mhat), _ptr(rho), _ptr(rss), _ptr(gcv), _ptr(nused), _stream()),
              "fkr_cv_full")
        if mhat is not None and cplx:
            mhat = torch.view_as_complex(mhat)
        return {"mhat": mhat, "rho": rho, "rss": rss, "gcv": gcv, "nused": nused}

    def moments_full(self, H, W: Optional[torch.Tensor] = None):
        Hb = np.ascontiguousarray(np.asarray(H, dtype=np.float64).reshape(-1, self.d, self.d))
        nh = Hb.shape[0]
        nw = 0 if W is None else (W.shape[1] if W.dim() > 1 else 1)
        if W is not None:
            W = W.reshape(W.shape[0], -1).contiguous()
        S = torch.empty((nh, self.n_s, self.Mtot), dtype=torch.float64, device=self.device)
        T = torch.empty((nh, nw, self.n_t, self.Mtot), dtype=torch.float64, device=self.device) if nw else None
        check(self.lib.fkr_moments_full(self._plan, nh, Hb.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), nw,
                                        _ptr(W), _dtype_code(W) if W is not None else 1, _ptr(S), _ptr(T),
                                        _stream()), "fkr_moments_full")
        return S, T

    # -- differentiation ------------------------------------------------
    def gcv_grad(self, h, Y: torch.Tensor, Np: int, seed: int = 0, want_dy: bool = True) -> dict:
        """GCV at h for one real response with Np Philox probes, its gradients
        in log h [d] and in y [N], and d m_hat / d log h_j of y and the probes
        [d][1+Np][M]."""
        hb = _hbuf(h, self.d)
        assert hb.shape[0] == 1, "one bandwidth"
        Yr, q, cplx = _real_view(Y.reshape(-1, 1))
        assert q == 1, "one response column"
        ny = 2 if cplx else 1
        N = Yr.shape[0]
        gcv = torch.empty(1, dtype=torch.float64, device=self.device)
        dlogh = torch.empty(self.d, dtype=torch.float64, device=self.device)
        dfit = torch.empty((self.d, ny + Np, self.Mtot), dtype=torch.float64, device=self.device)
        dy = torch.empty((N, ny), dtype=torch.float64, device=self.device) if want_dy else None
        check(self.lib.fkr_gcv_grad(self._plan, _hptr(hb), cplx, _ptr(Yr), _dtype_code(Yr), Np,
                                    ctypes.c_uint64(seed), _ptr(gcv), _ptr(dlogh), _ptr(dy), _ptr(dfit), _stream()),
              "fkr_gcv_grad")
        if dy is not None:
            dy = torch.view_as_complex(dy) if cplx else dy[:, 0]
        return {"gcv": gcv, "dlogh": dlogh, "dy": dy, "dfit": dfit}

    def gcv_grad_full(self, H, Y: torch.Tensor, Np: int, seed: int = 0, want_dy: bool = True) -> dict:
        """GCV at the full bandwidth matrix H (d x d) for one response with Np
        Philox probes, its gradients in the upper-triangle entries H_pq (p <= q,
        row-major) and in y [N], and d m_hat / d H_pq of y and the probes."""
        Hb = np.ascontiguousarray(np.asarray(H, dtype=np.float64).reshape(self.d, self.d))
        Yr, q, cplx = _real_view(Y.reshape(-1, 1))
        assert q == 1, "one response column"
        ny = 2 if cplx else 1
        nd = self.d * (self.d + 1) // 2
        gcv = torch.empty(1, dtype=torch.float64, device=self.device)
        dH = torch.empty(nd, dtype=torch.float64, device=self.device)
        dfit = torch.empty((nd, ny + Np, self.Mtot), dtype=torch.float64, device=self.device)
        dy = torch.empty((Yr.shape[0], ny), dtype=torch.float64, device=self.device) if want_dy else None
        check(self.lib.fkr_gcv_grad_full(self._plan, _hptr(Hb), cplx, _ptr(Yr), _dtype_code(Yr), Np,
                                         ctypes.c_uint64(seed), _ptr(gcv), _ptr(dH), _ptr(dy), _ptr(dfit),
                                         _stream()),
              "fkr_gcv_grad_full")
        if dy is not None:
            dy = torch.view_as_complex(dy) if cplx else dy[:, 0]
        return {"gcv": gcv, "dH": dH, "dy": dy, "dfit": dfit}

    # -- prediction and inference ---------------------------------------
    def interval(self, h, sigma2, mhat: Optional[torch.Tensor] = None, alpha: float = 0.05, H=None):
        """Variance of the fit Sigma [M] (eq. 27) for error variance sigma2 (a
        number, or a grid [M] interpolated to the samples), and with mhat the
        band mhat -/+ z_{1-alpha/2} sqrt(Sigma) (eq. 28).  With H (d x d) the
        full bandwidth matrix H in place of h."""
        if H is not None:
            hb = np.ascontiguousarray(np.asarray(H, dtype=np.float64).reshape(self.d, self.d))
        else:
            hb = _hbuf(h, self.d)
        Sigma = torch.empty(self.Mtot, dtype=torch.float64, device=self.device)
        band = mhat is not None
        lower = torch.empty_like(Sigma) if band else None
        upper = torch.empty_like(Sigma) if band else None
        m = mhat.reshape(self.Mtot).to(torch.float64).contiguous() if band else None
        if isinstance(sigma2, torch.Tensor):
            g = sigma2.reshape(self.Mtot).to(torch.float64).contiguous()
            kind, val = _lib.FKR_SIG_GRID, 0.0
        else:
            g, kind, val = None, _lib.FKR_SIG_SCALAR, float(sigma2)
        fn = self.lib.fkr_interval_full if H is not None else self.lib.fkr_interval
        check(fn(self._plan, _hptr(hb), kind, val, _ptr(g), _ptr(m), float(alpha), _ptr(Sigma), _ptr(lower),
                 _ptr(upper), _stream()), "fkr_interval_full" if H is not None else "fkr_interval")
        return {"Sigma": Sigma, "lower": lower, "upper": upper}

    def spline(self, G: torch.Tensor) -> torch.Tensor:
        """Spline coefficient blocks [nv][2^d][M] of grid functions G ([nv][M])."""
        G = G.reshape(-1, self.Mtot).to(torch.float64).contiguous()
        coef = torch.empty((G.shape[0], 1 << self.d, self.Mtot), dtype=torch.float64, device=self.device)
        check(self.lib.fkr_spline(self._plan, G.shape[0], _ptr(G), _ptr(coef), _stream()), "fkr_spline")
        return coef

    def predict(self, coef: torch.Tensor, Xq: torch.Tensor) -> torch.Tensor:
        """Spline values [nv][Nq] at the points Xq from fkr_spline's coefficients."""
        Xq = Xq.contiguous()
        if Xq.dim() == 1:
            Xq = Xq[:, None]
        nv = coef.shape[0]
        out = torch.empty((nv, Xq.shape[0]), dtype=torch.float64, device=self.device)
        check(self.lib.fkr_predict(self._plan, nv, _ptr(coef), Xq.shape[0], _ptr(Xq), _dtype_code(Xq),
                                   _ptr(out), _stream()), "fkr_predict")
        return out

    # -- stage timing ---------------------------------------------------
    def profile(self, on: bool = True) -> None:
        check(self.lib.fkr_profile_enable(self._plan, 1 if on else 0), "fkr_profile_enable")

    def profile_read(self) -> dict:
        """{stage: (device ms, launches)} since the previous read."""
        out = {}
        for k, name in enumerate(_lib.STAGES):
            ms = ctypes.c_double()
            n = ctypes.c_int64()
            check(self.lib.fkr_profile_read(self._plan, k, ctypes.byref(ms), ctypes.byref(n)),
                  "fkr_profile_read")
            out[name] = (ms.value, n.value)
        return out

    def diagnostics(self, allow_warn: bool = True) -> dict:
        dg = _lib.Diag()
        st = self.lib.fkr_get_diagnostics(self._plan, ctypes.byref(dg))
        return {"status": st, "n_points": dg.n_points, "out_of_domain": dg.out_of_domain,
                "ill_posed": dg.ill_posed, "n_jobs": dg.n_jobs, "max_tile_count": dg.max_tile_count}
