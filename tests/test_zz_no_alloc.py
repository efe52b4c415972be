"""fkr_fit_noalloc (the entry point that allocates nothing): through the C
ABI, two calls in a row on one plan bound to the library's own workspace,
the second with fewer samples and another response, each against fkr_fit on
a plan with a caller-owned workspace and against the oracle."""
import ctypes

import numpy as np
import pytest

from gpu_common import compare_fit, make_plan, to_dev

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _raw_plan(lib, _lib, d, order, M, h, eps, n_max, max_weights):
    desc = _lib.PlanDesc()
    desc.d, desc.order = d, order
    for j in range(d):
        desc.M[j] = M[j]
        desc.lo[j], desc.hi[j] = 0.0, 1.0
        desc.h_min[j] = desc.h_max[j] = h[j]
    desc.eps = eps
    desc.precision = _lib.FKR_F32
    desc.spread_kernel = _lib.FKR_KERNEL_ES
    desc.n_max = n_max
    desc.max_weights = max_weights
    desc.max_h = 1
    desc.transform_precision = _lib.FKR_TP_F64
    plan = ctypes.c_void_p()
    assert lib.fkr_plan_create(ctypes.byref(desc), ctypes.byref(plan)) == 0
    size = ctypes.c_size_t()
    assert lib.fkr_workspace_size(plan, ctypes.byref(size)) == 0
    assert size.value <= _lib.FKR_STATIC_WORKSPACE_BYTES
    return plan


def test_fit_noalloc_matches_fit(orc):
    from paper_2204_07716_amd import _lib
    lib = _lib.load()
    rng = np.random.default_rng(90)
    M, h, eps, d = (48, 40), (0.07, 0.08), 1e-6, 2
    n1, n2 = 30000, 11000
    plan = _raw_plan(lib, _lib, d, 1, M, h, eps, n1, 2)
    ref_plan = make_plan(d, 1, M, h, h, eps, "fp32", n_max=n1, max_weights=2, tprec="fp64")
    hb = np.ascontiguousarray(np.array(h, dtype=np.float64))
    hp = hb.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    stream = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    gp = orc.grid_points(M, (0, 0), (1, 1))
    try:
        for call, N in enumerate((n1, n2)):
            X = rng.random((N, d))
            y = np.sin(3 * X[:, 0] + call) * np.cos(2 * X[:, 1]) + 0.2 * rng.standard_normal(N)
            Xd, Yd = to_dev(X, torch.float32), to_dev(y[:, None], torch.float32)
            mh = torch.full((M[0] * M[1],), 7.0, dtype=torch.float64, device="cuda")
            st = lib.fkr_fit_noalloc(plan, N, ctypes.c_void_p(Xd.data_ptr()), _lib.FKR_F32, 1, hp, 1, 0,
                                     ctypes.c_void_p(Yd.data_ptr()), _lib.FKR_F32,
                                     ctypes.c_void_p(mh.data_ptr()), None, stream)
            assert st == 0, st
            dg = _lib.Diag()
            assert lib.fkr_get_diagnostics(plan, ctypes.byref(dg)) == 0 and dg.n_points == N
            ref_plan.set_points(Xd)
            mh_ref = ref_plan.fit(h, Yd)[0, 0]
            got, want = mh.cpu().numpy(), mh_ref.cpu().numpy()
            X32 = X.astype(np.float32).astype(np.float64)
            oref, S, T, r0, ill = orc.fit(X32, y.astype(np.float32).astype(np.float64), h, 1, gp,
                                          return_all=True)
            # same kernels, same inputs: equal up to the summation order of the LDS adds
            assert np.array_equal(np.isnan(got), np.isnan(want))
            fin = np.isfinite(want)
            assert np.abs(got[fin] - want[fin]).max() <= 1e-6 * np.abs(want[fin]).max()
            compare_fit(got, oref[:, 0], S, h, 1, d, 1e-5)
    finally:
        torch.cuda.synchronize()
        lib.fkr_plan_destroy(plan)


def test_fit_noalloc_rejects_a_plan_larger_than_its_array():
    from paper_2204_07716_amd import _lib
    lib = _lib.load()
    desc = _lib.PlanDesc()
    desc.d, desc.order = 2, 1
    for j in range(2):
        desc.M[j] = 256
        desc.lo[j], desc.hi[j] = 0.0, 1.0
        desc.h_min[j] = desc.h_max[j] = 0.03
    desc.eps, desc.precision, desc.n_max, desc.max_weights, desc.max_h = 1e-6, _lib.FKR_F32, 4_000_000, 2, 1
    desc.transform_precision = _lib.FKR_TP_F64
    plan = ctypes.c_void_p()
    assert lib.fkr_plan_create(ctypes.byref(desc), ctypes.byref(plan)) == 0
    size = ctypes.c_size_t()
    lib.fkr_workspace_size(plan, ctypes.byref(size))
    assert size.value > _lib.FKR_STATIC_WORKSPACE_BYTES
    h = np.array([0.03, 0.03])
    st = lib.fkr_fit_noalloc(plan, 10, None, _lib.FKR_F32, 1, h.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                             1, 0, None, _lib.FKR_F32, None, None, None)
    assert st == _lib.FKR_E_WORKSPACE
    lib.fkr_plan_destroy(plan)
