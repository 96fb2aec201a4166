"""Argument validation at the C ABI (include/rbfib.h), forced from the host.

Orientations must be unit quaternions (Sec. II): every entry point that takes
theta checks | |theta_p| - 1 | <= 1e-12 on the device and returns RBFIB_EINVAL
otherwise (also for a non-finite theta), leaving q and theta untouched; a
quaternion within the bound is accepted.  No kernel is given out-of-range data:
the check runs in the marker kernel, which reads only in-bounds entries.
"""
import numpy as np
import pytest

import workloads as W
from tests.helpers import dev, lib_context

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def rb():
    import paper_1901_06427_amd as rb
    return rb


def _code(fn):
    import paper_1901_06427_amd as rb
    try:
        fn()
    except rb.RBFIBError as e:
        return e.code
    return rb.RBFIB_OK


@pytest.mark.parametrize("scale,ok", [(1.0 + 1e-9, False), (1.0 - 3e-12, False), (float("nan"), False),
                                      (1.0 + 2e-14, True)])
def test_non_unit_quaternion(rb, scale, ok):
    import torch
    w = W.small_box(6, n=(12, 12, 12), n_bodies=2, R=1.5, shape="ico12")
    ctx = lib_context(rb, w, tol=1e-8)
    th0 = w.theta.copy()
    th0[1] *= scale
    q, th = dev(w.q), dev(th0)
    FT = dev(w.FT)
    U = torch.empty((w.nb, 6), dtype=torch.float64, device="cuda")
    x = torch.zeros(ctx.L, dtype=torch.float64, device="cuda")
    y = torch.empty_like(x)
    r = torch.empty((w.nm, 3), dtype=torch.float64, device="cuda")
    dF = torch.empty_like(U)
    dq = torch.empty((w.nb, 3), dtype=torch.float64, device="cuda")
    dphi = torch.empty_like(dq)
    calls = {
        "markers": lambda: rb.rbfib_markers(ctx, q, th, r),
        "apply_saddle": lambda: rb.rbfib_apply_saddle(ctx, q, th, x, y),
        "precondition": lambda: rb.rbfib_precondition(ctx, q, th, x, y),
        "solve_mobility": lambda: rb.rbfib_solve_mobility(ctx, q, th, FT, U, allow=()),
        "sem_step": lambda: rb.rbfib_sem_step(ctx, q, th, FT, 1.0, 0.01, 1, 0, U, allow=()),
        "mobility_vjp": lambda: rb.rbfib_mobility_vjp(ctx, q, th, FT, U, dF, dq, dphi, allow=()),
    }
    for name, fn in calls.items():
        print("quaternion scale", scale, name, flush=True)
        code = _code(fn)
        assert code == (rb.RBFIB_OK if ok else rb.RBFIB_EINVAL), (name, code)
        if not ok:
            th_now = th.cpu().numpy()
            assert np.array_equal(q.cpu().numpy(), w.q)
            assert np.array_equal(th_now, th0) or (np.isnan(scale) and np.isnan(th_now[1]).all())
    ctx.close()
