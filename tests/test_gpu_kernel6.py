"""The paper's 6-point delta kernel (Sec. III.B; rbfib_opts.kernel = 6) on the GPU,
through the C ABI, against the oracle (whose 6-point kernel is built from its
defining conditions, not from the GPU's closed form):

* the saddle apply, every block within 1e-10, on walled, ragged, periodic (a
  one-cell last tile, a body across the wrap), sliding-wall and crowded boxes;
* mobility solves with the FP32 preconditioner, within the bound their
  residuals imply (oracle gains for these configurations);
* one SEM step, within its residual bound;
* the vector-Jacobian product, whose position gradient uses the kernel's
  derivative, within 1e-7 of the oracle's adjoint gradient.
"""
import numpy as np
import pytest

import workloads as W
from oracle import adjoint as oadj
from oracle import sem
from oracle.saddle import Saddle
from tests.helpers import (dev, error_gains, lib_context, oracle_grid, oracle_to_padded, padded_to_oracle,
                           sem_error_bound)
from tests.parity_configs import kernel6_configs

pytestmark = pytest.mark.gpu

CONFIGS = kernel6_configs()


@pytest.fixture(scope="module")
def rb():
    import paper_1901_06427_amd as rb
    return rb


def _rel(a, b):
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))


@pytest.mark.parametrize("name", list(CONFIGS))
def test_apply_saddle_kernel6(rb, name):
    import torch
    w = CONFIGS[name]
    print("apply 6-point", name, flush=True)
    ctx = lib_context(rb, w)
    s = Saddle(oracle_grid(w), w.q, w.theta, w.r_ref, w.offsets)
    x = np.random.default_rng(5).standard_normal(s.n)
    yd = torch.full((ctx.L,), float("nan"), dtype=torch.float64, device="cuda")
    rb.rbfib_apply_saddle(ctx, dev(w.q), dev(w.theta), dev(oracle_to_padded(s, x)), yd)
    torch.cuda.synchronize()
    y, yr = padded_to_oracle(s, yd.cpu().numpy()), s.A @ x
    for sl in (s.sl_v, s.sl_p, s.sl_l, s.sl_u):
        if sl.stop > sl.start:
            assert _rel(y[sl], yr[sl]) < 1e-10, (name, sl)
    ctx.close()


@pytest.mark.parametrize("name", ["ragged_10x12x14_k6", "periodic_wrap_17x12x12_k6", "ensemble16_4spheres_k6",
                                  "two_spheres_16x16x32_k6"])
def test_solve_mobility_kernel6(rb, name):
    import torch
    w = CONFIGS[name]
    tol = 1e-8
    print("solve 6-point", name, flush=True)
    ctx = lib_context(rb, w, tol=tol, precond_fp32=1, max_iter=600)
    s = Saddle(oracle_grid(w), w.q, w.theta, w.r_ref, w.offsets)
    b = s.rhs(FT=w.FT)
    U = torch.empty((w.nb, 6), dtype=torch.float64, device="cuda")
    xo = torch.empty(ctx.L, dtype=torch.float64, device="cuda")
    info = rb.rbfib_solve_mobility(ctx, dev(w.q), dev(w.theta), dev(w.FT), U, x_out=xo, allow=())
    res = s.residual(padded_to_oracle(s, xo.cpu().numpy()), b)
    x_ref, _ = s.solve_fgmres(b, tol=1e-12)
    U_ref = s.split(x_ref)[3]
    bound = error_gains(name).reshape(-1, 6) * (res + s.residual(x_ref, b)) * np.linalg.norm(b)
    err = np.abs(U.cpu().numpy() - U_ref)
    print("  iters %d residual %.2e U rel err %.3e (max err / bound %.3f)"
          % (info[0].iters, res, _rel(U.cpu().numpy(), U_ref), (err / bound).max()), flush=True)
    assert res <= 1.05 * tol
    assert np.all(err <= bound * (1 + 1e-6) + 1e-15)
    ctx.close()


def test_sem_step_kernel6(rb):
    import torch
    name = "two_spheres_16x16x32_k6"
    w = CONFIGS[name]
    tol = 1e-10
    print("sem 6-point", name, flush=True)
    ctx = lib_context(rb, w, tol=tol, precond_fp32=1, max_iter=800)
    q, th = dev(w.q), dev(w.theta)
    U = torch.empty((w.nb, 6), dtype=torch.float64, device="cuda")
    info = rb.rbfib_sem_step(ctx, q, th, dev(w.FT), 1.0, 0.01, 11, 2, U, allow=())
    ref = sem.sem_step(oracle_grid(w), w.r_ref, w.offsets, w.q, w.theta, w.FT, 1.0, 0.01, 11, 2)
    assert ref.accepted
    err = np.abs(U.cpu().numpy() - ref.U)
    bound = sem_error_bound(name, ref.rhs_norms, tol, info[0].rel_residual)
    print("  iters %d U rel err %.3e (max err / bound %.3f)" % (info[0].iters, _rel(U.cpu().numpy(), ref.U),
                                                              (err / bound).max()), flush=True)
    assert np.all(err <= bound)
    ctx.close()


def test_vjp_kernel6(rb):
    import torch
    w = W.small_box(4, n=(10, 10, 12), n_bodies=2, R=1.5, shape="ico12")
    w.kernel = 6
    print("vjp 6-point", flush=True)
    ctx = lib_context(rb, w, tol=1e-12, max_iter=2000)
    q, th, FT = dev(w.q), dev(w.theta), dev(w.FT)
    U = torch.empty((w.nb, 6), dtype=torch.float64, device="cuda")
    rb.rbfib_solve_mobility(ctx, q, th, FT, U, include_bc=False, allow=())
    dF = torch.empty_like(U)
    dq = torch.empty((w.nb, 3), dtype=torch.float64, device="cuda")
    dphi = torch.empty_like(dq)
    rb.rbfib_mobility_vjp(ctx, q, th, FT, (2 * U).contiguous(), dF, dq, dphi, allow=())
    g = oracle_grid(w)
    s, x = oadj.solve_U(g, w.r_ref, w.offsets, w.q, w.theta, w.FT)
    rF, rq, rphi = oadj.mobility_vjp(g, w.r_ref, w.offsets, w.q, w.theta, w.FT, 2 * s.split(x)[3])
    for got, ref in ((dF, rF), (dq, rq), (dphi, rphi)):
        err = _rel(got.cpu().numpy(), ref)
        print("  rel err", err, flush=True)
        assert err < 1e-7
    ctx.close()
