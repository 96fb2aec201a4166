"""Free-slip walls (rbfib_grid.bc = RBFIB_SLIP) on the GPU, through the C ABI,
against the oracle: the saddle apply (every block within 1e-10), the fluctuating
forcing DT W with the same Philox numbers (1e-12: wall edges of a free-slip
axis carry no stress), mobility solves with both preconditioner precisions
within their residual bounds, and one SEM step within its bound; with the
4-point and the 6-point kernel.  Configurations that a free-slip axis leaves
singular are refused."""
import numpy as np
import pytest

from oracle import mac, sem
from oracle import rng as orng
from oracle.saddle import Saddle
from tests.helpers import (dev, error_gains, lib_context, oracle_grid, oracle_to_padded, padded_to_oracle,
                           sem_error_bound)
from tests.parity_configs import slip_configs

pytestmark = pytest.mark.gpu

CONFIGS = slip_configs()


@pytest.fixture(scope="module")
def rb():
    import paper_1901_06427_amd as rb
    return rb


def _rel(a, b):
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))


@pytest.mark.parametrize("name", list(CONFIGS))
def test_apply_saddle_slip(rb, name):
    import torch
    w = CONFIGS[name]
    print("apply free-slip", name, flush=True)
    ctx = lib_context(rb, w)
    s = Saddle(oracle_grid(w), w.q, w.theta, w.r_ref, w.offsets)
    x = np.random.default_rng(6).standard_normal(s.n)
    yd = torch.full((ctx.L,), float("nan"), dtype=torch.float64, device="cuda")
    rb.rbfib_apply_saddle(ctx, dev(w.q), dev(w.theta), dev(oracle_to_padded(s, x)), yd)
    torch.cuda.synchronize()
    y, yr = padded_to_oracle(s, yd.cpu().numpy()), s.A @ x
    for sl in (s.sl_v, s.sl_p, s.sl_l, s.sl_u):
        assert _rel(y[sl], yr[sl]) < 1e-10, (name, sl)
    ctx.close()


@pytest.mark.parametrize("name", ["slip_box_12x12x16", "periodic_x_wall_y_slip_z_16x12x12"])
def test_fluctuating_stress_slip(rb, name):
    import torch
    w = CONFIGS[name]
    ctx = lib_context(rb, w)
    g = oracle_grid(w)
    f = torch.zeros(ctx.L, dtype=torch.float64, device="cuda")
    rb.rbfib_fluctuating_stress(ctx, 0.7, 0.01, 321, 5, f)
    torch.cuda.synchronize()
    ref = mac.noise_stress_divergence(g, orng.fluid_normals(321, 5, g.nW), 0.7, 0.01)
    assert _rel(g.padded_to_compact(f.cpu().numpy()[:3 * g.ncell]), ref) < 1e-12
    ctx.close()


@pytest.mark.parametrize("fp32", [1, 0])
@pytest.mark.parametrize("name", list(CONFIGS))
def test_solve_mobility_slip(rb, name, fp32):
    import torch
    w = CONFIGS[name]
    tol = 1e-8
    print("solve free-slip", name, "fp32", fp32, flush=True)
    ctx = lib_context(rb, w, tol=tol, precond_fp32=fp32, max_iter=600)
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


@pytest.mark.parametrize("name", ["periodic_x_wall_y_slip_z_16x12x12", "slip_box_12x12x16"])
def test_sem_step_slip(rb, name):
    import torch
    w = CONFIGS[name]
    tol = 1e-10
    print("sem free-slip", name, flush=True)
    ctx = lib_context(rb, w, tol=tol, precond_fp32=1, max_iter=800)
    q, th = dev(w.q), dev(w.theta)
    U = torch.empty((w.nb, 6), dtype=torch.float64, device="cuda")
    info = rb.rbfib_sem_step(ctx, q, th, dev(w.FT), 1.0, 0.01, 13, 1, U, allow=())
    ref = sem.sem_step(oracle_grid(w), w.r_ref, w.offsets, w.q, w.theta, w.FT, 1.0, 0.01, 13, 1)
    assert ref.accepted
    err = np.abs(U.cpu().numpy() - ref.U)
    bound = sem_error_bound(name, ref.rhs_norms, tol, info[0].rel_residual)
    print("  iters %d U rel err %.3e (max err / bound %.3f)" % (info[0].iters, _rel(U.cpu().numpy(), ref.U),
                                                              (err / bound).max()), flush=True)
    assert np.all(err <= bound)
    ctx.close()


def test_singular_free_slip_layouts_refused(rb):
    import workloads as W
    w = CONFIGS["slip_box_12x12x16"]
    for bc in ((W.PERIODIC, W.PERIODIC, W.SLIP), (W.PERIODIC, W.SLIP, W.SLIP), (W.PERIODIC,) * 3, (3, 1, 1)):
        g = rb.make_grid(w.n, bc)
        with pytest.raises(rb.RBFIBError) as e:
            rb.rbfib_create(g, w.r_ref, w.offsets)
        assert e.value.code == rb.RBFIB_EINVAL
