"""Degenerate inputs through the C ABI: replicas without bodies.

* A body-free slit whose bottom wall slides (plane Couette flow) batched with a
  replica holding a sphere: the slit's flow matches the oracle's solve (whose
  discrete Couette profile is exactly linear) and the sphere replica's U equals
  its solve alone bit for bit.
* A context whose replicas all have no bodies: the saddle apply matches the
  oracle, the solve gives the Couette profile, and a SEM step (fluctuating fluid
  only) runs and reports success.
"""
import numpy as np
import pytest

import workloads as W
from oracle.saddle import Saddle
from tests.helpers import dev, lib_context, oracle_grid, oracle_to_padded, padded_to_oracle

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def rb():
    import paper_1901_06427_amd as rb
    return rb


def _couette(n=(8, 6, 10), speed=0.5):
    wv = W.zero_wall_vel()
    wv[2, 0, 0] = speed
    return W.Workload("couette", n, (W.PERIODIC, W.PERIODIC, W.WALL), 1.0, 1.0, wv, np.zeros((0, 3)),
                      np.array([0], dtype=np.int32), np.zeros((0, 3)), np.zeros((0, 4)), np.zeros((0, 6)),
                      np.zeros(0), kT=1.0, dt=0.01, tol=1e-10)


def _cat(ws, key, cols):
    a = [getattr(w, key) for w in ws]
    return dev(np.concatenate(a) if a else np.zeros((0, cols)))


def test_body_free_replica_in_batch(rb):
    import torch
    c = _couette()
    s_ = W.spheres_in_box(101, (16, 16, 16), 1, name="sphere")
    ws = [c, s_]
    ctx = lib_context(rb, ws, tol=1e-10, precond_fp32=1)
    U = torch.empty((1, 6), dtype=torch.float64, device="cuda")
    xo = torch.empty(ctx.L, dtype=torch.float64, device="cuda")
    info = rb.rbfib_solve_mobility(ctx, _cat(ws, "q", 3), _cat(ws, "theta", 4), _cat(ws, "FT", 6), U, x_out=xo,
                                   allow=())
    lay = ctx.layout.copy()
    ctx.close()
    print("iters", [i.iters for i in info], flush=True)
    # the slit: oracle solve with the same boundary data
    s = Saddle(oracle_grid(c), c.q, c.theta, c.r_ref, c.offsets)
    b = s.rhs(FT=c.FT, include_bc=True)
    x_ref = s.solve(b, tol=1e-12)
    a, e = int(lay[0][0]), int(lay[0][3])
    xg = padded_to_oracle(s, xo.cpu().numpy()[a:e])
    vg, vr = xg[s.sl_v], x_ref[s.sl_v]
    assert np.abs(vg - vr).max() <= 1e-7 * np.abs(vr).max()
    assert s.residual(xg, b) <= 1.05e-10
    # the sphere replica is unaffected by its body-free neighbour
    c1 = lib_context(rb, s_, tol=1e-10, precond_fp32=1)
    U1 = torch.empty((1, 6), dtype=torch.float64, device="cuda")
    rb.rbfib_solve_mobility(c1, dev(s_.q), dev(s_.theta), dev(s_.FT), U1, allow=())
    assert np.array_equal(U.cpu().numpy(), U1.cpu().numpy())
    c1.close()


def test_all_replicas_body_free(rb):
    import torch
    ws = [_couette(), _couette(n=(12, 8, 6), speed=-0.3)]
    ctx = lib_context(rb, ws, tol=1e-10, precond_fp32=1)
    empty3, empty4, empty6 = _cat(ws, "q", 3), _cat(ws, "theta", 4), _cat(ws, "FT", 6)
    lay = ctx.layout.copy()
    # apply, on random compact unknowns of each replica
    rng = np.random.default_rng(4)
    xf = np.zeros(ctx.L)
    xs = []
    for k, w in enumerate(ws):
        s = Saddle(oracle_grid(w), w.q, w.theta, w.r_ref, w.offsets)
        xs.append(rng.standard_normal(s.n))
        xf[int(lay[k][0]):int(lay[k][3])] = oracle_to_padded(s, xs[-1])
    x = dev(xf)
    y = torch.empty_like(x)
    rb.rbfib_apply_saddle(ctx, empty3, empty4, x, y)
    for k, w in enumerate(ws):
        s = Saddle(oracle_grid(w), w.q, w.theta, w.r_ref, w.offsets)
        yr = s.A @ xs[k]
        yg = padded_to_oracle(s, y.cpu().numpy()[int(lay[k][0]):int(lay[k][3])])
        assert np.abs(yg - yr).max() <= 1e-10 * np.abs(yr).max()
    # solve: Couette flow in both
    xo = torch.empty(ctx.L, dtype=torch.float64, device="cuda")
    info = rb.rbfib_solve_mobility(ctx, empty3, empty4, empty6, None, x_out=xo, allow=())
    for k, w in enumerate(ws):
        s = Saddle(oracle_grid(w), w.q, w.theta, w.r_ref, w.offsets)
        b = s.rhs(FT=w.FT, include_bc=True)
        a, e = int(lay[k][0]), int(lay[k][3])
        assert s.residual(padded_to_oracle(s, xo.cpu().numpy()[a:e]), b) <= 1.05e-10, info[k].iters
    # a SEM step with no bodies: fluctuating fluid only
    info = rb.rbfib_sem_step(ctx, empty3, empty4, empty6, 1.0, 0.01, 3, 0, None, allow=())
    assert all(i.status == 0 for i in info)
    ctx.close()
