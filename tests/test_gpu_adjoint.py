"""GPU vector-Jacobian product of the mobility solve, through the C ABI.

* Against the oracle's adjoint gradient (assembled operators, solves to 1e-12):
  dL/dF, dL/dq and dL/dphi for L = sum |U|^2.
* At the full 128^3 size with 64 spheres of 42 markers: central finite
  differences (eps = 1e-5, solves to 1e-12, FP64 preconditioner) along 8
  seeded directions in (forces and torques, positions, rotations), and the
  quaternion gradient along tangent directions.
* The torch.autograd.Function wrapper returns the same gradients and passes
  torch.autograd.gradcheck for positions and forces on a small system.
"""
import numpy as np
import pytest

import workloads as W
from oracle import adjoint as oadj
from oracle import bodies as B
from tests.helpers import dev, lib_context, oracle_grid

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def rb():
    import paper_1901_06427_amd as rb
    return rb


def _vjp(rb, ctx, w, q, th, FT):
    import torch
    U = torch.empty((w.nb, 6), dtype=torch.float64, device="cuda")
    rb.rbfib_solve_mobility(ctx, q, th, FT, U, include_bc=False, allow=())
    dF = torch.empty_like(U)
    dq = torch.empty((w.nb, 3), dtype=torch.float64, device="cuda")
    dphi = torch.empty_like(dq)
    dth = torch.empty((w.nb, 4), dtype=torch.float64, device="cuda")
    info = rb.rbfib_mobility_vjp(ctx, q, th, FT, (2 * U).contiguous(), dF, dq, dphi, dth, allow=())
    return U, dF, dq, dphi, dth, info


def _loss(rb, ctx, w, q, th, FT):
    import torch
    U = torch.empty((w.nb, 6), dtype=torch.float64, device="cuda")
    rb.rbfib_solve_mobility(ctx, dev(q), dev(th), dev(FT), U, include_bc=False, allow=())
    return float((U * U).sum().item())


@pytest.mark.parametrize("name", ["small_two_bodies", "box32_four_spheres"])
def test_vjp_matches_oracle(rb, name):
    if name == "small_two_bodies":
        w = W.small_box(4, n=(10, 10, 12), n_bodies=2, R=1.5, shape="ico12")
    else:
        w = W.spheres_in_box(55, (32, 32, 32), 4)
    ctx = lib_context(rb, w, tol=1e-12, max_iter=2000)
    U, dF, dq, dphi, dth, info = _vjp(rb, ctx, w, dev(w.q), dev(w.theta), dev(w.FT))
    print(name, "iters", info[0].iters, flush=True)
    g = oracle_grid(w)
    s, x = oadj.solve_U(g, w.r_ref, w.offsets, w.q, w.theta, w.FT)
    Uo = s.split(x)[3]
    rF, rq, rphi = oadj.mobility_vjp(g, w.r_ref, w.offsets, w.q, w.theta, w.FT, 2 * Uo)
    for got, ref in ((dF, rF), (dq, rq), (dphi, rphi)):
        err = np.abs(got.cpu().numpy() - ref).max() / np.abs(ref).max()
        print("  rel err", err, flush=True)
        assert err < 1e-7
    ctx.close()


def test_vjp_finite_differences_full_size(rb):
    import torch
    w = W.many_spheres()
    ctx = lib_context(rb, w, tol=1e-12, max_iter=3000, precond_fp32=0)
    U, dF, dq, dphi, dth, info = _vjp(rb, ctx, w, dev(w.q), dev(w.theta), dev(w.FT))
    print("128^3, 64 spheres: forward+adjoint iters", info[0].iters, "res", info[0].rel_residual, flush=True)
    dF, dq, dphi, dth = (t.cpu().numpy() for t in (dF, dq, dphi, dth))
    rng = np.random.default_rng(1901)
    eps = 1e-5
    # The 4-point kernel is only C^1, so central differences carry an O(eps) error
    # wherever a marker crosses a kernel breakpoint; it is compared with the size of
    # a typical directional derivative (the mean magnitude over the random directions).
    typical = []
    checks = []
    for k in range(8):
        a = rng.standard_normal((w.nb, 6))
        b = rng.standard_normal((w.nb, 3))
        c = rng.standard_normal((w.nb, 3))
        vals = []
        for sgn in (1.0, -1.0):
            q2 = w.q + sgn * eps * b
            th2 = B.rotate(w.theta, sgn * eps * c)
            vals.append(_loss(rb, ctx, w, q2, th2, w.FT + sgn * eps * a))
        fd = (vals[0] - vals[1]) / (2 * eps)
        an = np.sum(dF * a) + np.sum(dq * b) + np.sum(dphi * c)
        typical.append(abs(an))
        checks.append((fd, an))
        print("  direction", k, "fd", fd, "adjoint", an, "rel", abs(fd - an) / abs(fd), flush=True)
    scale = float(np.mean(typical))
    print("  typical directional derivative", scale, flush=True)
    # quaternion gradient along directions tangent to the unit sphere; the displaced
    # orientations are renormalised (the library accepts only unit quaternions), which
    # moves them by O(eps^2) along theta and leaves the tangent derivative unchanged
    def unit(th):
        return th / np.linalg.norm(th, axis=1, keepdims=True)

    for k in range(2):
        d = rng.standard_normal((w.nb, 4))
        d -= np.sum(d * w.theta, axis=1, keepdims=True) * w.theta
        vals = [_loss(rb, ctx, w, w.q, unit(w.theta + sgn * eps * d), w.FT) for sgn in (1.0, -1.0)]
        fd = (vals[0] - vals[1]) / (2 * eps)
        an = np.sum(dth * d)
        print("  quaternion direction", k, "fd", fd, "adjoint", an, flush=True)
        checks.append((fd, an))
    for fd, an in checks:
        assert abs(fd - an) <= 1e-5 * max(abs(fd), scale)
    ctx.close()


def test_autograd_function(rb):
    import torch
    w = W.small_box(9, n=(12, 12, 12), n_bodies=1, R=1.5, shape="ico12")
    ctx = lib_context(rb, w, tol=1e-12, max_iter=2000)
    q = dev(w.q).requires_grad_(True)
    th = dev(w.theta).requires_grad_(True)
    F = dev(w.FT).requires_grad_(True)
    U = rb.mobility_solve(ctx, q, th, F)
    (U * U).sum().backward()
    _, dF, dq, dphi, dth, _ = _vjp(rb, ctx, w, dev(w.q), dev(w.theta), dev(w.FT))
    assert torch.allclose(F.grad, dF, rtol=1e-9, atol=0)
    assert torch.allclose(q.grad, dq, rtol=1e-9, atol=0)
    assert torch.allclose(th.grad, dth, rtol=1e-9, atol=0)
    qq = dev(w.q).requires_grad_(True)
    FF = dev(w.FT).requires_grad_(True)
    thc = dev(w.theta)
    assert torch.autograd.gradcheck(lambda a, b: rb.mobility_solve(ctx, a, thc, b), (qq, FF), eps=1e-6, atol=1e-7,
                                    rtol=1e-5)
    ctx.close()
