"""The deterministically second-order SEM variants on the GPU (trapezoidal,
alpha = 1, and midpoint, alpha = 1/2), through rbfib_sem_rk2_predict /
rbfib_sem_rk2_correct.

* One step of two confined spheres driven by wall repulsion and a constant
  marker force, with noise, against the oracle's variant at the same random
  numbers: the predictor within alpha dt times the bound of Algorithm 1's
  velocities (oracle gains), the corrector's velocities and the new
  configuration within 1e-6 relative at solver tolerance 1e-11.
* kT = 0, a body settling onto a wall: differences between runs with 2, 4 and 8
  steps shrink by about 4 per halving (second order), against about 2 for
  rbfib_sem_step on the same problem.
* A predictor pushed through a wall rejects the step in both calls and leaves
  the state untouched; the corrector without a predictor is refused.
* The Adams-Bashforth variant (rbfib_sem_ab2_step): two noisy steps against the
  oracle's, and its kT = 0 convergence order.
"""
import numpy as np
import pytest

import workloads as W
from oracle import bodies as B
from oracle import sem
from oracle.potentials import body_forces
from tests.helpers import dev, lib_context, oracle_grid, sem_error_bound
from tests.parity_configs import sem_configs

pytestmark = pytest.mark.gpu

PHI0, DW, BW = 4.0, 1.0, 0.25
FC = [0.03, 0.01, -0.05]


@pytest.fixture(scope="module")
def rb():
    import paper_1901_06427_amd as rb
    return rb


def _gpu_forces(rb, ctx, q, th, nb):
    import torch
    FT = torch.empty((nb, 6), dtype=torch.float64, device="cuda")
    rb.rbfib_body_forces(ctx, q, th, PHI0, DW, BW, FC, FT)
    return FT


def _rk2_step(rb, ctx, q, th, nb, kT, dt, seed, step, alpha):
    """Predictor, forces at the predictor, corrector (q, th updated in place)."""
    import torch
    qp = torch.empty_like(q)
    tp = torch.empty_like(th)
    U = torch.empty((nb, 6), dtype=torch.float64, device="cuda")
    i1 = rb.rbfib_sem_rk2_predict(ctx, q, th, _gpu_forces(rb, ctx, q, th, nb), kT, dt, seed, step, qp, tp,
                                  alpha=alpha, allow=())
    i2 = rb.rbfib_sem_rk2_correct(ctx, q, th, _gpu_forces(rb, ctx, qp, tp, nb), U, allow=())
    return qp, tp, U, i1, i2


@pytest.mark.parametrize("alpha", [1.0, 0.5])
def test_rk2_step_matches_oracle(rb, alpha):
    import torch
    name = "two_spheres_16x16x32"
    w = sem_configs()[name]
    print("rk2", name, "alpha", alpha, flush=True)
    g = oracle_grid(w)
    F = lambda q, th: body_forces(g, q, th, w.r_ref, w.offsets, PHI0, DW, BW, FC)
    tol, kT, dt, seed, step = 1e-11, 1.0, 0.05, 41, 6
    ctx = lib_context(rb, w, tol=tol, precond_fp32=1, max_iter=600)
    q, th = dev(w.q), dev(w.theta)
    qp, tp, U, i1, i2 = _rk2_step(rb, ctx, q, th, w.nb, kT, dt, seed, step, alpha)
    torch.cuda.synchronize()
    ref = sem.sem_rk2_step(g, w.r_ref, w.offsets, w.q, w.theta, F, kT, dt, seed, step, alpha=alpha, tol=1e-12)
    assert ref.accepted and i1[0].status == 0 and i2[0].status == 0
    print("  iters", i1[0].iters, i2[0].iters, flush=True)
    # predictor: Q^n moved by alpha dt U^n, whose error is bounded by the oracle gains
    bound = sem_error_bound(name, ref.em.rhs_norms, tol, i1[0].rel_residual)
    assert np.abs(qp.cpu().numpy() - ref.q_pred).max() <= alpha * dt * bound.max() + 1e-13
    # corrector velocities and the new configuration
    Ug = U.cpu().numpy()
    err = np.abs(Ug - ref.U).max() / np.abs(ref.U).max()
    print("  U_c rel err %.3e" % err, flush=True)
    assert err < 1e-6
    assert np.abs(q.cpu().numpy() - ref.q).max() <= dt * np.abs(Ug - ref.U).max() + 1e-13
    assert np.abs(B.rotation_matrices(th.cpu().numpy()) - B.rotation_matrices(ref.theta)).max() \
        <= 2 * dt * np.abs(Ug - ref.U).max() + 1e-13
    # the corrector moved the bodies differently from the predictor
    assert np.abs(q.cpu().numpy() - qp.cpu().numpy()).max() > 1e-6
    ctx.close()


def _settling_case():
    w = W.small_box(5, n=(6, 6, 8), n_bodies=1, R=1.0, shape="ico12", gap=0.5)
    w.q = np.array([[3.1, 2.9, 2.1]])
    w.theta = W.random_unit_quaternions(np.random.default_rng(3), 1)
    return w


@pytest.mark.parametrize("alpha", [1.0, 0.5])
def test_rk2_second_order_deterministic(rb, alpha):
    import torch
    w = _settling_case()
    T = 4.0
    ctx = lib_context(rb, w, tol=1e-12, precond_fp32=0, max_iter=600)

    def run(n, trap):
        q, th = dev(w.q), dev(w.theta)
        U = torch.empty((1, 6), dtype=torch.float64, device="cuda")
        for k in range(n):
            if trap:
                _rk2_step(rb, ctx, q, th, 1, 0.0, T / n, 1, k, alpha)
            else:
                rb.rbfib_sem_step(ctx, q, th, _gpu_forces(rb, ctx, q, th, 1), 0.0, T / n, 1, k, U, allow=())
        torch.cuda.synchronize()
        return q.cpu().numpy(), th.cpu().numpy()

    def d(a, b):
        return np.abs(a[0] - b[0]).max() + np.abs(B.rotation_matrices(a[1]) - B.rotation_matrices(b[1])).max()

    for trap, lo, hi in ((False, 1.6, 2.6), (True, 3.2, 5.0)):
        Q = [run(n, trap) for n in (2, 4, 8)]
        ratio = d(Q[0], Q[1]) / d(Q[1], Q[2])
        print(("rk2 alpha %g" % alpha) if trap else "euler", "ratio %.3f" % ratio, flush=True)
        assert lo < ratio < hi
    assert np.abs(Q[2][0] - w.q).max() > 0.05
    ctx.close()


@pytest.mark.parametrize("alpha", [1.0, 0.5])
def test_rk2_rejection_and_order_of_calls(rb, alpha):
    import torch
    w = _settling_case()
    ctx = lib_context(rb, w, tol=1e-10)
    q, th = dev(w.q), dev(w.theta)
    FT = dev(np.array([[0.0, 0.0, -500.0, 0.0, 0.0, 0.0]]))
    # the corrector needs a predictor first
    with pytest.raises(rb.RBFIBError):
        rb.rbfib_sem_rk2_correct(ctx, q, th, FT, allow=())
    qp, tp = torch.empty_like(q), torch.empty_like(th)
    with pytest.raises(rb.RBFIBError):
        rb.rbfib_sem_rk2_predict(ctx, q, th, FT, 0.0, 1.0, 1, 0, qp, tp, alpha=1.5)
    i1 = rb.rbfib_sem_rk2_predict(ctx, q, th, FT, 0.0, 10.0, 1, 0, qp, tp, alpha=alpha)
    assert i1[0].status == rb.RBFIB_EREJECT
    assert np.array_equal(qp.cpu().numpy(), w.q)
    i2 = rb.rbfib_sem_rk2_correct(ctx, q, th, FT)
    assert i2[0].status == rb.RBFIB_EREJECT
    assert np.array_equal(q.cpu().numpy(), w.q) and np.array_equal(th.cpu().numpy(), w.theta)
    ctx.close()


def test_ab2_steps_match_oracle(rb):
    import torch
    name = "two_spheres_16x16x32"
    w = sem_configs()[name]
    g = oracle_grid(w)
    tol, kT, dt, seed = 1e-11, 1.0, 0.05, 41
    ctx = lib_context(rb, w, tol=tol, precond_fp32=1, max_iter=600)
    q, th = dev(w.q), dev(w.theta)
    prev = torch.empty((w.nb, 6), dtype=torch.float64, device="cuda")
    U = torch.empty_like(prev)
    qo, tho, po = w.q.copy(), w.theta.copy(), None
    for k in range(2):
        info = rb.rbfib_sem_ab2_step(ctx, q, th, _gpu_forces(rb, ctx, q, th, w.nb), kT, dt, seed, k, prev, k > 0, U,
                                     allow=())
        torch.cuda.synchronize()
        Fo = body_forces(g, qo, tho, w.r_ref, w.offsets, PHI0, DW, BW, FC)
        ref, po = sem.sem_ab2_step(g, w.r_ref, w.offsets, qo, tho, Fo, kT, dt, seed, k, U_det_prev=po, tol=1e-12)
        assert ref.accepted and info[0].status == 0
        err = np.abs(U.cpu().numpy() - ref.U).max() / np.abs(ref.U).max()
        print("ab2 step", k, "iters", info[0].iters, "U_c rel err %.3e" % err, flush=True)
        assert err < 1e-6
        assert np.abs(prev.cpu().numpy() - po).max() <= 1e-6 * np.abs(po).max()
        # continue both from the oracle's configuration so the steps stay comparable
        qo, tho = ref.q, ref.theta
        q.copy_(dev(qo))
        th.copy_(dev(tho))
    ctx.close()


def test_ab2_second_order_deterministic(rb):
    import torch
    w = _settling_case()
    T = 4.0
    ctx = lib_context(rb, w, tol=1e-12, precond_fp32=0, max_iter=600)

    def run(n):
        q, th = dev(w.q), dev(w.theta)
        prev = torch.empty((1, 6), dtype=torch.float64, device="cuda")
        for k in range(n):
            rb.rbfib_sem_ab2_step(ctx, q, th, _gpu_forces(rb, ctx, q, th, 1), 0.0, T / n, 1, k, prev, k > 0, allow=())
        torch.cuda.synchronize()
        return q.cpu().numpy(), th.cpu().numpy()

    def d(a, b):
        return np.abs(a[0] - b[0]).max() + np.abs(B.rotation_matrices(a[1]) - B.rotation_matrices(b[1])).max()

    Q = [run(n) for n in (4, 8, 16)]
    ratio = d(Q[0], Q[1]) / d(Q[1], Q[2])
    print("ab2 ratio %.3f" % ratio, flush=True)
    assert 3.2 < ratio < 5.0
    ctx.close()
