"""GPU parity of one Split-Euler-Maruyama step (Algorithm 1) against the oracle.

Both sides draw the same Philox normals (random forces/torques and the
fluctuating stress), take the same random finite differences with the same
delta, and solve to tight tolerances, so U^n and the new configuration must
agree to the accuracy the solver tolerance allows.  A step that pushes a
marker through a wall is rejected and leaves q and theta untouched.
"""
import numpy as np
import pytest

import workloads as W
from oracle import bodies as B
from oracle import sem
from tests.helpers import dev, lib_context, oracle_grid

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def rb():
    import paper_1901_06427_amd as rb
    return rb


def _rel(a, b):
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))


def _rot_err(th_a, th_b):
    Ra = B.rotation_matrices(th_a)
    Rb = B.rotation_matrices(th_b)
    return float(np.abs(Ra - Rb).max())


CASES = {
    "two_spheres_16x16x32": W.spheres_in_box(31, (16, 16, 32), 2, name="two_small"),
    "two_spheres_32x32x64": W.two_spheres(),
    "monolayer_32x16x12_sliding": W.monolayer(n=(32, 16, 12), rows=2, cols=8),
}


@pytest.mark.parametrize("name", list(CASES))
@pytest.mark.parametrize("fp32", [0, 1])
def test_sem_step_matches_oracle(rb, name, fp32):
    import torch
    w = CASES[name]
    print("sem", name, "fp32", fp32, flush=True)
    kT, dt, seed, step, delta = 1.0, 0.01, 77, 3, 1e-5
    ctx = lib_context(rb, w, tol=1e-11, precond_fp32=fp32, max_iter=600, rfd_delta=delta)
    q, th = dev(w.q), dev(w.theta)
    U = torch.empty((w.nb, 6), dtype=torch.float64, device="cuda")
    info = rb.rbfib_sem_step(ctx, q, th, dev(w.FT), kT, dt, seed, step, U, allow=())
    torch.cuda.synchronize()
    print("  iters", info[0].iters, "res", info[0].rel_residual, flush=True)
    g = oracle_grid(w)
    ref = sem.sem_step(g, w.r_ref, w.offsets, w.q, w.theta, w.FT, kT, dt, seed, step, delta=delta)
    assert ref.accepted
    errU = _rel(U.cpu().numpy(), ref.U)
    print("  U rel err", errU, flush=True)
    assert errU < 1e-6
    assert np.abs(q.cpu().numpy() - ref.q).max() < 1e-6 * dt * np.abs(ref.U).max() + 1e-14
    assert _rot_err(th.cpu().numpy(), ref.theta) < 1e-6 * dt * np.abs(ref.U).max() + 1e-14
    ctx.close()


def test_sem_step_default_tolerance(rb):
    """At the workload tolerance (1e-6 relative residual) the step tracks the exact
    step to about 1e-2: the noise dominates ||b||, so a relative residual of
    1e-6 leaves U (a small part of the solution) with a larger relative error."""
    import torch
    w = CASES["two_spheres_32x32x64"]
    ctx = lib_context(rb, w, tol=1e-6, precond_fp32=1)
    q, th = dev(w.q), dev(w.theta)
    U = torch.empty((w.nb, 6), dtype=torch.float64, device="cuda")
    info = rb.rbfib_sem_step(ctx, q, th, dev(w.FT), 1.0, 0.01, 5, 0, U, allow=())
    g = oracle_grid(w)
    ref = sem.sem_step(g, w.r_ref, w.offsets, w.q, w.theta, w.FT, 1.0, 0.01, 5, 0)
    err = _rel(U.cpu().numpy(), ref.U)
    print("  tol 1e-6: iters", info[0].iters, "U rel err", err, flush=True)
    assert info[0].rel_residual <= 1e-6
    assert err < 2e-2
    ctx.close()


def test_sem_step_rejection(rb):
    import torch
    w = W.small_box(2, n=(8, 8, 8), n_bodies=1, R=1.5, shape="ico12")
    q0 = np.array([[4.0, 4.0, 2.0]])
    F = np.array([[0.0, 0.0, -1e5, 0.0, 0.0, 0.0]])
    ctx = lib_context(rb, w, tol=1e-8)
    q, th = dev(q0), dev(w.theta)
    U = torch.empty((1, 6), dtype=torch.float64, device="cuda")
    info = rb.rbfib_sem_step(ctx, q, th, dev(F), 1.0, 1.0, 1, 0, U)
    assert info[0].status == rb.RBFIB_EREJECT
    assert np.array_equal(q.cpu().numpy(), q0)
    assert np.array_equal(th.cpu().numpy(), w.theta)
    info = rb.rbfib_sem_step(ctx, q, th, dev(F * 0), 1.0, 1e-3, 1, 0, U)
    assert info[0].status == rb.RBFIB_OK
    assert not np.array_equal(q.cpu().numpy(), q0)
    # a configuration that is already outside is rejected before any solve
    qbad = dev(np.array([[4.0, 4.0, 0.5]]))
    info = rb.rbfib_sem_step(ctx, qbad, th, dev(F * 0), 1.0, 1e-3, 1, 0, U)
    assert info[0].status == rb.RBFIB_EREJECT and info[0].iters == 0
    ctx.close()
