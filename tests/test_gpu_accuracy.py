"""Accuracy of the benchmark's own replica shapes against the oracle, through the
C ABI, with the FP32 multigrid preconditioner of the batched benchmark.

Two replicas of the 256-replica ensemble are compared directly with the oracle:
the crowded 16^3 box with four spheres (the slowest replicas, which set the
length of the batched iteration loop) and a 48^3 box.  For a mobility solve and
for one SEM step, at the workload tolerance (1e-6 relative residual) and at a
tighter one, the velocities stay within the bound their residuals imply
(oracle gains, tests/helpers.py), and at the tighter tolerance they agree with
the oracle to 1e-6 relative -- the accuracy the batched-versus-plain comparison
is stated at.  Each case prints its error, so the log reports both.
"""
import numpy as np
import pytest

from oracle import sem
from oracle.saddle import Saddle
from tests.helpers import dev, error_gains, lib_context, oracle_grid, padded_to_oracle, sem_error_bound
from tests.parity_configs import ensemble_replicas

pytestmark = pytest.mark.gpu

REPS = ensemble_replicas()


@pytest.fixture(scope="module")
def rb():
    import paper_1901_06427_amd as rb
    return rb


def _rel(a, b):
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))


@pytest.mark.parametrize("name", list(REPS))
@pytest.mark.parametrize("tol", [1e-6, 1e-9])
def test_ensemble_replica_solve(rb, name, tol):
    import torch
    w = REPS[name]
    print("ensemble solve", name, w.name, w.n, "bodies", w.nb, "tol", tol, flush=True)
    ctx = lib_context(rb, w, tol=tol, precond_fp32=1)
    g = oracle_grid(w)
    s = Saddle(g, w.q, w.theta, w.r_ref, w.offsets)
    b = s.rhs(FT=w.FT)
    U = torch.empty((w.nb, 6), dtype=torch.float64, device="cuda")
    xo = torch.empty(ctx.L, dtype=torch.float64, device="cuda")
    info = rb.rbfib_solve_mobility(ctx, dev(w.q), dev(w.theta), dev(w.FT), U, x_out=xo, allow=())
    res = s.residual(padded_to_oracle(s, xo.cpu().numpy()), b)
    x_ref, _ = s.solve_fgmres(b, tol=1e-12)
    U_ref = s.split(x_ref)[3]
    err = np.abs(U.cpu().numpy() - U_ref)
    bound = error_gains(name).reshape(-1, 6) * (res + s.residual(x_ref, b)) * np.linalg.norm(b)
    rel = _rel(U.cpu().numpy(), U_ref)
    print("  iters %d residual %.2e  U rel err %.3e  bound %.3e" % (info[0].iters, res, rel,
                                                                 bound.max() / np.abs(U_ref).max()), flush=True)
    assert res <= 1.05 * tol
    assert np.all(err <= bound * (1 + 1e-6) + 1e-15)
    if tol <= 1e-9:
        assert rel < 1e-6
    ctx.close()


@pytest.mark.parametrize("name", list(REPS))
@pytest.mark.parametrize("tol", [1e-6, 1e-10])
def test_ensemble_replica_sem_step(rb, name, tol):
    import torch
    w = REPS[name]
    k = int(w.name.split("_")[1])
    seed = 2024 + k                      # the draws replica k takes in the batched benchmark
    print("ensemble sem step", name, w.name, "tol", tol, flush=True)
    ctx = lib_context(rb, w, tol=tol, precond_fp32=1)
    q, th = dev(w.q), dev(w.theta)
    U = torch.empty((w.nb, 6), dtype=torch.float64, device="cuda")
    info = rb.rbfib_sem_step(ctx, q, th, dev(w.FT), 1.0, 0.01, seed, 0, U, allow=())
    ref = sem.sem_step(oracle_grid(w), w.r_ref, w.offsets, w.q, w.theta, w.FT, 1.0, 0.01, seed, 0)
    err = np.abs(U.cpu().numpy() - ref.U)
    bound = sem_error_bound(name, ref.rhs_norms, tol, info[0].rel_residual)
    rel = _rel(U.cpu().numpy(), ref.U)
    print("  iters %d  U rel err %.3e  bound %.3e" % (info[0].iters, rel, bound.max() / np.abs(ref.U).max()),
          flush=True)
    assert np.all(err <= bound)
    if tol <= 1e-10:
        assert rel < 1e-6
    ctx.close()
