"""Full-size and statistical checks on the GPU.

* Saddle apply at the full monolayer size (256x128x32, periodic x, sliding
  bottom wall, 1024 twelve-marker spheres) and the full 128^3 box with 64
  spheres, within 1e-10 of the oracle's assembled operator on random states.
* A mobility solve at each full size meets its relative-residual tolerance as
  measured with the oracle's assembled operator (a property that holds at any
  size), for the FP32 and the FP64 preconditioner.
* Fluctuation-dissipation balance: over a batch of identical replicas with
  different seeds, dt * Cov(U^n) of the SEM velocity with zero deterministic
  force matches 2 kT N (N assembled by the oracle's exact solves) within
  sampling error; the Brownian part dominates U^n at small dt.
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


FULL = {"monolayer_256x128x32": W.monolayer, "box128_64_spheres": W.many_spheres}


@pytest.mark.parametrize("name", list(FULL))
def test_full_size_apply_and_solve(rb, name):
    import torch
    w = FULL[name]()
    print(name, "bodies", w.nb, "markers", w.nm, flush=True)
    g = oracle_grid(w)
    s = Saddle(g, w.q, w.theta, w.r_ref, w.offsets)
    ctx = lib_context(rb, w, tol=1e-6, precond_fp32=1, max_iter=1200)
    rng = np.random.default_rng(8)
    x = rng.standard_normal(s.n)
    yd = torch.empty(ctx.L, dtype=torch.float64, device="cuda")
    rb.rbfib_apply_saddle(ctx, dev(w.q), dev(w.theta), dev(oracle_to_padded(s, x)), yd)
    y = padded_to_oracle(s, yd.cpu().numpy())
    yr = s.A @ x
    for sl in (s.sl_v, s.sl_p, s.sl_l, s.sl_u):
        assert np.abs(y[sl] - yr[sl]).max() < 1e-10 * np.abs(yr[sl]).max()
    b = s.rhs(FT=w.FT)
    for fp32 in (1, 0):
        c2 = lib_context(rb, w, tol=1e-6, precond_fp32=fp32, max_iter=1200) if fp32 == 0 else ctx
        U = torch.empty((w.nb, 6), dtype=torch.float64, device="cuda")
        xo = torch.empty(c2.L, dtype=torch.float64, device="cuda")
        info = rb.rbfib_solve_mobility(c2, dev(w.q), dev(w.theta), dev(w.FT), U, x_out=xo, allow=())
        res = s.residual(padded_to_oracle(s, xo.cpu().numpy()), b)
        print("  fp32" if fp32 else "  fp64", "iters", info[0].iters, "oracle residual", res, flush=True)
        assert res <= 1.05e-6
        if c2 is not ctx:
            c2.close()
    ctx.close()


def test_fluctuation_dissipation_statistics(rb):
    import torch
    base = W.spheres_in_box(77, (16, 16, 16), 1, R=2.5)
    nrep, nstep = 256, 8
    kT, dt = 1.0, 1e-4
    reps = [base] * nrep
    ctx = lib_context(rb, reps, tol=1e-8, precond_fp32=1)
    q0 = np.tile(base.q, (nrep, 1))
    th0 = np.tile(base.theta, (nrep, 1))
    zero = dev(np.zeros((nrep, 6)))
    U = torch.empty((nrep, 6), dtype=torch.float64, device="cuda")
    samples = []
    for k in range(nstep):
        q, th = dev(q0), dev(th0)            # every sample starts from the same configuration
        rb.rbfib_sem_step(ctx, q, th, zero, kT, dt, 4242, k, U, allow=())
        samples.append(U.cpu().numpy().copy())
    S = np.concatenate(samples)              # (nrep * nstep, 6)
    ctx.close()
    # N from six exact oracle solves (unit forces and torques)
    s = Saddle(oracle_grid(base), base.q, base.theta, base.r_ref, base.offsets)
    N = np.zeros((6, 6))
    for j in range(6):
        F = np.zeros((1, 6))
        F[0, j] = 1.0
        N[:, j] = s.split(s.solve(s.rhs(FT=F, include_bc=False)))[3][0]
    n = S.shape[0]
    C = dt * np.cov(S.T)
    target = 2 * kT * N
    # Wishart standard deviation of each covariance entry: sqrt((T_ij^2 + T_ii T_jj) / n)
    sd = np.sqrt((target ** 2 + np.outer(np.diag(target), np.diag(target))) / n)
    z = (C - target) / sd
    print("max |z| over the 6x6 covariance", np.abs(z).max(), flush=True)
    assert np.abs(z).max() < 5.0
    # the mean velocity (thermal drift + noise mean) is small against the noise scale
    assert np.all(np.abs(S.mean(axis=0)) < 5 * np.sqrt(np.diag(target) / dt / n) + 0.05 * np.sqrt(np.diag(target) / dt))
