"""GPU parity of the HIP hot path against the FP64 oracle, through the C ABI.

* marker positions, tile indices and the tile-sorted permutation: bit-exact;
* the homogeneous saddle operator y = A x: within 1e-10 relative (max-norm)
  on random state vectors, on walled, periodic, ragged (partial tiles),
  periodic-with-a-one-cell-last-tile and sliding-wall grids, up to the full
  monolayer size;
* the fluctuating-stress forcing DT W with the same Philox normals: 1e-12;
* mobility solves, with and without a prescribed marker slip: the GPU
  solution's true residual r, measured with the oracle's assembled operator,
  meets the requested tolerance, and every rigid-body velocity agrees with the
  oracle's exact solve within gain_k (||r|| + ||r_oracle||), the bound that
  residual implies (gain_k = ||A^+ e_{U,k}||, stored by the oracle).
"""
import numpy as np
import pytest

import workloads as W
from oracle import bodies as B
from oracle import mac
from oracle.saddle import Saddle
from tests.helpers import dev, error_gains, lib_context, oracle_grid, oracle_to_padded, padded_to_oracle
from tests.parity_configs import marker_slip, solve_configs

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def rb():
    import paper_1901_06427_amd as rb
    return rb


CONFIGS = {k: v for k, v in solve_configs().items() if not k.startswith("ensemble")}


def _rel(a, b):
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))


@pytest.mark.parametrize("name", list(CONFIGS))
def test_markers_bitexact(rb, name):
    import torch
    w = CONFIGS[name]
    print("markers", name, flush=True)
    ctx = lib_context(rb, w)
    q, th = dev(w.q), dev(w.theta)
    r = torch.empty((w.nm, 3), dtype=torch.float64, device="cuda")
    tile = torch.empty(w.nm, dtype=torch.int32, device="cuda")
    perm = torch.empty(w.nm, dtype=torch.int32, device="cuda")
    rb.rbfib_markers(ctx, q, th, r, tile, perm)
    torch.cuda.synchronize()
    g = oracle_grid(w)
    r_ref = B.marker_positions(w.q, w.theta, w.r_ref, w.offsets)
    t_ref, p_ref = B.marker_tiles(g, r_ref)
    assert np.array_equal(r.cpu().numpy(), r_ref)                 # bit for bit
    assert np.array_equal(tile.cpu().numpy(), t_ref)
    assert np.array_equal(perm.cpu().numpy(), p_ref)
    ctx.close()


@pytest.mark.parametrize("name", list(CONFIGS))
def test_apply_saddle(rb, name):
    import torch
    w = CONFIGS[name]
    print("apply", name, flush=True)
    ctx = lib_context(rb, w)
    g = oracle_grid(w)
    s = Saddle(g, w.q, w.theta, w.r_ref, w.offsets)
    rng = np.random.default_rng(5)
    x = rng.standard_normal(s.n)
    y_ref = s.A @ x
    xd = dev(oracle_to_padded(s, x))
    yd = torch.full((ctx.L,), float("nan"), dtype=torch.float64, device="cuda")
    rb.rbfib_apply_saddle(ctx, dev(w.q), dev(w.theta), xd, yd)
    torch.cuda.synchronize()
    y = padded_to_oracle(s, yd.cpu().numpy())
    # every block of the result separately
    for sl in (s.sl_v, s.sl_p, s.sl_l, s.sl_u):
        if sl.stop > sl.start:
            assert _rel(y[sl], y_ref[sl]) < 1e-10, (name, sl)
    # pinned wall-face slots are written as zero
    ypad = yd.cpu().numpy()
    assert np.all(np.isfinite(ypad))
    ctx.close()


@pytest.mark.parametrize("name", ["two_spheres_32x32x64", "periodic_x_16x12x12", "monolayer_64x32x16"])
def test_fluctuating_stress(rb, name):
    import torch
    from oracle import rng as orng
    w = CONFIGS[name]
    ctx = lib_context(rb, w)
    g = oracle_grid(w)
    f = torch.zeros(ctx.L, dtype=torch.float64, device="cuda")
    rb.rbfib_fluctuating_stress(ctx, 0.7, 0.01, 1234, 17, f)
    torch.cuda.synchronize()
    Wn = orng.fluid_normals(1234, 17, g.nW)
    ref = mac.noise_stress_divergence(g, Wn, 0.7, 0.01)
    got = g.padded_to_compact(f.cpu().numpy()[:3 * g.ncell])
    assert _rel(got, ref) < 1e-12
    assert np.all(f.cpu().numpy()[3 * g.ncell:] == 0.0)
    ctx.close()


def _solve_and_check(rb, name, w, tol, fp32, ks, slip=None):
    """One GPU mobility solve through the C ABI, checked against the oracle: the true
    residual meets tol, and |U - U_oracle| is within the bound the two residuals imply."""
    import torch
    ctx = lib_context(rb, w, tol=tol, precond_fp32=fp32, max_iter=400, krylov_s=ks)
    g = oracle_grid(w)
    s = Saddle(g, w.q, w.theta, w.r_ref, w.offsets)
    b = s.rhs(FT=w.FT, slip=slip)
    U = torch.empty((w.nb, 6), dtype=torch.float64, device="cuda")
    xo = torch.empty(ctx.L, dtype=torch.float64, device="cuda")
    info = rb.rbfib_solve_mobility(ctx, dev(w.q), dev(w.theta), dev(w.FT), U, x_out=xo,
                                   slip=None if slip is None else dev(slip), allow=())
    torch.cuda.synchronize()
    print("  iters", info[0].iters, "rel_residual", info[0].rel_residual, flush=True)
    x = padded_to_oracle(s, xo.cpu().numpy())
    res = s.residual(x, b)
    assert res <= tol * 1.05, res
    assert abs(res - info[0].rel_residual) <= 1e-3 * tol + 1e-14
    x_ref, _ = s.solve_fgmres(b, tol=1e-12)
    U_ref = s.split(x_ref)[3]
    nb_ = np.linalg.norm(b)
    bound = error_gains(name).reshape(-1, 6) * (res + s.residual(x_ref, b)) * nb_
    errU = np.abs(U.cpu().numpy() - U_ref)
    print("  U rel err %.3e, bound %.3e (max over components of err / bound %.3f)"
          % (_rel(U.cpu().numpy(), U_ref), bound.max() / np.abs(U_ref).max(), (errU / bound).max()), flush=True)
    assert np.all(errU <= bound * (1 + 1e-6) + 1e-15)
    ctx.close()
    return errU, U_ref


@pytest.mark.parametrize("ks", [2, 1])
@pytest.mark.parametrize("name,tol,fp32", [("single_sphere_32", 1e-8, 0), ("two_spheres_32x32x64", 1e-6, 0),
                                           ("ragged_10x12x14", 1e-8, 0), ("periodic_x_16x12x12", 1e-8, 0),
                                           ("monolayer_64x32x16", 1e-6, 0), ("single_sphere_32", 1e-8, 1),
                                           ("monolayer_64x32x16", 1e-6, 1)])
def test_solve_mobility(rb, name, tol, fp32, ks):
    print("solve", name, tol, fp32, "krylov_s", ks, flush=True)
    _solve_and_check(rb, name, CONFIGS[name], tol, fp32, ks)


@pytest.mark.parametrize("name,fp32", [("two_spheres_32x32x64", 1), ("ragged_10x12x14", 0),
                                       ("monolayer_64x32x16", 1)])
def test_solve_mobility_with_slip(rb, name, fp32):
    """A prescribed marker slip (Sec. II eq. rigidBC) enters row 3 of the right-hand side
    as -slip (Jv = KU + slip); the slip alone (zero force) drives the bodies, and with
    force and slip together the GPU meets the same residual bound.  The sliding wall of
    the monolayer adds its J_bc term to the same rows."""
    w = CONFIGS[name]
    slip = marker_slip(w)
    print("solve with slip", name, fp32, flush=True)
    errU, U_ref = _solve_and_check(rb, name, w, 1e-8, fp32, 2, slip=slip)
    # the slip really moves the bodies: zero force, slip only
    w0 = type(w)(**{**w.__dict__, "FT": np.zeros_like(w.FT)})
    errU0, U0 = _solve_and_check(rb, name, w0, 1e-8, fp32, 2, slip=slip)
    assert np.abs(U0).max() > 1e-3 * np.abs(slip).max()


@pytest.mark.parametrize("ks", [2, 3, 4])
def test_block_steps_match_single_steps(rb, ks):
    """s-step Arnoldi blocks (one pass over the basis for s new vectors, Cholesky QR of
    their Gram matrix) against one step at a time on a batch of replicas of different
    sizes and body counts: every replica converges to the tolerance and the body
    velocities agree to the accuracy it allows.  With two steps per block the iteration
    counts stay within a few steps (a block can run one step past convergence); longer
    blocks lose orthogonality in their power basis and may need more."""
    import torch
    ws = W.ensemble(5, n_replicas=6, sizes=(16, 24, 32), max_bodies=3)
    tol = 1e-6
    print("block steps", ks, flush=True)
    q = dev(np.concatenate([w.q for w in ws]))
    th = dev(np.concatenate([w.theta for w in ws]))
    nb = sum(w.nb for w in ws)
    FT = torch.as_tensor(np.random.default_rng(3).standard_normal((nb, 6)), dtype=torch.float64).cuda()
    out = {}
    for ks_ in (1, ks):
        ctx = lib_context(rb, ws, tol=tol, krylov_s=ks_)
        U = torch.empty((nb, 6), dtype=torch.float64, device="cuda")
        info = rb.rbfib_solve_mobility(ctx, q, th, FT, U, include_bc=False, allow=())
        torch.cuda.synchronize()
        out[ks_] = (U.cpu().numpy(), [i.iters for i in info], [i.rel_residual for i in info])
        ctx.close()
    print("  iters s=1", out[1][1], "s=%d" % ks, out[ks][1], flush=True)
    assert all(r <= tol * 1.05 for r in out[ks][2])
    if ks == 2:
        assert all(abs(a - b) <= 4 for a, b in zip(out[1][1], out[2][1]))
    assert _rel(out[ks][0], out[1][0]) < 2e3 * tol
