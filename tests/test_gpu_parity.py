"""GPU parity of the HIP hot path against the FP64 oracle, through the C ABI.

* marker positions, tile indices and the tile-sorted permutation: bit-exact;
* the homogeneous saddle operator y = A x: within 1e-10 relative (max-norm)
  on random state vectors, on walled, periodic, ragged (partial tiles),
  periodic-with-a-one-cell-last-tile and sliding-wall grids, up to the full
  monolayer size;
* the fluctuating-stress forcing DT W with the same Philox normals: 1e-12;
* mobility solves: the GPU solution's true residual, measured with the
  oracle's assembled operator, meets the requested tolerance, and U agrees
  with the oracle's exact solve to the accuracy that tolerance allows.
"""
import numpy as np
import pytest

import workloads as W
from oracle import bodies as B
from oracle import mac
from oracle.saddle import Saddle
from tests.helpers import dev, lib_context, oracle_grid, oracle_to_padded, padded_to_oracle

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def rb():
    import paper_1901_06427_amd as rb
    return rb


def _configs():
    out = {
        "single_sphere_32": W.single_sphere(),
        "two_spheres_32x32x64": W.two_spheres(),
        "ragged_10x12x14": W.small_box(21, n=(10, 12, 14), n_bodies=3, R=1.5, shape="ico12"),
    }
    w = W.small_box(22, n=(16, 12, 12), n_bodies=3, R=1.5, shape="ico12")
    w.bc = (0, 1, 1)
    out["periodic_x_16x12x12"] = w
    # periodic x of 17 cells: the last tile holds one cell, and markers of the body
    # at x = 0.15 h in cell 0 reach cell 15 (tile 3) through the wrap
    w = W.small_box(23, n=(17, 12, 12), n_bodies=2, R=1.5, shape="ico12")
    w.bc = (W.PERIODIC, W.WALL, W.WALL)
    w.q[0, 0] = 0.15 * w.h
    out["periodic_wrap_17x12x12"] = w
    m = W.monolayer(n=(64, 32, 16), rows=4, cols=16)
    out["monolayer_64x32x16"] = m
    return out


CONFIGS = _configs()


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


@pytest.mark.parametrize("ks", [2, 1])
@pytest.mark.parametrize("name,tol,fp32", [("single_sphere_32", 1e-8, 0), ("two_spheres_32x32x64", 1e-6, 0),
                                           ("ragged_10x12x14", 1e-8, 0), ("periodic_x_16x12x12", 1e-8, 0),
                                           ("monolayer_64x32x16", 1e-6, 0), ("single_sphere_32", 1e-8, 1),
                                           ("monolayer_64x32x16", 1e-6, 1)])
def test_solve_mobility(rb, name, tol, fp32, ks):
    import torch
    w = CONFIGS[name]
    print("solve", name, tol, fp32, "krylov_s", ks, flush=True)
    ctx = lib_context(rb, w, tol=tol, precond_fp32=fp32, max_iter=400, krylov_s=ks)
    g = oracle_grid(w)
    s = Saddle(g, w.q, w.theta, w.r_ref, w.offsets)
    b = s.rhs(FT=w.FT)
    U = torch.empty((w.nb, 6), dtype=torch.float64, device="cuda")
    xo = torch.empty(ctx.L, dtype=torch.float64, device="cuda")
    info = rb.rbfib_solve_mobility(ctx, dev(w.q), dev(w.theta), dev(w.FT), U, x_out=xo, allow=())
    torch.cuda.synchronize()
    print("  iters", info[0].iters, "rel_residual", info[0].rel_residual, flush=True)
    x = padded_to_oracle(s, xo.cpu().numpy())
    res = s.residual(x, b)
    assert res <= tol * 1.05, res
    assert abs(res - info[0].rel_residual) <= 1e-3 * tol + 1e-14
    x_ref, inf = s.solve_fgmres(b, tol=1e-12)
    U_ref = s.split(x_ref)[3]
    err = _rel(U.cpu().numpy(), U_ref)
    print("  U rel err", err, flush=True)
    assert err < 2e3 * tol
    ctx.close()


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
