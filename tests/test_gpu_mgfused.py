"""Fused multigrid level kernels against the separate smoother / restriction /
prolongation kernels, through rbfib_precondition.

The fused kernels implement two sweeps per level, so both run a V(2,2) cycle (damped Jacobi, full-weighting restriction,
linear prolongation, dense coarsest solve) with the same association of every
floating-point operation, so the preconditioner outputs are identical: grids
with ragged tiles, a periodic axis, a sliding wall, an axis that stops
coarsening before the others, a batch whose replicas have different depths,
and the full 128^3 and 256x128x32 sizes, in FP32 and FP64.  The FP64 and FP32
cycles are the same linear map in two precisions, so they agree to FP32
rounding (a transfer operator with a wrong weight on one component shows up
here as a difference of order one).
"""
import numpy as np
import pytest

import workloads as W
from tests.helpers import dev, lib_context

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def rb():
    import paper_1901_06427_amd as rb
    return rb


def _cases():
    per = W.small_box(22, n=(16, 12, 12), n_bodies=3, R=1.5, shape="ico12")
    per.bc = (0, 1, 1)
    return {
        "ragged_10x12x14": [W.small_box(21, n=(10, 12, 14), n_bodies=3, R=1.5, shape="ico12")],
        "periodic_x_16x12x12": [per],
        "uneven_16x12x20": [W.small_box(23, n=(16, 12, 20), n_bodies=2, R=1.5, shape="ico12")],
        "monolayer_64x32x16": [W.monolayer(n=(64, 32, 16), rows=4, cols=16)],
        "batch_mixed_depths": W.ensemble(7, n_replicas=6, sizes=(16, 24, 32, 48), max_bodies=2),
        "many_spheres_128": [W.many_spheres()],
        "monolayer_256x128x32": [W.monolayer()],
    }


CASES = _cases()
TOL = {1: 0.0, 0: 0.0}


def _state(ws, ctx, seed):
    import torch
    q = dev(np.concatenate([w.q for w in ws]))
    th = dev(np.concatenate([w.theta for w in ws]))
    r = torch.as_tensor(np.random.default_rng(seed).standard_normal(ctx.L), dtype=torch.float64).cuda()
    return q, th, r


@pytest.mark.parametrize("fp32", [1, 0])
@pytest.mark.parametrize("name", list(CASES))
def test_fused_vcycle_matches_separate_kernels(rb, name, fp32):
    import torch
    ws = CASES[name]
    print("mgfused", name, "fp32", fp32, flush=True)
    ctx = lib_context(rb, ws, precond_fp32=fp32, mg_fused=0, mg_sweeps=2)
    q, th, r = _state(ws, ctx, 11)
    z0 = torch.full((ctx.L,), float("nan"), dtype=torch.float64, device="cuda")
    rb.rbfib_precondition(ctx, q, th, r, z0)
    rb.rbfib_set_opts(ctx, rb.rbfib_default_opts(precond_fp32=fp32, mg_fused=2, mg_sweeps=2))
    z1 = torch.full_like(z0, float("nan"))
    rb.rbfib_precondition(ctx, q, th, r, z1)
    torch.cuda.synchronize()
    a, b = z1.cpu().numpy(), z0.cpu().numpy()
    assert np.all(np.isfinite(a)) and np.all(np.isfinite(b))
    err = float(np.abs(a - b).max() / np.abs(b).max())
    print("  max rel diff", err, flush=True)
    assert err <= TOL[fp32]
    ctx.close()


@pytest.mark.parametrize("fp32", [1, 0])
def test_fused_solve_matches_separate_kernels(rb, fp32):
    import torch
    w = W.two_spheres()
    out = []
    for fused in (0, 2):
        ctx = lib_context(rb, w, tol=1e-8, precond_fp32=fp32, mg_fused=fused, mg_sweeps=2)
        U = torch.empty((w.nb, 6), dtype=torch.float64, device="cuda")
        info = rb.rbfib_solve_mobility(ctx, dev(w.q), dev(w.theta), dev(w.FT), U, include_bc=False)
        print("fused", fused, "fp32", fp32, "iters", info[0].iters, "res", info[0].rel_residual, flush=True)
        assert info[0].rel_residual <= 1e-8 * 1.05
        out.append((info[0].iters, U.cpu().numpy()))
        ctx.close()
    assert abs(out[0][0] - out[1][0]) <= 2
    assert np.abs(out[0][1] - out[1][1]).max() <= 1e-6 * np.abs(out[0][1]).max()


@pytest.mark.parametrize("fused", [2, 0])
@pytest.mark.parametrize("name", ["ragged_10x12x14", "periodic_x_16x12x12", "uneven_16x12x20",
                                  "monolayer_64x32x16", "batch_mixed_depths"])
def test_fp64_cycle_matches_fp32_cycle(rb, name, fused):
    import torch
    ws = CASES[name]
    z = {}
    for fp32 in (0, 1):
        ctx = lib_context(rb, ws, precond_fp32=fp32, mg_fused=fused, mg_sweeps=2)
        q, th, r = _state(ws, ctx, 12)
        out = torch.full((ctx.L,), float("nan"), dtype=torch.float64, device="cuda")
        rb.rbfib_precondition(ctx, q, th, r, out)
        torch.cuda.synchronize()
        z[fp32] = out.cpu().numpy()
        lay = ctx.layout
        ctx.close()
    # per replica and per field (u, v, w, p, lambda, U)
    worst = 0.0
    for k in range(len(ws)):
        bounds = [lay[k][0] + i * int(np.prod(ws[k].n)) for i in range(5)] + [lay[k][3], lay[k][3] + 6 * ws[k].nb]
        for a, b in zip(bounds[:-1], bounds[1:]):
            ref = z[0][a:b]
            if b > a and np.abs(ref).max() > 0:
                worst = max(worst, float(np.abs(z[1][a:b] - ref).max() / np.abs(ref).max()))
    print(name, "fused", fused, "fp32 vs fp64 worst field rel diff", worst, flush=True)
    assert worst < 2e-5


@pytest.mark.parametrize("fp32", [1, 0])
def test_mixed_levels_match_separate_kernels(rb, fp32):
    """mg_fused = 1 picks fused or separate kernels per level by workgroup count
    (the 128^3 grid: fused on the fine levels, separate on the coarse ones)."""
    import torch
    ws = CASES["many_spheres_128"]
    ctx = lib_context(rb, ws, precond_fp32=fp32, mg_fused=0, mg_sweeps=2)
    q, th, r = _state(ws, ctx, 13)
    z = []
    for mode in (0, 1):
        rb.rbfib_set_opts(ctx, rb.rbfib_default_opts(precond_fp32=fp32, mg_fused=mode, mg_sweeps=2))
        out = torch.full((ctx.L,), float("nan"), dtype=torch.float64, device="cuda")
        rb.rbfib_precondition(ctx, q, th, r, out)
        torch.cuda.synchronize()
        z.append(out.cpu().numpy())
    assert np.all(np.isfinite(z[1]))
    assert np.array_equal(z[0], z[1])
    ctx.close()
