"""The LDS-resident bottom of the V-cycle against the separate kernels.

With mg_bottom = K > 0 each replica's levels from the first one whose grids fit
K KB of one workgroup's LDS down to the dense coarsest solve run in a single
kernel (K = 64 takes whole 16^3 replicas, K = 24 every level from 12^3 down,
K = 2 little more than the coarsest levels); with
mg_bottom = 0 every level runs in the separate smoother / residual / restriction /
prolongation kernels and the coarsest solve in its own kernel.  Both evaluate
every point with the same helpers in the same order, so the preconditioner
outputs and whole FGMRES solves are identical to the bit: ragged grids, a
periodic axis, an axis that stops coarsening first, batches whose replicas start
the bottom kernel at different levels (including level 0), the fused level
kernels above the bottom levels, and the full 256-replica ensemble (large
enough for the four-point vector paths of the separate kernels), in FP32 and FP64.
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
        "batch_mixed_depths": W.ensemble(7, n_replicas=8, sizes=(16, 24, 32, 48), max_bodies=2),
    }


CASES = _cases()


def _state(ws, L, seed):
    import torch
    q = dev(np.concatenate([w.q for w in ws]))
    th = dev(np.concatenate([w.theta for w in ws]))
    r = torch.as_tensor(np.random.default_rng(seed).standard_normal(L), dtype=torch.float64).cuda()
    return q, th, r


def _precondition(rb, ws, fp32, bottom, seed=11, **kw):
    import torch
    ctx = lib_context(rb, ws, precond_fp32=fp32, mg_bottom=bottom, **kw)
    q, th, r = _state(ws, ctx.L, seed)
    z = torch.full((ctx.L,), float("nan"), dtype=torch.float64, device="cuda")
    rb.rbfib_precondition(ctx, q, th, r, z)
    torch.cuda.synchronize()
    out = z.cpu().numpy()
    ctx.close()
    return out


@pytest.mark.parametrize("budget", [64, 24, 2])
@pytest.mark.parametrize("fp32", [1, 0])
@pytest.mark.parametrize("name", list(CASES))
def test_bottom_vcycle_matches_separate_kernels(rb, name, fp32, budget):
    ws = CASES[name]
    print("mgbottom", name, "fp32", fp32, "budget", budget, flush=True)
    a = _precondition(rb, ws, fp32, budget)
    b = _precondition(rb, ws, fp32, 0)
    assert np.all(np.isfinite(a)) and np.all(np.isfinite(b))
    assert np.array_equal(a, b), float(np.abs(a - b).max() / np.abs(b).max())


@pytest.mark.parametrize("cheby", [0.27, 0.0])
@pytest.mark.parametrize("fp32", [1, 0])
def test_bottom_with_fused_levels(rb, fp32, cheby):
    """Fused level kernels above the bottom kernel, with per-sweep (Chebyshev) or
    constant weights."""
    ws = CASES["batch_mixed_depths"]
    print("mgbottom fused levels fp32", fp32, "cheby", cheby, flush=True)
    a = _precondition(rb, ws, fp32, 24, mg_sweeps=2, mg_sweeps_p=2, mg_fused=2, mg_cheby=cheby)
    b = _precondition(rb, ws, fp32, 0, mg_sweeps=2, mg_sweeps_p=2, mg_fused=0, mg_cheby=cheby)
    assert np.array_equal(a, b)


def test_bottom_full_ensemble(rb):
    ws = W.ensemble()
    print("mgbottom full ensemble", flush=True)
    b = _precondition(rb, ws, 1, 0, restart=4)
    for budget in (64, 24):
        a = _precondition(rb, ws, 1, budget, restart=4)
        assert np.array_equal(a, b), budget


@pytest.mark.parametrize("fp32", [1, 0])
def test_bottom_solve_identical(rb, fp32):
    import torch
    ws = W.ensemble(5, n_replicas=6, sizes=(16, 24, 32), max_bodies=3)
    print("mgbottom solve fp32", fp32, flush=True)
    outs = []
    for bottom in (24, 0):
        ctx = lib_context(rb, ws, precond_fp32=fp32, mg_bottom=bottom)
        q = dev(np.concatenate([w.q for w in ws]))
        th = dev(np.concatenate([w.theta for w in ws]))
        nb = sum(w.nb for w in ws)
        FT = torch.as_tensor(np.random.default_rng(3).standard_normal((nb, 6)), dtype=torch.float64).cuda()
        U = torch.empty((nb, 6), dtype=torch.float64, device="cuda")
        info = rb.rbfib_solve_mobility(ctx, q, th, FT, U, include_bc=False)
        torch.cuda.synchronize()
        outs.append((U.cpu().numpy(), [i.iters for i in info], [i.status for i in info]))
        ctx.close()
    assert all(s == rb.RBFIB_OK for s in outs[0][2])
    assert outs[0][1] == outs[1][1]
    assert np.array_equal(outs[0][0], outs[1][0])
