"""The first two smoother sweeps of a down pass as one kernel against two sweeps.

With mg_first2 = 1 every level with at least two sweeps runs the first sweep from
zero and the second sweep as one launch that rebuilds the first iterate from the
right-hand side: the four-point kernel on FP32 levels whose rows are a multiple of 4
long, the one-point kernel on every other level and on FP64 pools (single-sweep
cycles keep one launch).  The fused sweep computes every value with the same
operations as the two separate ones, so preconditioner outputs and whole FGMRES
solves are identical to the bit: walls on every axis (wall terms of the diagonal at
the first and last points of a row, and at the neighbours whose first iterate is
rebuilt), a periodic x axis (wrapped neighbours), ragged levels, constant and
Chebyshev weights, two and three pressure sweeps, FP64 pools, and the full
256-replica ensemble (four-point levels).
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
        "walls_16x12x20": [W.small_box(23, n=(16, 12, 20), n_bodies=2, R=1.5, shape="ico12")],
        "periodic_x_16x12x12": [per],
        "ragged_10x12x14": [W.small_box(21, n=(10, 12, 14), n_bodies=3, R=1.5, shape="ico12")],
        "monolayer_64x32x16": [W.monolayer(n=(64, 32, 16), rows=4, cols=16)],
        "batch_mixed_depths": W.ensemble(7, n_replicas=8, sizes=(16, 24, 32, 48), max_bodies=2),
    }


CASES = _cases()


def _precondition(rb, ws, first2, seed=11, **kw):
    import torch
    ctx = lib_context(rb, ws, mg_first2=first2, **kw)
    q = dev(np.concatenate([w.q for w in ws]))
    th = dev(np.concatenate([w.theta for w in ws]))
    r = torch.as_tensor(np.random.default_rng(seed).standard_normal(ctx.L), dtype=torch.float64).cuda()
    z = torch.full((ctx.L,), float("nan"), dtype=torch.float64, device="cuda")
    rb.rbfib_precondition(ctx, q, th, r, z)
    torch.cuda.synchronize()
    out = z.cpu().numpy()
    ctx.close()
    return out


@pytest.mark.parametrize("sweeps", [(2, 3), (3, 2), (1, 2)])
@pytest.mark.parametrize("cheby", [0.27, 0.0])
@pytest.mark.parametrize("name", list(CASES))
def test_first2_matches_two_sweeps(rb, name, cheby, sweeps):
    ws = CASES[name]
    print("first2", name, "cheby", cheby, "sweeps", sweeps, flush=True)
    kw = dict(precond_fp32=1, mg_cheby=cheby, mg_sweeps=sweeps[0], mg_sweeps_p=sweeps[1])
    a = _precondition(rb, ws, 1, **kw)
    b = _precondition(rb, ws, 0, **kw)
    assert np.all(np.isfinite(a)) and np.all(np.isfinite(b))
    assert np.array_equal(a, b), float(np.abs(a - b).max() / np.abs(b).max())


def test_first2_fp64_pools(rb):
    ws = CASES["batch_mixed_depths"]
    print("first2 fp64", flush=True)
    assert np.array_equal(_precondition(rb, ws, 1, precond_fp32=0), _precondition(rb, ws, 0, precond_fp32=0))


def test_first2_full_ensemble(rb):
    ws = W.ensemble()
    print("first2 full ensemble", flush=True)
    a = _precondition(rb, ws, 1, precond_fp32=1, restart=4)
    b = _precondition(rb, ws, 0, precond_fp32=1, restart=4)
    assert np.array_equal(a, b)


def test_first2_solve_identical(rb):
    import torch
    ws = W.ensemble(5, n_replicas=6, sizes=(16, 24, 32), max_bodies=3)
    print("first2 solve", flush=True)
    outs = []
    for first2 in (1, 0):
        ctx = lib_context(rb, ws, precond_fp32=1, mg_first2=first2)
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
