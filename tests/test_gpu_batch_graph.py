"""Batched replicas and captured-graph replay, through the C ABI.

* Replicas of different grid sizes and body counts solved in one batched
  context give the same U, bit for bit, as each replica solved alone: every
  replica keeps its own Krylov recurrence (per-replica dots, Givens state and
  convergence mask), so batching changes only how launches are shared.
* A batched SEM step equals the per-replica steps (replica r draws seed + r).
* The FGMRES iterations replayed from captured HIP graphs give bit-identical
  results to eager launches, over several replays with eager work and
  synchronisation in between.

The per-replica dot products sum Krylov chunks in a fixed order, so a batch and
its replicas agree bit for bit when they use the same Krylov chunk; the launch-
geometry table may choose different chunks for a large batch and a single box,
so every context here is created under one forced table (the multigrid points
per thread keep their size rule: four on the 10.9M-cell batch, one alone).
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


@pytest.fixture(autouse=True)
def one_geometry(tmp_path):
    import os
    p = tmp_path / "tuning.txt"
    p.write_text("# one launch geometry for batches and single replicas\n"
                 "0 9223372036854775807 1 1000000 1024 16384 32 0 0\n")
    old = os.environ.get("RBFIB_TUNING")
    os.environ["RBFIB_TUNING"] = str(p)
    yield
    if old is None:
        os.environ.pop("RBFIB_TUNING", None)
    else:
        os.environ["RBFIB_TUNING"] = old


def _replicas():
    return [W.spheres_in_box(101, (16, 16, 16), 1, name="r0"),
            W.spheres_in_box(102, (24, 24, 24), 3, name="r1"),
            W.spheres_in_box(103, (32, 32, 32), 2, name="r2"),
            W.spheres_in_box(104, (16, 16, 16), 4, R=1.5, shape="ico12", name="r3")]


def _cat(arrs):
    return np.concatenate([np.asarray(a) for a in arrs], axis=0)


@pytest.mark.parametrize("fp32", [0, 1])
def test_batched_solve_equals_individual(rb, fp32):
    import torch
    reps = _replicas()
    ctx = lib_context(rb, reps, tol=1e-8, precond_fp32=fp32)
    U = torch.empty((sum(w.nb for w in reps), 6), dtype=torch.float64, device="cuda")
    info = rb.rbfib_solve_mobility(ctx, dev(_cat([w.q for w in reps])), dev(_cat([w.theta for w in reps])),
                                   dev(_cat([w.FT for w in reps])), U, allow=())
    Ub = U.cpu().numpy()
    ctx.close()
    b0 = 0
    for r, w in enumerate(reps):
        c1 = lib_context(rb, w, tol=1e-8, precond_fp32=fp32)
        U1 = torch.empty((w.nb, 6), dtype=torch.float64, device="cuda")
        i1 = rb.rbfib_solve_mobility(c1, dev(w.q), dev(w.theta), dev(w.FT), U1, allow=())
        print("replica", r, "batched iters", info[r].iters, "alone", i1[0].iters, flush=True)
        assert info[r].iters == i1[0].iters
        assert np.array_equal(Ub[b0:b0 + w.nb], U1.cpu().numpy())
        b0 += w.nb
        c1.close()


def test_batched_sem_step_equals_individual(rb):
    import torch
    reps = _replicas()
    ctx = lib_context(rb, reps, tol=1e-8, precond_fp32=1)
    q = dev(_cat([w.q for w in reps]))
    th = dev(_cat([w.theta for w in reps]))
    nb = sum(w.nb for w in reps)
    U = torch.empty((nb, 6), dtype=torch.float64, device="cuda")
    rb.rbfib_sem_step(ctx, q, th, dev(_cat([w.FT for w in reps])), 1.0, 0.01, 900, 2, U, allow=())
    qb, Ub = q.cpu().numpy(), U.cpu().numpy()
    ctx.close()
    b0 = 0
    for r, w in enumerate(reps):
        c1 = lib_context(rb, w, tol=1e-8, precond_fp32=1)
        q1, th1 = dev(w.q), dev(w.theta)
        U1 = torch.empty((w.nb, 6), dtype=torch.float64, device="cuda")
        rb.rbfib_sem_step(c1, q1, th1, dev(w.FT), 1.0, 0.01, 900 + r, 2, U1, allow=())
        assert np.array_equal(Ub[b0:b0 + w.nb], U1.cpu().numpy())
        assert np.array_equal(qb[b0:b0 + w.nb], q1.cpu().numpy())
        b0 += w.nb
        c1.close()


def test_graph_replay_matches_eager(rb):
    import torch
    w = W.two_spheres()
    cg = lib_context(rb, w, tol=1e-7, use_graphs=1)
    ce = lib_context(rb, w, tol=1e-7, use_graphs=0)
    q, th = dev(w.q), dev(w.theta)
    Ue = torch.empty((w.nb, 6), dtype=torch.float64, device="cuda")
    rb.rbfib_solve_mobility(ce, q, th, dev(w.FT), Ue, allow=())
    ref = Ue.cpu().numpy()
    rng = np.random.default_rng(3)
    for k in range(4):
        Ug = torch.empty((w.nb, 6), dtype=torch.float64, device="cuda")
        rb.rbfib_solve_mobility(cg, q, th, dev(w.FT), Ug, allow=())
        torch.cuda.synchronize()
        assert np.array_equal(Ug.cpu().numpy(), ref), k
        # eager work between replays: a different right-hand side through the eager context
        tmp = torch.empty_like(Ue)
        rb.rbfib_solve_mobility(ce, q, th, dev(rng.standard_normal((w.nb, 6))), tmp, allow=())
        torch.cuda.synchronize()
    # a different right-hand side and configuration through the same graphs
    F2 = rng.standard_normal((w.nb, 6))
    q2 = w.q + 0.3
    Ug = torch.empty_like(Ue)
    Ue2 = torch.empty_like(Ue)
    rb.rbfib_solve_mobility(cg, dev(q2), th, dev(F2), Ug, allow=())
    rb.rbfib_solve_mobility(ce, dev(q2), th, dev(F2), Ue2, allow=())
    assert np.array_equal(Ug.cpu().numpy(), Ue2.cpu().numpy())
    cg.close()
    ce.close()


@pytest.mark.parametrize("fp32", [1, 0])
def test_large_batch_paths_equal_single_replica(rb, fp32):
    """The 256-replica ensemble (10.9M cells) runs the grid kernels with four points
    per thread (the FP32 smoother on aligned groups of four x points); single
    replicas run one point per thread.  Preconditioner outputs and full solves agree
    bit for bit on the replicas' segments."""
    import torch
    ens = W.ensemble()
    picks = [0, 1, 2, 3, 100, 255]
    ctx = lib_context(rb, ens, tol=1e-6, precond_fp32=fp32)
    q = dev(_cat([w.q for w in ens]))
    th = dev(_cat([w.theta for w in ens]))
    r = torch.as_tensor(np.random.default_rng(31).standard_normal(ctx.L), dtype=torch.float64).cuda()
    z = torch.full_like(r, float("nan"))
    rb.rbfib_precondition(ctx, q, th, r, z)
    U = torch.empty((sum(w.nb for w in ens), 6), dtype=torch.float64, device="cuda")
    info = rb.rbfib_solve_mobility(ctx, q, th, dev(_cat([w.FT for w in ens])), U, allow=())
    torch.cuda.synchronize()
    zb, Ub, lay = z.cpu().numpy(), U.cpu().numpy(), ctx.layout.copy()
    ctx.close()
    body0 = np.cumsum([0] + [w.nb for w in ens])
    for k in picks:
        w = ens[k]
        a, e = int(lay[k][0]), int(lay[k][3]) + 6 * w.nb
        c1 = lib_context(rb, w, tol=1e-6, precond_fp32=fp32)
        assert c1.L == e - a
        z1 = torch.full((c1.L,), float("nan"), dtype=torch.float64, device="cuda")
        rb.rbfib_precondition(c1, dev(w.q), dev(w.theta), r[a:e].contiguous(), z1)
        U1 = torch.empty((w.nb, 6), dtype=torch.float64, device="cuda")
        i1 = rb.rbfib_solve_mobility(c1, dev(w.q), dev(w.theta), dev(w.FT), U1, allow=())
        torch.cuda.synchronize()
        print("replica", k, w.n, "iters batched", info[k].iters, "alone", i1[0].iters, flush=True)
        assert np.array_equal(zb[a:e], z1.cpu().numpy())
        assert info[k].iters == i1[0].iters
        assert np.array_equal(Ub[body0[k]:body0[k + 1]], U1.cpu().numpy())
        c1.close()
