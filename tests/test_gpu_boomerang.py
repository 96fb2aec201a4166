"""GPU parity for the App. A boomerang in its 64x64x16 slit (6-point kernel).

* rbfib_body_forces against the oracle's forces and torques: the soft
  blob-wall repulsion of eq. Usoft on both walls (exponential and linear
  ranges) plus the buoyant weight of every blob, for single boomerangs and a
  batch of replicas;
* one Split-Euler-Maruyama step driven by those forces, with the random
  finite differences (Algorithm 1) and without them (the naive scheme whose
  equilibrium App. A shows to be biased), against the oracle's step at the
  same seed: U^n within the bound that the GPU's solve residuals imply;
* a short ensemble run: with the drift the boomerangs keep their
  Gibbs-Boltzmann distance to the walls, without it they drift towards them;
  so do the midpoint and Adams-Bashforth variants of the step (with noise).
"""
import numpy as np
import pytest

import workloads as W
from oracle import sem
from oracle.potentials import body_forces
from tests.helpers import dev, lib_context, oracle_grid, sem_error_bound
from tests.parity_configs import boomerang_configs

pytestmark = pytest.mark.gpu

POT = W.BOOMERANG_POTENTIAL
FCONST = [0.0, 0.0, -POT["weight"]]


@pytest.fixture(scope="module")
def rb():
    import paper_1901_06427_amd as rb
    return rb


def _oracle_forces(w):
    return body_forces(oracle_grid(w), w.q, w.theta, w.r_ref, w.offsets, POT["phi0"], POT["d"], POT["b"], FCONST)


def _gpu_forces(rb, ctx, q, th, nb):
    import torch
    FT = torch.full((nb, 6), float("nan"), dtype=torch.float64, device="cuda")
    rb.rbfib_body_forces(ctx, q, th, POT["phi0"], POT["d"], POT["b"], FCONST, FT)
    torch.cuda.synchronize()
    return FT


@pytest.mark.parametrize("name", list(boomerang_configs()))
def test_body_forces_match_oracle(rb, name):
    print("forces", name, flush=True)
    w = boomerang_configs()[name]
    ctx = lib_context(rb, w, tol=1e-6)
    FT = _gpu_forces(rb, ctx, dev(w.q), dev(w.theta), w.nb).cpu().numpy()
    ref = _oracle_forces(w)
    scale = np.abs(ref).max()
    assert scale > 10.0                                  # the wall repulsion is active
    assert np.abs(FT - ref).max() <= 1e-13 * scale, (FT, ref)
    ctx.close()


def test_body_forces_batch(rb):
    """A batch of replicas at seeded heights and orientations (some blobs in the
    linear range of either wall) against the oracle replica by replica."""
    print("forces batch", flush=True)
    rng = np.random.default_rng(8)
    ws = W.boomerang_slit(seed=9, n_replicas=12)
    for w in ws:
        while True:
            t = rng.standard_normal(4)
            t /= np.linalg.norm(t)
            w.theta = t[None, :]
            w.q = np.array([[w.q[0, 0], w.q[0, 1], rng.uniform(0.5, 15.5)]])
            from oracle.bodies import marker_positions
            z = marker_positions(w.q, w.theta, w.r_ref, w.offsets)[:, 2]
            if z.min() > 0.3 and z.max() < 15.7:
                break
    ctx = lib_context(rb, ws, tol=1e-6)
    q = dev(np.concatenate([w.q for w in ws]))
    th = dev(np.concatenate([w.theta for w in ws]))
    FT = _gpu_forces(rb, ctx, q, th, len(ws)).cpu().numpy()
    ref = np.concatenate([_oracle_forces(w) for w in ws])
    assert np.abs(FT - ref).max() <= 1e-13 * np.abs(ref).max()
    ctx.close()


def test_body_forces_rejects_bad_parameters(rb):
    w = boomerang_configs()["boomerang_64x64x16_k6"]
    ctx = lib_context(rb, w, tol=1e-6)
    import torch
    FT = torch.zeros((1, 6), dtype=torch.float64, device="cuda")
    with pytest.raises(rb.RBFIBError):
        rb.rbfib_body_forces(ctx, dev(w.q), dev(w.theta), 4.0, 1.47, 0.0, FCONST, FT)
    with pytest.raises(rb.RBFIBError):
        rb.rbfib_body_forces(ctx, dev(w.q), dev(w.theta), float("nan"), 1.47, 0.1, FCONST, FT)
    ctx.close()


@pytest.mark.parametrize("drift", [True, False])
def test_boomerang_sem_step_matches_oracle(rb, drift):
    import torch
    name = "boomerang_64x64x16_k6"
    print("boomerang sem drift", drift, flush=True)
    w = boomerang_configs()[name]
    tol, kT, dt, seed, step = 1e-11, 1.0, W.boomerang_dt(0.036), 77, 3
    ctx = lib_context(rb, w, tol=tol, precond_fp32=1, max_iter=600, no_drift=0 if drift else 1)
    q, th = dev(w.q), dev(w.theta)
    FT = _gpu_forces(rb, ctx, q, th, w.nb)
    U = torch.empty((w.nb, 6), dtype=torch.float64, device="cuda")
    info = rb.rbfib_sem_step(ctx, q, th, FT, kT, dt, seed, step, U, allow=())
    torch.cuda.synchronize()
    print("  iters", info[0].iters, "res", info[0].rel_residual, flush=True)
    ref = sem.sem_step(oracle_grid(w), w.r_ref, w.offsets, w.q, w.theta, _oracle_forces(w), kT, dt, seed, step,
                       drift=drift)
    assert ref.accepted
    bound = sem_error_bound(name, ref.rhs_norms, tol, info[0].rel_residual)
    err = np.abs(U.cpu().numpy() - ref.U)
    print("  max err / bound %.3f" % (err / bound).max(), flush=True)
    assert np.all(err <= bound)
    assert np.abs(q.cpu().numpy() - ref.q).max() <= dt * err.max() + 1e-13
    ctx.close()


def test_drift_changes_the_step(rb):
    """Same seed with and without the drift: the random finite differences move
    U by far more than the solve tolerance (the drift is not silently zero)."""
    import torch
    w = boomerang_configs()["boomerang_64x64x16_k6"]
    out = []
    for nd in (0, 1):
        ctx = lib_context(rb, w, tol=1e-10, precond_fp32=1, no_drift=nd)
        q, th = dev(w.q), dev(w.theta)
        FT = _gpu_forces(rb, ctx, q, th, w.nb)
        U = torch.empty((w.nb, 6), dtype=torch.float64, device="cuda")
        rb.rbfib_sem_step(ctx, q, th, FT, 1.0, W.boomerang_dt(0.036), 5, 1, U, allow=())
        torch.cuda.synchronize()
        out.append(U.cpu().numpy())
        ctx.close()
    assert np.abs(out[0] - out[1]).max() > 1e-4 * np.abs(out[0]).max()


def test_drift_removes_wall_bias(rb):
    """End to end (App. A): 256 boomerangs from exact Gibbs-Boltzmann draws, 100 SEM
    steps at dtau = 0.14.  With the random finite differences the fraction of time the
    cross point spends within 3h of a wall stays at its Gibbs-Boltzmann value (0.160,
    tests/golden/boomerang_gb.json); the naive scheme without the drift drives it to
    about 0.29 within 50 steps.  Measured over steps 50-99 (long runs:
    0.159 +- 0.005 with the drift, 0.335 +- 0.005 without)."""
    import json
    import os
    import torch
    from tests.boomerang_study import initial_state
    ref = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "boomerang_gb.json")))
    ze = np.asarray(ref["z_edges"])
    zc = 0.5 * (ze[1:] + ze[:-1])
    p_ref = float(np.sum(np.asarray(ref["p_height"])[(zc < 3) | (zc > 13)]))
    R, dtau = 256, 0.14
    frac = {}
    for nd in (0, 1):
        print("boomerang ensemble, no_drift", nd, flush=True)
        ws = W.boomerang_slit(seed=5, n_replicas=R, dtau=dtau, tol=1e-5)
        ctx = lib_context(rb, ws, tol=1e-5, precond_fp32=1, no_drift=nd)
        q0, th0 = initial_state(R, 77)
        q, th = dev(q0), dev(th0)
        FT = torch.empty((R, 6), dtype=torch.float64, device="cuda")
        U = torch.empty_like(FT)
        near = []
        for k in range(100):
            rb.rbfib_body_forces(ctx, q, th, POT["phi0"], POT["d"], POT["b"], FCONST, FT)
            rb.rbfib_sem_step(ctx, q, th, FT, 1.0, W.boomerang_dt(dtau), 9, k, U, allow=(rb.RBFIB_EREJECT,))
            if k >= 50:
                z = q[:, 2].cpu().numpy()
                near.append(np.mean((z < 3.0) | (z > 13.0)))
        ctx.close()
        frac[nd] = float(np.mean(near))
        print("  wall fraction %.3f (Gibbs-Boltzmann %.3f)" % (frac[nd], p_ref), flush=True)
    assert abs(frac[0] - p_ref) < 0.04
    assert frac[1] > p_ref + 0.06


@pytest.mark.parametrize("scheme", ["mid", "ab2"])
def test_second_order_variants_keep_gibbs_boltzmann(rb, scheme):
    """The deterministically second-order variants of the SEM step (the two-stage
    family at alpha = 1/2, with the forces evaluated again at the predictor, and the
    Adams-Bashforth extrapolation) with noise: 256 boomerangs from exact
    Gibbs-Boltzmann draws, 100 steps at dtau = 0.14; the fraction of time the cross
    point spends within 3h of a wall stays at its Gibbs-Boltzmann value (0.160).
    Long runs of 512 replicas x 1000 steps: 0.166 +- 0.004 (midpoint), 0.153 +- 0.004
    (Adams-Bashforth)."""
    import json
    import os
    import torch
    from tests.boomerang_study import initial_state
    ref = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "boomerang_gb.json")))
    ze = np.asarray(ref["z_edges"])
    zc = 0.5 * (ze[1:] + ze[:-1])
    p_ref = float(np.sum(np.asarray(ref["p_height"])[(zc < 3) | (zc > 13)]))
    R, dtau = 256, 0.14
    dt = W.boomerang_dt(dtau)
    print("boomerang ensemble, scheme", scheme, flush=True)
    ws = W.boomerang_slit(seed=5, n_replicas=R, dtau=dtau, tol=1e-5)
    ctx = lib_context(rb, ws, tol=1e-5, precond_fp32=1)
    q0, th0 = initial_state(R, 78)
    q, th = dev(q0), dev(th0)
    FT = torch.empty((R, 6), dtype=torch.float64, device="cuda")
    U = torch.empty_like(FT)
    qp, thp, FTp, Udp = torch.empty_like(q), torch.empty_like(th), torch.empty_like(FT), torch.zeros_like(FT)
    allow = (rb.RBFIB_EREJECT,)
    near = []
    for k in range(100):
        rb.rbfib_body_forces(ctx, q, th, POT["phi0"], POT["d"], POT["b"], FCONST, FT)
        if scheme == "ab2":
            rb.rbfib_sem_ab2_step(ctx, q, th, FT, 1.0, dt, 9, k, Udp, k > 0, U, allow=allow)
        else:
            rb.rbfib_sem_rk2_predict(ctx, q, th, FT, 1.0, dt, 9, k, qp, thp, alpha=0.5, allow=allow)
            rb.rbfib_body_forces(ctx, qp, thp, POT["phi0"], POT["d"], POT["b"], FCONST, FTp)
            rb.rbfib_sem_rk2_correct(ctx, q, th, FTp, U, allow=allow)
        if k >= 30:
            z = q[:, 2].cpu().numpy()
            near.append(np.mean((z < 3.0) | (z > 13.0)))
    ctx.close()
    frac = float(np.mean(near))
    print("  wall fraction %.3f (Gibbs-Boltzmann %.3f)" % (frac, p_ref), flush=True)
    assert abs(frac - p_ref) < 0.04
