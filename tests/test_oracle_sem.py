"""Pins of the oracle's SEM step (paper Sec. IV, Algorithm 1, Appendix).

* Pointwise drift: for one random draw, the extra velocity produced by the
  RFD terms equals the random finite difference of N itself,
  (1/delta)[N(Q+) - N(Q-)] W^FT, up to O(delta^2) -- this catches any sign
  slip among D^KT, D^K, D^J and D^S.
* Discrete fluctuation-dissipation balance: the linear map B from the noise
  W to the Brownian body velocity satisfies dt B B^T = 2 kT N exactly
  (N assembled by separate solves), which holds only if DT DT^T = -Lm and the
  noise amplitude is sqrt(2 kT eta / (dV dt)).
* A step that would push a marker through a wall is rejected and leaves the
  state unchanged.
"""
import numpy as np

import workloads as W
from oracle import bodies as B
from oracle import mac, sem
from oracle.saddle import Saddle


def test_drift_pointwise_matches_rfd_on_N():
    w = W.small_box(3, n=(10, 10, 12), n_bodies=2, R=1.5, shape="ico12")
    g = mac.Grid(w.n, w.bc, w.h, w.eta)
    zero = np.zeros((2, 6))
    for step, delta in ((0, 1e-4), (1, 1e-3)):
        res = sem.sem_step(g, w.r_ref, w.offsets, w.q, w.theta, zero, kT=1.0, dt=0.01, seed=11,
                           step=step, delta=delta, noise=False)
        ref = sem.drift_pointwise(g, w.r_ref, w.offsets, w.q, w.theta, kT=1.0, seed=11, step=step,
                                  delta=delta)
        err = np.abs(res.U - ref).max() / np.abs(ref).max()
        assert err < 50 * delta ** 2 + 1e-7, (delta, err)
    # without the drift terms the velocity would be zero (F = 0, no noise)
    assert np.abs(res.U).max() > 1e-4


def test_discrete_fdb():
    w = W.small_box(6, n=(8, 8, 8), n_bodies=1, R=1.5, shape="ico12")
    g = mac.Grid(w.n, w.bc, 1.0, 1.3)
    s = Saddle(g, w.q, w.theta, w.r_ref, w.offsets)
    kT, dt = 0.7, 0.05
    N = np.zeros((6, 6))
    T = np.zeros((6, g.nv))
    for k in range(6):
        e = np.zeros(6)
        e[k] = 1.0
        x = s.solve(s.rhs(FT=e, include_bc=False))
        N[:, k] = s.split(x)[3].ravel()
        T[k] = x[s.sl_v]                 # A is symmetric at h = 1: row k of the map f -> U
    DT = mac.tensor_divergence(g).toarray()
    scale = np.sqrt(2 * kT * g.eta / (g.dV * dt))
    Bm = scale * T @ DT
    lhs = dt * Bm @ Bm.T
    assert np.abs(lhs - 2 * kT * N).max() < 1e-9 * np.abs(N).max()
    # and the map really is the one a noise solve applies
    rng = np.random.default_rng(1)
    Wn = rng.standard_normal(g.nW)
    x = s.solve(s.rhs(fluid=mac.noise_stress_divergence(g, Wn, kT, dt), include_bc=False))
    assert np.abs(s.split(x)[3].ravel() - Bm @ Wn).max() < 1e-9 * np.abs(Bm @ Wn).max()


def test_rejection_leaves_state():
    w = W.small_box(2, n=(8, 8, 8), n_bodies=1, R=1.5, shape="ico12")
    g = mac.Grid(w.n, w.bc, w.h, w.eta)
    q = np.array([[4.0, 4.0, 2.0]])
    F = np.array([[0.0, 0.0, -1e5, 0.0, 0.0, 0.0]])
    res = sem.sem_step(g, w.r_ref, w.offsets, q, w.theta, F, kT=1.0, dt=1.0, seed=1, step=0)
    assert not res.accepted
    assert np.array_equal(res.q, q) and np.array_equal(res.theta, w.theta)
    res = sem.sem_step(g, w.r_ref, w.offsets, q, w.theta, F * 0, kT=1.0, dt=1e-3, seed=1, step=0)
    assert res.accepted
    assert not np.array_equal(res.q, q)
