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
import pytest

import workloads as W
from oracle import bodies as B
from oracle import mac, rng, sem
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


def _kT_div_N(g, w, kT, eps=1e-4):
    """kT times the divergence of the body mobility with respect to the configuration,
    sum_k d N_{:,k} / d Q_k, by central differences of single columns of the dense N
    (translations of q_p, and lab-frame rotation vectors of theta_p)."""
    nb = w.nb
    div = np.zeros(6 * nb)
    for k in range(6 * nb):
        p, a = divmod(k, 6)
        cols = []
        for sgn in (1.0, -1.0):
            dq = np.zeros((nb, 3))
            dphi = np.zeros((nb, 3))
            if a < 3:
                dq[p, a] = sgn * eps
            else:
                dphi[p, a - 3] = sgn * eps
            s = Saddle(g, w.q + dq, B.rotate(w.theta, dphi), w.r_ref, w.offsets)
            e = np.zeros(6 * nb)
            e[k] = 1.0
            x = s.solve(s.rhs(FT=e.reshape(nb, 6), include_bc=False))
            cols.append(s.split(x)[3].ravel())
        div += (cols[0] - cols[1]) / (2 * eps)
    return kT * div


def test_mean_drift_equals_kT_div_N():
    """The mean of the random-finite-difference drift is kT div_Q N (Sec. IV, eqs. RFD
    and DriDef), independent of how the random force W^FT and the displacement of
    Q+- are scaled individually -- only their product is fixed.  With no deterministic
    force and no fluid noise, the velocity a step returns is the drift alone, a
    quadratic form in the 6 N_b body normals up to O(delta^2); the mean of a quadratic
    form in standard normals is its trace, which the cubature sum over the unit
    vectors W = e_k evaluates exactly.  Two bodies near walls and each other, kT != 1,
    so that a wrong kT, L_p or delta/2 factor, or a dropped cross-body term, fails."""
    w = W.small_box(7, n=(6, 8, 10), n_bodies=2, R=1.0, shape="ico12", gap=0.7)
    g = mac.Grid(w.n, w.bc, w.h, w.eta)
    kT = 2.5
    ref = _kT_div_N(g, w, kT)
    zero = np.zeros((w.nb, 6))
    mean = np.zeros(6 * w.nb)
    for k in range(6 * w.nb):
        e = np.zeros(6 * w.nb)
        e[k] = 1.0
        e = e.reshape(w.nb, 6)
        res = sem.sem_step(g, w.r_ref, w.offsets, w.q, w.theta, zero, kT=kT, dt=0.01, seed=5, step=0,
                           delta=1e-4, noise=False, normals=(e[:, :3], e[:, 3:]))
        mean += res.U.ravel()
    assert np.abs(mean - ref).max() < 1e-5 * np.abs(ref).max()
    # the drift is not small against its own derivative scale: every body moves
    assert np.all(np.abs(ref.reshape(2, 6)[:, :3]).max(axis=1) > 1e-4)


def test_mean_drift_statistical():
    """The same mean over the step's own Philox draws (W^f, W^tau independent
    standard normals): the sample mean of the drift lies within 3 standard errors of
    kT div_Q N in every component.  This exercises the random-number path that the
    cubature check bypasses."""
    w = W.small_box(7, n=(6, 6, 8), n_bodies=1, R=1.0, shape="ico12", gap=0.7)
    g = mac.Grid(w.n, w.bc, w.h, w.eta)
    kT = 2.5
    ref = _kT_div_N(g, w, kT)
    zero = np.zeros((1, 6))
    n = 120
    S = np.array([sem.sem_step(g, w.r_ref, w.offsets, w.q, w.theta, zero, kT=kT, dt=0.01, seed=5, step=k,
                               delta=1e-4, noise=False).U.ravel() for k in range(n)])
    z = (S.mean(axis=0) - ref) / (S.std(axis=0, ddof=1) / np.sqrt(n))
    assert np.all(np.abs(z) < 3.0), z


def test_rejection_on_displaced_configurations():
    """A step whose displaced configuration Q+ or Q- (the random finite difference
    around Q^n) puts a marker outside the fluid is rejected, even when Q^n and Q^{n+1}
    are inside: S and J are not defined there.  A lowest marker 1e-3 h above the wall
    with delta = 0.1 moves by about 0.15 |W^f_z| h, so one of Q+- leaves the domain."""
    w = W.small_box(2, n=(8, 8, 8), n_bodies=1, R=1.5, shape="ico12")
    g = mac.Grid(w.n, w.bc, w.h, w.eta)
    r0 = B.marker_positions(w.q, w.theta, w.r_ref, w.offsets)
    q = w.q.copy()
    q[0, 2] += 1e-3 - r0[:, 2].min()
    zero = np.zeros((1, 6))
    res = sem.sem_step(g, w.r_ref, w.offsets, q, w.theta, zero, kT=1.0, dt=1e-6, seed=3, step=0, delta=0.1,
                       noise=False)
    Wf, _ = rng.body_normals(3, 0, 1)
    assert abs(Wf[0, 2]) > 0.05                  # the draw does push one side through the wall
    assert not res.accepted
    assert np.array_equal(res.q, q) and np.array_equal(res.theta, w.theta)
    # the same configuration with a small delta keeps Q+- inside and is accepted
    res = sem.sem_step(g, w.r_ref, w.offsets, q, w.theta, zero, kT=1.0, dt=1e-6, seed=3, step=0, delta=1e-6,
                       noise=False)
    assert res.accepted


def _trap_case():
    from oracle.potentials import body_forces
    g = mac.Grid((6, 6, 8), (mac.WALL, mac.WALL, mac.WALL), 1.0, 1.0)
    r_ref = W.icosahedron(1.0)
    offs = np.array([0, 12], dtype=np.int32)
    q0 = np.array([[3.1, 2.9, 2.1]])
    th0 = W.random_unit_quaternions(np.random.default_rng(3), 1)
    F = lambda q, th: body_forces(g, q, th, r_ref, offs, 4.0, 1.0, 0.25, [0.03, 0.01, -0.05])
    return g, r_ref, offs, q0, th0, F


@pytest.mark.parametrize("alpha", [1.0, 0.5])
def test_rk2_second_order_deterministic(alpha):
    """kT = 0: a body settling onto a wall under its weight and the wall repulsion
    (translation and rotation couple through the wall).  Differences between runs
    with 2, 4 and 8 steps over the same time shrink by 4 per halving for the
    trapezoidal (alpha = 1) and midpoint (alpha = 1/2) variants (second order) and
    by 2 for Algorithm 1 (Euler)."""
    g, r_ref, offs, q0, th0, F = _trap_case()
    T = 4.0

    def run(n, trap):
        q, th = q0.copy(), th0.copy()
        for k in range(n):
            if trap:
                r = sem.sem_rk2_step(g, r_ref, offs, q, th, F, 0.0, T / n, 1, k, alpha=alpha)
            else:
                r = sem.sem_step(g, r_ref, offs, q, th, F(q, th), 0.0, T / n, 1, k)
            assert r.accepted
            q, th = r.q, r.theta
        return q, th

    def d(a, b):
        return np.abs(a[0] - b[0]).max() + np.abs(B.rotation_matrices(a[1]) - B.rotation_matrices(b[1])).max()

    for trap, lo, hi in ((False, 1.6, 2.6), (True, 3.2, 5.0)):
        Q = [run(n, trap) for n in (2, 4, 8)]
        ratio = d(Q[0], Q[1]) / d(Q[1], Q[2])
        assert lo < ratio < hi, (trap, alpha, ratio)
    # the body moved: the test is not trivially satisfied
    assert np.abs(Q[2][0] - q0).max() > 0.05


@pytest.mark.parametrize("alpha", [1.0, 0.5])
def test_rk2_pieces_and_rejection(alpha):
    """With noise: the predictor is the Euler-Maruyama update of Algorithm 1 at the
    same random numbers, the corrector adds half the change of the deterministic
    velocity, and a predictor outside the domain rejects the step untouched."""
    g, r_ref, offs, q0, th0, F = _trap_case()
    r = sem.sem_rk2_step(g, r_ref, offs, q0, th0, F, 1.0, 0.05, 4, 2, alpha=alpha)
    em = sem.sem_step(g, r_ref, offs, q0, th0, F(q0, th0), 1.0, 0.05, 4, 2)
    assert r.accepted and em.accepted
    assert np.allclose(r.U_em, em.U, rtol=0, atol=1e-12)
    assert np.allclose(r.q_pred, q0 + alpha * 0.05 * em.U[:, :3], rtol=0, atol=1e-12)
    if alpha == 1.0:
        assert np.allclose(r.q_pred, em.q, rtol=0, atol=1e-12)
    assert np.allclose(r.U, em.U + (r.U_det1 - r.U_det0) / (2 * alpha), rtol=0, atol=1e-15)
    assert np.allclose(r.q, q0 + 0.05 * r.U[:, :3], rtol=0, atol=1e-15)
    # a huge step pushes the predictor through the wall: rejected, state untouched
    big = lambda q, th: F(q, th) + np.array([0.0, 0.0, -500.0, 0.0, 0.0, 0.0])
    r2 = sem.sem_rk2_step(g, r_ref, offs, q0, th0, big, 0.0, 10.0, 4, 2, alpha=alpha)
    assert not r2.accepted and np.array_equal(r2.q, q0) and np.array_equal(r2.theta, th0)


def test_ab2_second_order_deterministic():
    """kT = 0: the Adams-Bashforth variant (started by one Algorithm 1 step) on the
    settling body: differences shrink by about 4 per halving of the step."""
    g, r_ref, offs, q0, th0, F = _trap_case()
    T = 4.0

    def run(n):
        q, th, prev = q0.copy(), th0.copy(), None
        for k in range(n):
            r, prev = sem.sem_ab2_step(g, r_ref, offs, q, th, F(q, th), 0.0, T / n, 1, k, U_det_prev=prev)
            assert r.accepted
            q, th = r.q, r.theta
        return q, th

    def d(a, b):
        return np.abs(a[0] - b[0]).max() + np.abs(B.rotation_matrices(a[1]) - B.rotation_matrices(b[1])).max()

    Q = [run(n) for n in (4, 8, 16)]
    ratio = d(Q[0], Q[1]) / d(Q[1], Q[2])
    assert 3.2 < ratio < 5.0, ratio


def test_ab2_pieces():
    """With noise: without a previous velocity the step is Algorithm 1's; with one,
    U_c = U^n + (U_det^n - U_det^{n-1})/2 at the same random numbers."""
    g, r_ref, offs, q0, th0, F = _trap_case()
    em = sem.sem_step(g, r_ref, offs, q0, th0, F(q0, th0), 1.0, 0.05, 4, 2)
    r0, Ud = sem.sem_ab2_step(g, r_ref, offs, q0, th0, F(q0, th0), 1.0, 0.05, 4, 2)
    assert np.allclose(r0.U, em.U, rtol=0, atol=1e-12) and np.allclose(r0.q, em.q, rtol=0, atol=1e-12)
    prev = Ud + 0.01
    r1, _ = sem.sem_ab2_step(g, r_ref, offs, q0, th0, F(q0, th0), 1.0, 0.05, 4, 2, U_det_prev=prev)
    assert np.allclose(r1.U, em.U + 0.5 * (Ud - prev), rtol=0, atol=1e-12)
