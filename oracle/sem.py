"""One Split-Euler-Maruyama (SEM) step with random-finite-difference drift.

Follows Sec. IV and Algorithm 1 of the paper, with these readings where the
printed signs disagree with each other (the chain rule of eq. RFDsplit and
the first term of eq. DriDef carry flipped signs; the correct expansion is
dN = -N (dK^T) M^-1 K N + N K^T M^-1 (dM) M^-1 K N - N K^T M^-1 (dK) N):

  1. W^FT_p = kT [W^f_p / L_p ; W^tau_p], L_p the largest marker-pair distance.
  2. Constrained solve with force W^FT, homogeneous boundary data, no noise:
     U^R = N W^FT, lambda^R = M^-1 K U^R, and v^R = +L^-1 S lambda^R (the fluid
     velocity the solve returns).
  3. q^+- = q +- (delta/2) L_p W^f ; theta^+- = Rotate(theta, +-(delta/2) W^tau).
  4. f# = (1/delta)[S(Q+) - S(Q-)] lambda^R ; unconstrained Stokes solve v# = L^-1 f#.
  5. D^KT = (1/delta)[K^T(Q+) - K^T(Q-)] lambda^R, D^K = (1/delta)[K(Q+) - K(Q-)] U^R,
     D^J = (1/delta)[J(Q+) - J(Q-)] v^R, D^S = J(Q) v#.
  6. Constrained solve with force F - D^KT, slip  slip + D^K - D^J - D^S, and
     fluid forcing sqrt(2 kT eta / (dV dt)) DT W plus the moving-wall terms.
  7. q <- q + dt u ; theta <- Rotate(theta, dt omega).
A step is rejected, and the state left unchanged, when a marker of the new
configuration Q^{n+1} or of one of the displaced configurations Q+- leaves the
open domain along a wall axis (S and J are not defined for a marker outside
the fluid), or when body centres come closer than ``min_body_dist``; the
caller repeats it with fresh random numbers.  A rejected step still returns
the velocities its solves produced.

The random forces and torques of step 1 come from the Philox stream of
(seed, step); ``normals = (W^f, W^tau)`` replaces them with given values (used
to evaluate the drift at chosen directions).  ``drift = False`` sets the random
finite differences of step 5 to zero: the naive Euler-Maruyama scheme whose
bias the paper shows for the boomerang (Appendix A).
"""
from __future__ import annotations

import dataclasses
from typing import Optional

import numpy as np

from . import bodies as B
from . import ib
from . import mac
from . import rng
from .saddle import Saddle


@dataclasses.dataclass
class SEMResult:
    accepted: bool
    q: np.ndarray
    theta: np.ndarray
    U: np.ndarray
    WFT: np.ndarray
    UR: np.ndarray
    lamR: np.ndarray
    DKT: np.ndarray
    DK: np.ndarray
    DJ: np.ndarray
    DS: np.ndarray
    x_final: np.ndarray
    rhs_norms: tuple = ()      # ||b|| of the RFD, unconstrained and final solves


def sem_step(g: mac.Grid, r_ref, offsets, q, theta, FT, kT: float, dt: float, seed: int, step: int,
             delta: float = 1e-5, slip: Optional[np.ndarray] = None, min_body_dist: float = 0.0,
             tol: float = 1e-12, noise: bool = True, normals=None, drift: bool = True) -> SEMResult:
    q = np.asarray(q, dtype=np.float64).reshape(-1, 3)
    theta = np.asarray(theta, dtype=np.float64).reshape(-1, 4)
    nb = q.shape[0]
    FT = np.asarray(FT, dtype=np.float64).reshape(nb, 6)
    Lp = B.body_length(r_ref, offsets)

    # 1. random forces and torques
    if normals is None:
        Wf, Wt = rng.body_normals(seed, step, nb)
    else:
        Wf = np.asarray(normals[0], dtype=np.float64).reshape(nb, 3)
        Wt = np.asarray(normals[1], dtype=np.float64).reshape(nb, 3)
    WFT = np.concatenate([kT * Wf / Lp[:, None], kT * Wt], axis=1)

    # 2. RFD solve at Q^n (homogeneous data)
    s0 = Saddle(g, q, theta, r_ref, offsets)
    b1 = s0.rhs(FT=WFT, include_bc=False)
    xR = s0.solve(b1, tol=tol)
    vR, _, lamR, UR = s0.split(xR)

    # 3. displaced configurations
    qp = q + 0.5 * delta * Lp[:, None] * Wf
    qm = q - 0.5 * delta * Lp[:, None] * Wf
    thp = B.rotate(theta, 0.5 * delta * Wt)
    thm = B.rotate(theta, -0.5 * delta * Wt)
    rp = B.marker_positions(qp, thp, r_ref, offsets)
    rm = B.marker_positions(qm, thm, r_ref, offsets)
    displaced_inside = B.inside_open_domain(g, rp) and B.inside_open_domain(g, rm)

    # 4. unconstrained Stokes solve with the spread difference
    Jp = ib.interpolation(g, rp)
    Jm = ib.interpolation(g, rm)
    fsharp = ((Jp.T @ lamR.ravel()) - (Jm.T @ lamR.ravel())) / (g.dV * delta)
    sf = Saddle(g, q, theta, r_ref, offsets, fluid_only=True)
    b2 = sf.rhs(fluid=fsharp, include_bc=False)
    xs = sf.solve(b2, tol=tol)
    vsharp = xs[sf.sl_v]

    # 5. random finite differences
    DKT = (B.apply_KT(thp, r_ref, offsets, lamR) - B.apply_KT(thm, r_ref, offsets, lamR)) / delta
    DK = (B.apply_K(thp, r_ref, offsets, UR) - B.apply_K(thm, r_ref, offsets, UR)) / delta
    DJ = ((Jp @ vR) - (Jm @ vR)).reshape(-1, 3) / delta
    DS = (s0.J @ vsharp).reshape(-1, 3)

    # 6. velocities with noise and drift
    fluid = None
    if noise and kT > 0.0:
        W = rng.fluid_normals(seed, step, g.nW)
        fluid = mac.noise_stress_divergence(g, W, kT, dt)
    if not drift:
        # naive Euler-Maruyama: the random finite differences are dropped
        DKT, DK, DJ, DS = (np.zeros_like(a) for a in (DKT, DK, DJ, DS))
    slip2 = DK - DJ - DS
    if slip is not None:
        slip2 = slip2 + np.asarray(slip).reshape(-1, 3)
    b3 = s0.rhs(FT=FT - DKT, slip=slip2, fluid=fluid, include_bc=True)
    x = s0.solve(b3, tol=tol)
    U = s0.split(x)[3].copy()

    # 7. update and rejection test
    qn = q + dt * U[:, :3]
    thn = B.rotate(theta, dt * U[:, 3:])
    rn = B.marker_positions(qn, thn, r_ref, offsets)
    ok = displaced_inside and B.inside_open_domain(g, rn)
    if ok and min_body_dist > 0.0 and nb > 1:
        d = np.linalg.norm(qn[:, None, :] - qn[None, :, :], axis=2) + np.eye(nb) * 1e300
        ok = bool(d.min() >= min_body_dist)
    if not ok:
        qn, thn = q.copy(), theta.copy()
    norms = tuple(float(np.linalg.norm(b)) for b in (b1, b2, b3))
    return SEMResult(ok, qn, thn, U, WFT, UR.copy(), lamR.copy(), DKT, DK, DJ, DS, x, norms)


@dataclasses.dataclass
class RK2Result:
    accepted: bool
    q: np.ndarray
    theta: np.ndarray
    U: np.ndarray              # velocities of the corrector (the combination that moved Q^n)
    U_em: np.ndarray           # U^n of Algorithm 1 at Q^n
    U_det0: np.ndarray         # N(Q^n) F(Q^n) with slip and boundary data
    U_det1: np.ndarray         # N(Q*) F(Q*) at the predictor
    q_pred: np.ndarray
    theta_pred: np.ndarray
    em: SEMResult


def sem_rk2_step(g: mac.Grid, r_ref, offsets, q, theta, forces, kT: float, dt: float, seed: int, step: int,
                 alpha: float = 1.0, delta: float = 1e-5, slip: Optional[np.ndarray] = None,
                 slip_pred: Optional[np.ndarray] = None, tol: float = 1e-12, noise: bool = True) -> RK2Result:
    """Deterministically second-order variants of the SEM step (alpha = 1: trapezoidal,
    alpha = 1/2: midpoint).

    The Conclusion names trapezoidal, midpoint and Adams-Bashforth extensions of
    the scheme without writing one out; the reading taken here keeps the random
    part of Algorithm 1 unchanged and treats the deterministic part with the
    two-stage Runge-Kutta rule of predictor fraction alpha:
      1. Algorithm 1 at Q^n with forces F(Q^n) gives U^n (and its rejection test);
      2. U_det^n = N(Q^n) F(Q^n) (with the slip and boundary data, no noise, no drift);
      3. predictor Q* = (q^n + alpha dt u^n, Rotate(theta^n, alpha dt omega^n)) and
         U_det* = N(Q*) F(Q*) (slip_pred at Q*, default slip);
      4. corrector U_c = U^n + (U_det* - U_det^n) / (2 alpha) and
         Q^{n+1} = (q^n + dt u_c, Rotate(theta^n, dt omega_c)).
    With kT = 0, U^n = U_det^n and U_c = (1 - 1/(2 alpha)) U_det^n + U_det* / (2 alpha):
    Heun's method at alpha = 1 and the explicit midpoint rule at alpha = 1/2, both
    second order.  The step is rejected, state untouched, when Algorithm 1 rejects
    its step, or Q* or Q^{n+1} leaves the domain.  ``forces(q, theta)`` returns the
    (nb, 6) forces and torques of a configuration.
    """
    if not (0.0 < alpha <= 1.0):
        raise ValueError("alpha must lie in (0, 1]")
    q = np.asarray(q, dtype=np.float64).reshape(-1, 3)
    theta = np.asarray(theta, dtype=np.float64).reshape(-1, 4)
    F0 = np.asarray(forces(q, theta), dtype=np.float64)
    em = sem_step(g, r_ref, offsets, q, theta, F0, kT, dt, seed, step, delta=delta, slip=slip, tol=tol, noise=noise)
    nb = q.shape[0]
    z = np.zeros((nb, 6))
    qs = q + alpha * dt * em.U[:, :3]
    ths = B.rotate(theta, alpha * dt * em.U[:, 3:])
    if not em.accepted or not B.inside_open_domain(g, B.marker_positions(qs, ths, r_ref, offsets)):
        return RK2Result(False, q.copy(), theta.copy(), z, em.U, z, z, q.copy(), theta.copy(), em)
    s0 = Saddle(g, q, theta, r_ref, offsets)
    Ud0 = s0.split(s0.solve(s0.rhs(FT=F0, slip=slip, include_bc=True), tol=tol))[3].copy()
    F1 = np.asarray(forces(qs, ths), dtype=np.float64)
    s1 = Saddle(g, qs, ths, r_ref, offsets)
    sp = slip if slip_pred is None else slip_pred
    Ud1 = s1.split(s1.solve(s1.rhs(FT=F1, slip=sp, include_bc=True), tol=tol))[3].copy()
    Uc = em.U + (Ud1 - Ud0) / (2.0 * alpha)
    qn = q + dt * Uc[:, :3]
    thn = B.rotate(theta, dt * Uc[:, 3:])
    ok = B.inside_open_domain(g, B.marker_positions(qn, thn, r_ref, offsets))
    if not ok:
        qn, thn = q.copy(), theta.copy()
    return RK2Result(ok, qn, thn, Uc, em.U, Ud0, Ud1, qs, ths, em)


def sem_ab2_step(g: mac.Grid, r_ref, offsets, q, theta, FT, kT: float, dt: float, seed: int, step: int,
                 U_det_prev: Optional[np.ndarray] = None, delta: float = 1e-5, slip: Optional[np.ndarray] = None,
                 tol: float = 1e-12, noise: bool = True):
    """Adams-Bashforth variant of the SEM step (deterministically second order).

    Reading of the Conclusion's Adams-Bashforth extension: Algorithm 1 at Q^n gives
    U^n; the deterministic velocity U_det^n = N(Q^n) F(Q^n) (slip and boundary data,
    no noise, no drift) is extrapolated with the one of the previous step,
    U_c = U^n + (U_det^n - U_det^{n-1}) / 2, and Q^{n+1} = (q^n + dt u_c,
    Rotate(theta^n, dt omega_c)).  Without a previous velocity (the first step)
    U_det^{n-1} = U_det^n, i.e. Algorithm 1 itself.  At kT = 0 this is the two-step
    Adams-Bashforth rule 3/2 f^n - 1/2 f^{n-1}.  Rejection as in Algorithm 1 plus
    Q^{n+1} outside the domain.  Returns (SEMResult of the step, U_det^n) -- the
    SEMResult's U is U_c.
    """
    q = np.asarray(q, dtype=np.float64).reshape(-1, 3)
    theta = np.asarray(theta, dtype=np.float64).reshape(-1, 4)
    em = sem_step(g, r_ref, offsets, q, theta, FT, kT, dt, seed, step, delta=delta, slip=slip, tol=tol, noise=noise)
    s0 = Saddle(g, q, theta, r_ref, offsets)
    Ud = s0.split(s0.solve(s0.rhs(FT=FT, slip=slip, include_bc=True), tol=tol))[3].copy()
    prev = Ud if U_det_prev is None else np.asarray(U_det_prev, dtype=np.float64).reshape(-1, 6)
    Uc = em.U + 0.5 * (Ud - prev)
    qn = q + dt * Uc[:, :3]
    thn = B.rotate(theta, dt * Uc[:, 3:])
    ok = em.accepted and B.inside_open_domain(g, B.marker_positions(qn, thn, r_ref, offsets))
    if not ok:
        qn, thn = q.copy(), theta.copy()
    return dataclasses.replace(em, accepted=ok, q=qn, theta=thn, U=Uc), Ud


def drift_pointwise(g: mac.Grid, r_ref, offsets, q, theta, kT: float, seed: int, step: int,
                    delta: float = 1e-5, tol: float = 1e-12):
    """Brute-force RFD on N itself for the same random draw:
    (1/delta)[N(Q+) - N(Q-)] W^FT, by two constrained solves at Q+ and Q-."""
    q = np.asarray(q, dtype=np.float64).reshape(-1, 3)
    theta = np.asarray(theta, dtype=np.float64).reshape(-1, 4)
    nb = q.shape[0]
    Lp = B.body_length(r_ref, offsets)
    Wf, Wt = rng.body_normals(seed, step, nb)
    WFT = np.concatenate([kT * Wf / Lp[:, None], kT * Wt], axis=1)
    out = []
    for sgn in (1.0, -1.0):
        qs = q + sgn * 0.5 * delta * Lp[:, None] * Wf
        ths = B.rotate(theta, sgn * 0.5 * delta * Wt)
        s = Saddle(g, qs, ths, r_ref, offsets)
        x = s.solve(s.rhs(FT=WFT, include_bc=False), tol=tol)
        out.append(s.split(x)[3])
    return (out[0] - out[1]) / delta
