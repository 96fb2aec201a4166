"""Gradient of a loss of the rigid velocities through the mobility solve.

For U = U(F, Q) from the constrained system A(Q) x = b(F) and a loss L(U):
with U-bar = dL/dU, the adjoint system A^T y = (0, 0, 0, U-bar) is solved with
the same operator (A^T = P A P^-1, P = diag(1, 1, 1/dV, 1/dV)), giving
  y = (v-bar, pi-bar, lambda-bar, U-hat),  U-hat = N U-bar,
and for every configuration coordinate Q_k
  dL/dQ_k = -y^T (d_k A) x
          = (1/dV) lambda.(d_k J) v-bar + lambda-bar.(d_k J) v
            - lambda-bar.(d_k K) U - U-hat.(d_k K^T) lambda ,
while dL/dF = U-hat.  Marker position r_i moves with the body translation
q_p and rotation vector phi_p (r_i -> r_i + phi_p x d_i); K depends only on
d_i = R(theta_p) r_i^ref.  This follows from differentiating eqs. D1-D4 of the
paper; the kernel derivative enters through d phi / d r.
"""
from __future__ import annotations

import numpy as np

from . import bodies as B
from . import ib
from . import mac
from .saddle import Saddle


def loss_sum_sq(U: np.ndarray) -> float:
    return float(np.sum(U * U))


def solve_U(g: mac.Grid, r_ref, offsets, q, theta, FT, tol=1e-12):
    s = Saddle(g, q, theta, r_ref, offsets)
    x = s.solve(s.rhs(FT=FT, include_bc=False), tol=tol)
    return s, x


def mobility_vjp(g: mac.Grid, r_ref, offsets, q, theta, FT, Ubar, tol=1e-12):
    """Returns (dL/dFT [nb,6], dL/dq [nb,3], dL/dphi [nb,3]) for the cotangent Ubar."""
    s, x = solve_U(g, r_ref, offsets, q, theta, FT, tol)
    v, _, lam, U = s.split(x)
    nb = s.nb
    bU = np.zeros(s.n)
    bU[s.sl_u] = g.dV * np.asarray(Ubar).ravel()
    xa = s.solve(bU, tol=tol)
    vbar, _, lam_a, U_a = s.split(xa)
    lam_bar = lam_a / g.dV
    U_hat = U_a / g.dV
    r = s.r
    d = B.marker_offsets(s.theta, s.r_ref, s.offsets)
    body = B.body_of_marker(s.offsets)
    Gi = ib.interpolation_gradient(g, r, v, lam_bar) + ib.interpolation_gradient(g, r, vbar, lam) / g.dV
    Ei = -np.cross(lam_bar, U[body, 3:]) - np.cross(lam, U_hat[body, 3:])
    dq = np.zeros((nb, 3))
    dphi = np.zeros((nb, 3))
    np.add.at(dq, body, Gi)
    np.add.at(dphi, body, np.cross(d, Gi + Ei))
    return U_hat.copy(), dq, dphi


def finite_difference(g: mac.Grid, r_ref, offsets, q, theta, FT, dF, dq, dphi, eps=1e-5, tol=1e-12):
    """Central difference of L = sum U^2 along (dF, dq, rotation dphi)."""
    vals = []
    for sgn in (1.0, -1.0):
        q2 = q + sgn * eps * dq
        th2 = B.rotate(theta, sgn * eps * dphi)
        F2 = FT + sgn * eps * dF
        s, x = solve_U(g, r_ref, offsets, q2, th2, F2, tol)
        vals.append(loss_sum_sq(s.split(x)[3]))
    return (vals[0] - vals[1]) / (2 * eps)
