"""Conservative forces of the paper's test problems, in FP64.

Test infrastructure: only the tests, the smoke check and the benchmark's CPU
leg use this package.

The paper drives its confined suspensions with caller-side forces that enter
the saddle system as the body forces and torques F (Algorithm 1).  Two kinds
are written out here:

  * the soft repulsion of eq. Usoft between a marker and a wall face at
    distance r,  Phi(r) = Phi0 (1 + (d - r)/b) for r < d and
    Phi0 exp((d - r)/b) for r >= d  (Sec. V.A; App. A uses it between every
    blob and both walls of the slit, with d = a, the blob radius);
  * a constant force on every marker, such as the buoyant weight -m_e g z-hat
    of each blob of the boomerang (App. A).

The energy of a configuration is the sum over markers and over the two faces
of every non-periodic axis; marker i of body p sits at r_i = q_p + R(theta_p)
r_i^ref.  The force on a marker is minus the gradient of its energy, and a
body receives F_p = sum_i f_i and T_p = sum_i d_i x f_i (d_i = R r_i^ref,
torque about the tracking point q_p), which is minus the derivative of the
energy under translation and under a lab-frame rotation of the body.

Parity pins: the tests check the piecewise profile against its closed-form
properties (value Phi0 and slope -Phi0/b from both sides at r = d, value
Phi0/2 at r = d + b ln 2, value Phi0 (1 + d/b) at the face) and the forces
and torques against central differences of the energy under translations and
rotations.
"""
from __future__ import annotations

import numpy as np

from .bodies import marker_offsets, body_of_marker
from .mac import Grid, PERIODIC


def soft_profile(r: np.ndarray, phi0: float, d: float, b: float):
    """(Phi(r), Phi'(r)) of eq. Usoft: linear inside r < d, exponential tail beyond."""
    r = np.asarray(r, dtype=np.float64)
    inner = r < d
    e = np.exp(np.minimum((d - r) / b, 0.0))
    val = np.where(inner, phi0 * (1.0 + (d - r) / b), phi0 * e)
    der = np.where(inner, -phi0 / b, -phi0 / b * e)
    return val, der


def marker_energy_forces(g: Grid, r: np.ndarray, phi0: float, d: float, b: float, fconst):
    """Per-marker energy and force (nm,), (nm, 3) at marker positions r (nm, 3).

    The constant force fconst contributes energy -fconst . r (a uniform field).
    """
    r = np.asarray(r, dtype=np.float64)
    fc = np.asarray(fconst, dtype=np.float64)
    energy = -(r @ fc)
    force = np.tile(fc, (r.shape[0], 1))
    for a in range(3):
        if g.bc[a] == PERIODIC:
            continue
        L = g.n[a] * g.h
        v_lo, d_lo = soft_profile(r[:, a], phi0, d, b)          # distance to the face x_a = 0
        v_hi, d_hi = soft_profile(L - r[:, a], phi0, d, b)      # distance to the face x_a = L
        energy = energy + v_lo + v_hi
        force[:, a] += -d_lo + d_hi
    return energy, force


def body_energy(g: Grid, q, theta, r_ref, offsets, phi0, d, b, fconst) -> np.ndarray:
    """Energy of each body (nb,)."""
    r = q[body_of_marker(offsets)] + marker_offsets(theta, r_ref, offsets)
    e, _ = marker_energy_forces(g, r, phi0, d, b, fconst)
    out = np.zeros(len(offsets) - 1)
    np.add.at(out, body_of_marker(offsets), e)
    return out


def body_forces(g: Grid, q, theta, r_ref, offsets, phi0, d, b, fconst) -> np.ndarray:
    """F_p = sum_i f_i, T_p = sum_i d_i x f_i  (nb, 6)."""
    body = body_of_marker(offsets)
    dd = marker_offsets(theta, r_ref, offsets)
    r = q[body] + dd
    _, f = marker_energy_forces(g, r, phi0, d, b, fconst)
    out = np.zeros((len(offsets) - 1, 6))
    np.add.at(out[:, :3], body, f)
    np.add.at(out[:, 3:], body, np.cross(dd, f))
    return out
