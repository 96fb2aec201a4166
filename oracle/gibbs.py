"""Gibbs-Boltzmann reference for one rigid body in a slit (App. A), in FP64.

Test infrastructure: only the tests, the smoke check and the benchmark's CPU
leg use this package.

At equilibrium the configuration Q = (q, theta) of a rigid body has density
proportional to exp(-U(Q)/kT) with respect to Lebesgue measure on q and the
Haar measure on the orientations.  In the slit of App. A the energy (soft
blob-wall repulsion on both walls plus the buoyant weight of every blob)
depends only on the height q_z of the tracking point and on the orientation,
so the x and y coordinates are uniform and drop out of every marginal.  The
paper obtains its reference curves with an MCMC method; two routes to the
same density are written here:

  ``gb_marginals``  deterministic-quadrature route: M seeded Haar orientations
      (unit quaternions from normalised 4-D Gaussians) and, for each, the
      height integral of exp(-U/kT) on a fine trapezoid grid.  The height
      marginal is the orientation average of exp(-U(z, R)/kT); the angle
      marginal weighs each orientation by its height integral.  Its only
      error is the Monte-Carlo error of the orientation average, which it
      estimates from independent batches.
  ``metropolis``    a random-walk Metropolis chain on (q_z, theta) with
      symmetric proposals (a Gaussian step in height, a left-multiplied
      rotation by a Gaussian rotation vector, whose density is symmetric
      under inversion), as the paper's MCMC reference.

A configuration with a marker outside the open slit has density zero (the
time integrator rejects such steps as well).

The observables of App. A: the height of the cross point (the blob at the
bend of the L) and the angle between the z axis and the unit vector p-hat
that lies in the plane of the boomerang and bisects the right angle at the
cross point.

Parity pins: a single blob reduces to a one-dimensional Boltzmann integral
(compared with scipy quadrature); with no energy the angle marginal of a
fixed body vector is sin(theta)/2; the Metropolis chain and the quadrature
agree within their statistical errors.
"""
from __future__ import annotations

import numpy as np

from .bodies import rotation_matrices, quat_mul
from .potentials import soft_profile


def haar_quaternions(rng: np.random.Generator, m: int) -> np.ndarray:
    """m unit quaternions uniform on S^3 (Haar-distributed rotations)."""
    x = rng.standard_normal((m, 4))
    return x / np.linalg.norm(x, axis=1, keepdims=True)


def slit_energy(zm: np.ndarray, Lz: float, phi0: float, d: float, b: float, weight: float) -> np.ndarray:
    """Energy (units of kT) of markers at heights zm, summed over the last axis.

    Soft repulsion from the faces z = 0 and z = Lz plus weight * z per marker
    (a downward force of size weight).  Infinite when a marker is outside (0, Lz).
    """
    v_lo, _ = soft_profile(zm, phi0, d, b)
    v_hi, _ = soft_profile(Lz - zm, phi0, d, b)
    e = np.sum(v_lo + v_hi + weight * zm, axis=-1)
    outside = np.any((zm <= 0.0) | (zm >= Lz), axis=-1)
    return np.where(outside, np.inf, e)


def _heights(theta: np.ndarray, r_ref: np.ndarray) -> np.ndarray:
    """z offsets (M, nm) of the markers from the tracking point for each orientation."""
    R = rotation_matrices(theta)
    return R[:, 2, :] @ r_ref.T


def angle_with_z(theta: np.ndarray, p_body: np.ndarray) -> np.ndarray:
    """Angle in [0, pi] between the z axis and R(theta) p_body for each orientation."""
    R = rotation_matrices(theta)
    pz = R[:, 2, :] @ (p_body / np.linalg.norm(p_body))
    return np.arccos(np.clip(pz, -1.0, 1.0))


def gb_marginals(r_ref: np.ndarray, p_body: np.ndarray, Lz: float, phi0: float, d: float, b: float,
                 weight: float, z_edges: np.ndarray, ang_edges: np.ndarray, m: int = 200000,
                 seed: int = 0, nz: int = 2000, batches: int = 10, chunk: int = 500):
    """Bin probabilities of the tracking-point height and of the p-hat angle.

    Returns (p_height, p_angle, se_height, se_angle): probabilities per bin of
    z_edges and ang_edges, and the standard errors of the orientation average
    estimated from ``batches`` independent batches.  The height bins are
    normalised over the edges given (a conditional marginal if they do not
    span the slit); the angle marginal always covers every height.
    """
    rng = np.random.default_rng(seed)
    z = np.linspace(0.0, Lz, nz + 1)
    dz = z[1] - z[0]
    tw = np.full(z.shape, dz)
    tw[0] = tw[-1] = 0.5 * dz                      # trapezoid weights in height
    nbz, nba = len(z_edges) - 1, len(ang_edges) - 1
    hz = np.zeros((batches, nbz))
    ha = np.zeros((batches, nba))
    per = m // batches
    for k in range(batches):
        dens = np.zeros(z.shape)
        for c0 in range(0, per, chunk):
            th = haar_quaternions(rng, min(chunk, per - c0))
            off = _heights(th, r_ref)                               # (chunk, nm)
            U = slit_energy(z[None, :, None] + off[:, None, :], Lz, phi0, d, b, weight)   # (chunk, nz+1)
            w = np.exp(-U)                                          # exp(-inf) = 0
            dens += w.sum(axis=0)
            wz = w @ tw                                             # height integral per orientation
            ab = np.searchsorted(ang_edges, angle_with_z(th, p_body), side="right") - 1
            np.add.at(ha[k], np.clip(ab, 0, nba - 1), wz)
        # bin mass: the cumulative trapezoid integral of the density, read at the edges
        cum = np.concatenate([[0.0], np.cumsum(0.5 * dz * (dens[1:] + dens[:-1]))])
        hz[k] = np.diff(np.interp(z_edges, z, cum))
    # normalise each batch (the same partition function for both marginals)
    Z = hz.sum(axis=1, keepdims=True)
    hz /= Z
    ha /= ha.sum(axis=1, keepdims=True)
    se = lambda h: h.std(axis=0, ddof=1) / np.sqrt(batches)
    return hz.mean(axis=0), ha.mean(axis=0), se(hz), se(ha)


def small_rotation(rng: np.random.Generator, sigma: float) -> np.ndarray:
    """Unit quaternion of a Gaussian rotation vector with per-component std sigma."""
    phi = sigma * rng.standard_normal(3)
    ang = np.linalg.norm(phi)
    if ang == 0.0:
        return np.array([1.0, 0.0, 0.0, 0.0])
    return np.concatenate([[np.cos(0.5 * ang)], np.sin(0.5 * ang) * phi / ang])


def metropolis(r_ref: np.ndarray, Lz: float, phi0: float, d: float, b: float, weight: float,
               z0: float, theta0: np.ndarray, n_steps: int, seed: int = 0, sz: float = 0.3,
               srot: float = 0.15, thin: int = 10):
    """Random-walk Metropolis chain of (height, orientation); returns thinned samples.

    Proposals: z' = z + sz N(0,1) and theta' = [small rotation] (x) theta, both
    symmetric, accepted with probability min(1, exp(-(U' - U))).
    Returns (z samples, theta samples (n, 4), acceptance rate).
    """
    rng = np.random.default_rng(seed)
    z = float(z0)
    th = np.asarray(theta0, dtype=np.float64).reshape(4)
    U = float(slit_energy((z + _heights(th[None], r_ref))[0], Lz, phi0, d, b, weight))
    if not np.isfinite(U):
        raise ValueError("the starting configuration has a marker outside the slit")
    zs, ths, acc = [], [], 0
    for k in range(n_steps):
        zp = z + sz * rng.standard_normal()
        tp = quat_mul(small_rotation(rng, srot), th)
        tp /= np.linalg.norm(tp)
        Up = float(slit_energy((zp + _heights(tp[None], r_ref))[0], Lz, phi0, d, b, weight))
        if np.isfinite(Up) and rng.random() < np.exp(min(0.0, -(Up - U))):
            z, th, U = zp, tp, Up
            acc += 1
        if (k + 1) % thin == 0:
            zs.append(z)
            ths.append(th.copy())
    return np.array(zs), np.array(ths), acc / max(n_steps, 1)


def gb_samples(r_ref: np.ndarray, Lz: float, phi0: float, d: float, b: float, weight: float,
               n: int, seed: int = 0):
    """n independent exact draws of (height, orientation) by rejection sampling.

    Proposals: uniform height in (0, Lz) and a Haar orientation, accepted with
    probability exp(-(U - U_min)), U_min the minimum over a first batch lowered
    by a margin (checked: no accepted proposal may have a lower energy).
    """
    rng = np.random.default_rng(seed)
    th = haar_quaternions(rng, 20000)
    zz = rng.uniform(0.0, Lz, 20000)
    U = slit_energy(zz[:, None] + _heights(th, r_ref), Lz, phi0, d, b, weight)
    umin = float(np.min(U)) - 2.0
    out_z, out_t = [], []
    while len(out_z) < n:
        th = haar_quaternions(rng, 20000)
        zz = rng.uniform(0.0, Lz, 20000)
        U = slit_energy(zz[:, None] + _heights(th, r_ref), Lz, phi0, d, b, weight)
        if np.min(U) < umin:
            raise RuntimeError("rejection bound violated; lower the energy floor")
        keep = rng.random(20000) < np.exp(-(U - umin))
        out_z.extend(zz[keep].tolist())
        out_t.extend(th[keep].tolist())
    return np.array(out_z[:n]), np.array(out_t[:n])
