"""Rigid bodies: orientations, marker positions, the geometric matrix K and tiles.

Follows Sec. II (configuration Q_p = [q_p, theta_p], unit quaternions for the
orientation) and Sec. III.B (the definitions of K U and K^T lambda) of the
paper.

Reading of K (the printed cross product order in K U is not the transpose of
the printed torque in K^T lambda; the physical rigid motion is used):
    (K U)_i = u_p + omega_p x d_i,   (K^T lambda)_p = [sum_i lambda_i ; sum_i d_i x lambda_i]
with d_i = R(theta_p) r_i^ref the marker offset from the tracking point, so
that <K U, lambda> = <U, K^T lambda> exactly.

Quaternions are scalar first, theta = (w, x, y, z).  Rotate(theta, phi)
left-multiplies by the unit quaternion of the lab-frame rotation vector phi,
[cos(|phi|/2), sin(|phi|/2) phi/|phi|] (x) theta, and renormalises; phi = 0
returns theta unchanged.

Marker positions r_i = q_p + R(theta_p) r_i^ref are formed with a fixed
operation order (R entries from products of quaternion components, then
(R_a0 x + R_a1 y) + R_a2 z, then q_a + d_a) so that integer indexing derived
from them can be compared bit for bit.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

from .mac import Grid, PERIODIC, WALL


def rotation_matrices(theta: np.ndarray) -> np.ndarray:
    """(nb, 3, 3) rotation matrices of unit quaternions (w, x, y, z)."""
    w, x, y, z = theta[:, 0], theta[:, 1], theta[:, 2], theta[:, 3]
    xx, yy, zz = x * x, y * y, z * z
    xy, xz, yz = x * y, x * z, y * z
    wx, wy, wz = w * x, w * y, w * z
    R = np.empty((theta.shape[0], 3, 3))
    R[:, 0, 0] = 1.0 - 2.0 * (yy + zz)
    R[:, 0, 1] = 2.0 * (xy - wz)
    R[:, 0, 2] = 2.0 * (xz + wy)
    R[:, 1, 0] = 2.0 * (xy + wz)
    R[:, 1, 1] = 1.0 - 2.0 * (xx + zz)
    R[:, 1, 2] = 2.0 * (yz - wx)
    R[:, 2, 0] = 2.0 * (xz - wy)
    R[:, 2, 1] = 2.0 * (yz + wx)
    R[:, 2, 2] = 1.0 - 2.0 * (xx + yy)
    return R


def quat_mul(a: np.ndarray, b: np.ndarray) -> np.ndarray:
    """Hamilton product a (x) b for arrays of quaternions (scalar first)."""
    aw, av = a[..., 0], a[..., 1:]
    bw, bv = b[..., 0], b[..., 1:]
    w = aw * bw - np.sum(av * bv, axis=-1)
    v = aw[..., None] * bv + bw[..., None] * av + np.cross(av, bv)
    return np.concatenate([w[..., None], v], axis=-1)


def rotate(theta: np.ndarray, phi: np.ndarray) -> np.ndarray:
    """Rotate(theta, phi): lab-frame rotation by the rotation vector phi, renormalised."""
    ang = np.linalg.norm(phi, axis=1)
    half = 0.5 * ang
    axis = np.where(ang[:, None] > 0.0, phi / np.where(ang > 0.0, ang, 1.0)[:, None], 0.0)
    dq = np.concatenate([np.cos(half)[:, None], np.sin(half)[:, None] * axis], axis=1)
    out = quat_mul(dq, theta)
    out /= np.linalg.norm(out, axis=1, keepdims=True)
    return np.where(ang[:, None] > 0.0, out, theta)


def body_of_marker(offsets: np.ndarray) -> np.ndarray:
    nb = len(offsets) - 1
    return np.repeat(np.arange(nb), np.diff(offsets))


def marker_offsets(theta: np.ndarray, r_ref: np.ndarray, offsets: np.ndarray) -> np.ndarray:
    """d_i = R(theta_p) r_i^ref (nm, 3)."""
    R = rotation_matrices(theta)[body_of_marker(offsets)]
    x, y, z = r_ref[:, 0], r_ref[:, 1], r_ref[:, 2]
    d = np.empty(r_ref.shape)
    for a in range(3):
        d[:, a] = (R[:, a, 0] * x + R[:, a, 1] * y) + R[:, a, 2] * z
    return d


def marker_positions(q: np.ndarray, theta: np.ndarray, r_ref: np.ndarray, offsets: np.ndarray) -> np.ndarray:
    """r_i = q_p + R(theta_p) r_i^ref."""
    return q[body_of_marker(offsets)] + marker_offsets(theta, r_ref, offsets)


def _cross_matrix(d: np.ndarray) -> np.ndarray:
    """[d]_x such that [d]_x w = d x w, for each row of d."""
    z = np.zeros(d.shape[0])
    return np.stack([np.stack([z, -d[:, 2], d[:, 1]], axis=1),
                     np.stack([d[:, 2], z, -d[:, 0]], axis=1),
                     np.stack([-d[:, 1], d[:, 0], z], axis=1)], axis=1)


def geometric_matrix(theta: np.ndarray, r_ref: np.ndarray, offsets: np.ndarray) -> sp.csr_matrix:
    """K: [nb, 6] -> [nm, 3].  Block for marker i of body p: [I, -[d_i]_x]."""
    d = marker_offsets(theta, r_ref, offsets)
    body = body_of_marker(offsets)
    nm = d.shape[0]
    nb = len(offsets) - 1
    C = _cross_matrix(d)
    rows, cols, vals = [], [], []
    for a in range(3):
        rows.append(3 * np.arange(nm) + a); cols.append(6 * body + a); vals.append(np.ones(nm))
        for b in range(3):
            rows.append(3 * np.arange(nm) + a); cols.append(6 * body + 3 + b); vals.append(-C[:, a, b])
    return sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                         shape=(3 * nm, 6 * nb))


def apply_K(theta, r_ref, offsets, U: np.ndarray) -> np.ndarray:
    """(K U)_i = u_p + omega_p x d_i, (nm, 3)."""
    d = marker_offsets(theta, r_ref, offsets)
    body = body_of_marker(offsets)
    U = U.reshape(-1, 6)
    return U[body, :3] + np.cross(U[body, 3:], d)


def apply_KT(theta, r_ref, offsets, lam: np.ndarray) -> np.ndarray:
    """(K^T lambda)_p = [sum lambda_i, sum d_i x lambda_i], (nb, 6)."""
    d = marker_offsets(theta, r_ref, offsets)
    body = body_of_marker(offsets)
    nb = len(offsets) - 1
    lam = lam.reshape(-1, 3)
    out = np.zeros((nb, 6))
    np.add.at(out[:, :3], body, lam)
    np.add.at(out[:, 3:], body, np.cross(d, lam))
    return out


def body_length(r_ref: np.ndarray, offsets: np.ndarray) -> np.ndarray:
    """L_p: maximum pairwise distance between the markers of body p (Sec. IV.B)."""
    nb = len(offsets) - 1
    out = np.zeros(nb)
    for p in range(nb):
        x = r_ref[offsets[p]:offsets[p + 1]]
        if x.shape[0] > 1:
            out[p] = np.max(np.linalg.norm(x[:, None, :] - x[None, :, :], axis=2))
    return out


# ---------------------------------------------------------------- tiles
TILE = 4


def tile_dims(g: Grid):
    return tuple((g.n[a] + TILE - 1) // TILE for a in range(3))


def marker_cells(g: Grid, r: np.ndarray) -> np.ndarray:
    """Containing cell per axis: floor(r * (1/h)), wrapped on periodic axes."""
    inv_h = 1.0 / g.h
    cell = np.floor(r * inv_h).astype(np.int64)
    for a in range(3):
        if g.bc[a] == PERIODIC:
            cell[:, a] %= g.n[a]
    return cell


def marker_tiles(g: Grid, r: np.ndarray):
    """Tile linear index (x fastest) of the 4^3-cell tile holding each marker,
    and the stable permutation sorting markers by (tile, marker id)."""
    cell = marker_cells(g, r)
    tc = cell // TILE
    td = tile_dims(g)
    tile = tc[:, 0] + td[0] * (tc[:, 1] + td[1] * tc[:, 2])
    perm = np.argsort(tile, kind="stable")
    return tile, perm


def inside_open_domain(g: Grid, r: np.ndarray) -> bool:
    """True when every marker lies strictly inside the box along every wall axis."""
    L = np.array(g.n) * g.h
    for a in range(3):
        if g.bc[a] != PERIODIC and (np.any(r[:, a] <= 0.0) or np.any(r[:, a] >= L[a])):
            return False
    return bool(np.all(np.isfinite(r)))
