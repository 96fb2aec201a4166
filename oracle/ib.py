"""Immersed-boundary interpolation J and spreading S with the Peskin 4-point kernel.

Follows Sec. III.B of the paper: (J v)_i = sum_alpha delta_h(x_alpha - r_i) v(x_alpha)
and (S lambda)_alpha = (1/dV) sum_i delta_h(x_alpha - r_i) lambda_i, with the
adjoint relation J = dV S^*.  delta_h(x) = phi(x/h) phi(y/h) phi(z/h) are
dimensionless weights.

Kernel (the configurations here use Peskin's standard 4-point function; the
paper's own runs use a 6-point kernel):
    phi(r) = (3 - 2|r| + sqrt(1 + 4|r| - 4 r^2)) / 8      |r| <= 1
           = (5 - 2|r| - sqrt(-7 + 12|r| - 4 r^2)) / 8     1 <= |r| <= 2
           = 0                                              otherwise

Walls (the paper defers to ghost points across the boundary that keep J and
S adjoint; reading used here -- odd reflection):
  * velocity component c, axis a == c (normal): support face p = 0 or N is a
    wall face and contributes nothing; ghost face -m folds to +m and N + m to
    N - m, each with sign -1;
  * axis a != c (tangential): ghost cell -1 - m folds to m and N + m to
    N - 1 - m, each with sign -1;
  * periodic axes wrap; signs multiply across axes.
  * A wall moving with tangential velocity U adds the affine term
    J_bc = sum over ghost points across that wall of w * 2U * (product of the
    signs of the other reflections of that point).

Marker indexing: s = r * (1/h) - o (o = 0 along the face-normal axis, 1/2
otherwise), base = floor(s) - 1, the four support points base .. base + 3.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

from .mac import Grid, PERIODIC, WALL, _face_col


def phi4(r):
    """Peskin 4-point kernel (vectorised)."""
    a = np.abs(np.asarray(r, dtype=np.float64))
    out = np.zeros(a.shape)
    m1 = a <= 1.0
    m2 = (a > 1.0) & (a < 2.0)
    a1 = a[m1]
    out[m1] = (3.0 - 2.0 * a1 + np.sqrt(1.0 + 4.0 * a1 - 4.0 * a1 * a1)) / 8.0
    a2 = a[m2]
    out[m2] = (5.0 - 2.0 * a2 - np.sqrt(-7.0 + 12.0 * a2 - 4.0 * a2 * a2)) / 8.0
    return out


def dphi4(r):
    """d phi / d r of the 4-point kernel (odd function, C^0, zero at 0 and |r| = 2)."""
    r = np.asarray(r, dtype=np.float64)
    a = np.abs(r)
    s = np.sign(r)
    out = np.zeros(a.shape)
    m1 = a <= 1.0
    m2 = (a > 1.0) & (a < 2.0)
    a1 = a[m1]
    out[m1] = (-2.0 + (4.0 - 8.0 * a1) / (2.0 * np.sqrt(1.0 + 4.0 * a1 - 4.0 * a1 * a1))) / 8.0
    a2 = a[m2]
    out[m2] = (-2.0 - (12.0 - 8.0 * a2) / (2.0 * np.sqrt(-7.0 + 12.0 * a2 - 4.0 * a2 * a2))) / 8.0
    return out * s


def axis_offset(c: int, a: int) -> float:
    return 0.0 if a == c else 0.5


def base_index(g: Grid, r: np.ndarray, c: int) -> np.ndarray:
    """(nm, 3) int: floor(r * (1/h) - o) - 1 per axis for component c."""
    inv_h = 1.0 / g.h
    out = np.empty(r.shape, dtype=np.int64)
    for a in range(3):
        s = r[:, a] * inv_h - axis_offset(c, a)
        out[:, a] = np.floor(s).astype(np.int64) - 1
    return out


def fold(g: Grid, c: int, a: int, p: np.ndarray):
    """Fold raw support indices p along axis a for component c.

    Returns (index, sign, valid, crossed) where crossed is 0 (inside), 1 (lower
    wall) or 2 (upper wall).
    """
    N = g.n[a]
    if g.bc[a] == PERIODIC:
        return p % N, np.ones(p.shape), np.ones(p.shape, dtype=bool), np.zeros(p.shape, dtype=np.int64)
    idx = p.copy()
    sign = np.ones(p.shape)
    crossed = np.zeros(p.shape, dtype=np.int64)
    if a == c:
        valid = (p != 0) & (p != N)
        lo = p < 0
        hi = p > N
        idx[lo] = -p[lo]
        idx[hi] = 2 * N - p[hi]
    else:
        valid = np.ones(p.shape, dtype=bool)
        lo = p < 0
        hi = p >= N
        idx[lo] = -1 - p[lo]
        idx[hi] = 2 * N - 1 - p[hi]
    sign[lo | hi] = -1.0
    crossed[lo] = 1
    crossed[hi] = 2
    valid &= (idx >= 0) & (idx < N)
    return idx, sign, valid, crossed


def _support(g: Grid, r: np.ndarray, c: int):
    """Per marker, the 64 support points of component c: (columns, signed weights, valid, crossed, raw phis)."""
    nm = r.shape[0]
    b = base_index(g, r, c)
    inv_h = 1.0 / g.h
    per_axis = []
    for a in range(3):
        s = r[:, a] * inv_h - axis_offset(c, a)
        p = b[:, a][:, None] + np.arange(4)[None, :]
        w = phi4(s[:, None] - p)
        idx, sign, valid, crossed = fold(g, c, a, p)
        per_axis.append((idx, sign, valid, crossed, w))
    ix, sx, vx, cx, wx = per_axis[0]
    iy, sy, vy, cy, wy = per_axis[1]
    iz, sz, vz, cz, wz = per_axis[2]
    # broadcast to (nm, 4, 4, 4) in (z, y, x) order -> flatten to 64
    I = np.broadcast_to(ix[:, None, None, :], (nm, 4, 4, 4)).reshape(nm, 64)
    J = np.broadcast_to(iy[:, None, :, None], (nm, 4, 4, 4)).reshape(nm, 64)
    K = np.broadcast_to(iz[:, :, None, None], (nm, 4, 4, 4)).reshape(nm, 64)
    sgn = (sz[:, :, None, None] * sy[:, None, :, None] * sx[:, None, None, :]).reshape(nm, 64)
    w = (wz[:, :, None, None] * wy[:, None, :, None] * wx[:, None, None, :]).reshape(nm, 64)
    valid = (vz[:, :, None, None] & vy[:, None, :, None] & vx[:, None, None, :]).reshape(nm, 64)
    cross = [np.broadcast_to(cx[:, None, None, :], (nm, 4, 4, 4)).reshape(nm, 64),
             np.broadcast_to(cy[:, None, :, None], (nm, 4, 4, 4)).reshape(nm, 64),
             np.broadcast_to(cz[:, :, None, None], (nm, 4, 4, 4)).reshape(nm, 64)]
    signs = [np.broadcast_to(sx[:, None, None, :], (nm, 4, 4, 4)).reshape(nm, 64),
             np.broadcast_to(sy[:, None, :, None], (nm, 4, 4, 4)).reshape(nm, 64),
             np.broadcast_to(sz[:, :, None, None], (nm, 4, 4, 4)).reshape(nm, 64)]
    Ic = np.where(valid, I, 0)
    Jc = np.where(valid, J, 0)
    Kc = np.where(valid, K, 0)
    col = _face_col(g, c, (Ic, Jc, Kc))
    valid = valid & (col >= 0)
    return col, sgn * w, valid, cross, signs, w


def interpolation(g: Grid, r: np.ndarray) -> sp.csr_matrix:
    """J: velocity (compact) -> markers [nm, 3] (row 3*i + c)."""
    nm = r.shape[0]
    rows, cols, vals = [], [], []
    for c in range(3):
        col, sw, valid, _, _, _ = _support(g, r, c)
        row = np.broadcast_to((3 * np.arange(nm) + c)[:, None], col.shape)
        rows.append(row[valid]); cols.append(col[valid]); vals.append(sw[valid])
    return sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                         shape=(3 * nm, g.nv))


def spreading(g: Grid, r: np.ndarray) -> sp.csr_matrix:
    """S = J^T / dV (the paper's adjoint relation J = dV S^*)."""
    return (interpolation(g, r).T / g.dV).tocsr()


def interpolation_bc(g: Grid, r: np.ndarray) -> np.ndarray:
    """Affine part J_bc of interpolating a field whose ghosts carry moving-wall velocities."""
    nm = r.shape[0]
    out = np.zeros((nm, 3))
    if not np.any(g.wall_vel != 0.0):
        return out
    for c in range(3):
        col, sw, valid, cross, signs, w = _support(g, r, c)
        # rebuild validity without the unknown-column test so that ghost points of
        # tangential components (all valid) are counted exactly as the kernel sees them
        aff = np.zeros(col.shape)
        for a in range(3):
            if a == c or g.bc[a] != WALL:
                continue
            other = np.ones(col.shape)
            for b in range(3):
                if b != a:
                    other = other * signs[b]
            for side in (0, 1):
                U = g.wall_vel[a, side, c]
                if U == 0.0:
                    continue
                aff += np.where(cross[a] == side + 1, 2.0 * U * other, 0.0)
        out[:, c] = np.sum(np.where(valid, w * aff, 0.0), axis=1)
    return out


def interpolation_gradient(g: Grid, r: np.ndarray, v: np.ndarray, mu: np.ndarray) -> np.ndarray:
    """For each marker i, the gradient wrt r_i of mu_i . (J(r) v)_i with v fixed.

    Returns (nm, 3).  Uses d/dr of the product kernel: the derivative along axis
    a replaces phi_a by phi_a' / h.  Folding signs and indices are constant
    within each smooth piece.
    """
    nm = r.shape[0]
    out = np.zeros((nm, 3))
    inv_h = 1.0 / g.h
    for c in range(3):
        b = base_index(g, r, c)
        ax = []
        for a in range(3):
            s = r[:, a] * inv_h - axis_offset(c, a)
            p = b[:, a][:, None] + np.arange(4)[None, :]
            idx, sign, valid, _ = fold(g, c, a, p)
            ax.append((idx, sign, valid, phi4(s[:, None] - p), dphi4(s[:, None] - p) * inv_h))
        (ix, sx, vx, wx, dx), (iy, sy, vy, wy, dy), (iz, sz, vz, wz, dz) = ax
        I = np.broadcast_to(ix[:, None, None, :], (nm, 4, 4, 4))
        J = np.broadcast_to(iy[:, None, :, None], (nm, 4, 4, 4))
        K = np.broadcast_to(iz[:, :, None, None], (nm, 4, 4, 4))
        valid = vz[:, :, None, None] & vy[:, None, :, None] & vx[:, None, None, :]
        col = _face_col(g, c, (np.where(valid, I, 0), np.where(valid, J, 0), np.where(valid, K, 0)))
        valid = valid & (col >= 0)
        vals = np.where(valid, v[np.where(valid, col, 0)], 0.0)
        sgn = sz[:, :, None, None] * sy[:, None, :, None] * sx[:, None, None, :]
        gx = np.sum(sgn * wz[:, :, None, None] * wy[:, None, :, None] * dx[:, None, None, :] * vals, axis=(1, 2, 3))
        gy = np.sum(sgn * wz[:, :, None, None] * dy[:, None, :, None] * wx[:, None, None, :] * vals, axis=(1, 2, 3))
        gz = np.sum(sgn * dz[:, :, None, None] * wy[:, None, :, None] * wx[:, None, None, :] * vals, axis=(1, 2, 3))
        out += mu[:, c][:, None] * np.stack([gx, gy, gz], axis=1)
    return out
