"""Immersed-boundary interpolation J and spreading S with a regularised delta kernel.

Follows Sec. III.B of the paper: (J v)_i = sum_alpha delta_h(x_alpha - r_i) v(x_alpha)
and (S lambda)_alpha = (1/dV) sum_i delta_h(x_alpha - r_i) lambda_i, with the
adjoint relation J = dV S^*.  delta_h(x) = phi(x/h) phi(y/h) phi(z/h) are
dimensionless weights.

Kernels (the grid's `kernel` width selects one):
  * 4: Peskin's standard 4-point function
        phi(r) = (3 - 2|r| + sqrt(1 + 4|r| - 4 r^2)) / 8      |r| <= 1
               = (5 - 2|r| - sqrt(-7 + 12|r| - 4 r^2)) / 8     1 <= |r| <= 2
               = 0                                              otherwise
  * 6: the 6-point function of the paper's runs (Sec. III.B; Bao, Kaiser & Peskin,
    J. Comput. Phys. 2016), supported on |r| < 3 and defined, for every shift x,
    by conditions on its six values at x - k: even and odd sums 1/2 each, first
    and third moments 0, second moment K = 59/60 - sqrt(29)/20 (the value that
    makes the function three times continuously differentiable), and sum of
    squares C, the value those conditions give at x = 0 (where phi(+-3) = 0).
    Five conditions are linear in the six values; the quadratic one fixes the
    last free value, on the branch that is continuous with phi(-3) = 0.  The
    values are computed here by solving exactly that system (no closed form).

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
otherwise), base = floor(s) - (W/2 - 1), the W support points base .. base + W - 1.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

from .mac import Grid, PERIODIC, SLIP, WALL, _face_col


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


K6 = 59.0 / 60.0 - np.sqrt(29.0) / 20.0


def _phi6_values(x, K=K6):
    """For shifts x in [0, 1) (real or complex, for complex-step derivatives), the six
    kernel values phi(x - k), k = -2 .. 3, as an array (len(x), 6).  K is the second
    moment (K6 for the kernel; other values only to show what the smoothness needs)."""
    x = np.asarray(x)
    n = x.shape[0]
    ks = np.arange(-2, 4)
    d = x[:, None] - ks[None, :]                       # distances x - k
    A = np.zeros((n, 5, 6), dtype=x.dtype)
    A[:, 0, [0, 2, 4]] = 1.0                           # even sum (k = -2, 0, 2)
    A[:, 1, [1, 3, 5]] = 1.0                           # odd sum (k = -1, 1, 3)
    A[:, 2] = d                                        # first moment
    A[:, 3] = d ** 2                                   # second moment
    A[:, 4] = d ** 3                                   # third moment
    b = np.zeros((n, 5), dtype=x.dtype)
    b[:, 0] = b[:, 1] = 0.5
    b[:, 3] = K
    # the last value t = phi(x - 3) is free: values = p + t q
    M = A[:, :, :5]
    p = np.linalg.solve(M, b[:, :, None])[:, :, 0]
    q = np.linalg.solve(M, -A[:, :, 5:6])[:, :, 0]
    p = np.concatenate([p, np.zeros((n, 1), dtype=x.dtype)], axis=1)
    q = np.concatenate([q, np.ones((n, 1), dtype=x.dtype)], axis=1)
    # sum of squares: C from x = 0, where phi(+-3) = 0 and the linear conditions
    # fix the other five values (phi(+-1) = 1/4, phi(+-2) = (K - 1/2)/8)
    f2 = (K - 0.5) / 8.0
    C = (0.5 - 2.0 * f2) ** 2 + 2.0 * 0.25 ** 2 + 2.0 * f2 ** 2
    qa = np.sum(q * q, axis=1)
    qb = 2.0 * np.sum(p * q, axis=1)
    qc = np.sum(p * p, axis=1) - C
    t = (-qb + np.sqrt(qb * qb - 4.0 * qa * qc)) / (2.0 * qa)   # the root with t = 0 at x = 0
    return p + t[:, None] * q


def phi6(r):
    """The 6-point kernel (vectorised)."""
    a = np.abs(np.asarray(r, dtype=np.float64)).ravel()
    out = np.zeros(a.shape)
    m = a < 3.0
    k = np.floor(a[m]).astype(np.int64)
    vals = _phi6_values(a[m] - k)
    out[m] = vals[np.arange(k.size), 2 - k]            # phi(x + k) is the value at -k
    return out.reshape(np.shape(r))


def dphi6(r):
    """d phi / d r of the 6-point kernel, by a complex-step derivative of the same
    construction (exact to rounding: the values are analytic in the shift)."""
    r = np.asarray(r, dtype=np.float64)
    a = np.abs(r).ravel()
    out = np.zeros(a.shape)
    m = a < 3.0
    k = np.floor(a[m]).astype(np.int64)
    h = 1e-30
    vals = _phi6_values((a[m] - k) + 1j * h)
    out[m] = vals[np.arange(k.size), 2 - k].imag / h
    return (out * np.sign(r.ravel())).reshape(r.shape)


def kernel_of(g: Grid):
    """(width, phi, dphi) of the grid's delta kernel."""
    return (6, phi6, dphi6) if getattr(g, "kernel", 4) == 6 else (4, phi4, dphi4)


def axis_offset(c: int, a: int) -> float:
    return 0.0 if a == c else 0.5


def base_index(g: Grid, r: np.ndarray, c: int) -> np.ndarray:
    """(nm, 3) int: floor(r * (1/h) - o) - (W/2 - 1) per axis for component c (W the
    kernel width: the support is the W points base .. base + W - 1)."""
    W = kernel_of(g)[0]
    inv_h = 1.0 / g.h
    out = np.empty(r.shape, dtype=np.int64)
    for a in range(3):
        s = r[:, a] * inv_h - axis_offset(c, a)
        out[:, a] = np.floor(s).astype(np.int64) - (W // 2 - 1)
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
    # the reflected value's sign: the normal component is odd about any wall, a
    # tangential one odd about a no-slip wall and even about a free-slip wall
    refl = 1.0 if (a != c and g.bc[a] == SLIP) else -1.0
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
    sign[lo | hi] = refl
    crossed[lo] = 1
    crossed[hi] = 2
    valid &= (idx >= 0) & (idx < N)
    return idx, sign, valid, crossed


def _support(g: Grid, r: np.ndarray, c: int):
    """Per marker, the W^3 support points of component c: (columns, signed weights, valid, crossed, raw phis)."""
    W, phi, _ = kernel_of(g)
    W3 = W ** 3
    nm = r.shape[0]
    b = base_index(g, r, c)
    inv_h = 1.0 / g.h
    per_axis = []
    for a in range(3):
        s = r[:, a] * inv_h - axis_offset(c, a)
        p = b[:, a][:, None] + np.arange(W)[None, :]
        w = phi(s[:, None] - p)
        idx, sign, valid, crossed = fold(g, c, a, p)
        per_axis.append((idx, sign, valid, crossed, w))
    ix, sx, vx, cx, wx = per_axis[0]
    iy, sy, vy, cy, wy = per_axis[1]
    iz, sz, vz, cz, wz = per_axis[2]
    # broadcast to (nm, W, W, W) in (z, y, x) order -> flatten to W^3
    sh = (nm, W, W, W)
    I = np.broadcast_to(ix[:, None, None, :], sh).reshape(nm, W3)
    J = np.broadcast_to(iy[:, None, :, None], sh).reshape(nm, W3)
    K = np.broadcast_to(iz[:, :, None, None], sh).reshape(nm, W3)
    sgn = (sz[:, :, None, None] * sy[:, None, :, None] * sx[:, None, None, :]).reshape(nm, W3)
    w = (wz[:, :, None, None] * wy[:, None, :, None] * wx[:, None, None, :]).reshape(nm, W3)
    valid = (vz[:, :, None, None] & vy[:, None, :, None] & vx[:, None, None, :]).reshape(nm, W3)
    cross = [np.broadcast_to(cx[:, None, None, :], sh).reshape(nm, W3),
             np.broadcast_to(cy[:, None, :, None], sh).reshape(nm, W3),
             np.broadcast_to(cz[:, :, None, None], sh).reshape(nm, W3)]
    signs = [np.broadcast_to(sx[:, None, None, :], sh).reshape(nm, W3),
             np.broadcast_to(sy[:, None, :, None], sh).reshape(nm, W3),
             np.broadcast_to(sz[:, :, None, None], sh).reshape(nm, W3)]
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
    W, phi, dphi = kernel_of(g)
    nm = r.shape[0]
    out = np.zeros((nm, 3))
    inv_h = 1.0 / g.h
    for c in range(3):
        b = base_index(g, r, c)
        ax = []
        for a in range(3):
            s = r[:, a] * inv_h - axis_offset(c, a)
            p = b[:, a][:, None] + np.arange(W)[None, :]
            idx, sign, valid, _ = fold(g, c, a, p)
            ax.append((idx, sign, valid, phi(s[:, None] - p), dphi(s[:, None] - p) * inv_h))
        (ix, sx, vx, wx, dx), (iy, sy, vy, wy, dy), (iz, sz, vz, wz, dz) = ax
        I = np.broadcast_to(ix[:, None, None, :], (nm, W, W, W))
        J = np.broadcast_to(iy[:, None, :, None], (nm, W, W, W))
        K = np.broadcast_to(iz[:, :, None, None], (nm, W, W, W))
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
