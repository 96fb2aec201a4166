"""Staggered (MAC) grid operators of the discrete fluctuating Stokes equations.

Follows Sec. III.A of the paper (the paragraph defining the staggered grid,
D, G = -D^*, DT, GT = -DT^*, L = D G and Lm = DT GT, and eq. (DFHD)).

Conventions (the paper defers boundary details to its references; the
readings used here are stated):

* Cells (i, j, k), 0 <= i < Nx etc.; pressure at cell centres; velocity
  component c lives on c-faces: face index f along axis c is the face at
  coordinate f*h, and the other two coordinates are cell centred.
* Along a WALL (no-slip) or SLIP (free-slip) axis a, the c = a faces 0 and N_a
  lie on the walls and are not unknowns (normal velocity vanishes).  Along a
  PERIODIC axis everything wraps.
* Compact unknowns: for each component the true unknown faces in x-fastest
  order; the velocity vector is [u_x | u_y | u_z].
* Padded layout (used at the library boundary): each component stored as an
  Nx*Ny*Nz array indexed by (face index along c, cell indices otherwise); the
  wall face 0 along a wall c-axis occupies a slot that is always zero.
* Vector Laplacian, ghost-cell form: tangential ghost u_g = 2 U_w - u_interior
  (U_w the wall velocity) at a no-slip wall, u_g = u_interior at a free-slip
  wall (no tangential stress), normal wall faces Dirichlet 0.  This equals
  DT GT when the one-sided gradient on a wall edge carries weight sqrt(2)/h at
  a no-slip wall and 0 at a free-slip wall (where the tangential gradient
  vanishes), which is the discrete fluctuation-dissipation balance the paper
  requires.  Free-slip walls are one of the combinations of boundary
  conditions the paper's formulation admits (Introduction, Conclusion); they
  do not move.
* Noise index space W: nine families (c, b) in the order
  xx, yy, zz, xy, xz, yx, yz, zx, zy.  Family (c, c) lives on cells; family
  (c, b != c) lives on edges: node index along b (N_b + 1 nodes on a wall
  axis, N_b when periodic), padded face index along c, cell index along the
  third axis.  Each family is stored x-fastest.
"""
from __future__ import annotations

import math
from typing import List, Tuple

import numpy as np
import scipy.sparse as sp

PERIODIC = 0
WALL = 1          # no-slip wall (possibly sliding)
SLIP = 2          # free-slip wall

FAMILIES: List[Tuple[int, int]] = [(0, 0), (1, 1), (2, 2), (0, 1), (0, 2), (1, 0), (1, 2), (2, 0), (2, 1)]


class Grid:
    """A box of Nx x Ny x Nz cells of width h, with a BC per axis and wall velocities."""

    def __init__(self, n, bc, h: float = 1.0, eta: float = 1.0, wall_vel=None, kernel: int = 4):
        self.n = tuple(int(v) for v in n)
        if any(int(b) not in (PERIODIC, WALL, SLIP) for b in bc):
            raise ValueError("boundary conditions are PERIODIC, WALL or SLIP")
        # width of the immersed-boundary delta kernel used with this grid (ib.py): 4
        # (Peskin's 4-point function) or 6 (the 6-point function of the paper's runs)
        if kernel not in (4, 6):
            raise ValueError("kernel width must be 4 or 6")
        self.kernel = int(kernel)
        self.bc = tuple(int(v) for v in bc)
        self.h = float(h)
        self.eta = float(eta)
        self.wall_vel = np.zeros((3, 2, 3)) if wall_vel is None else np.asarray(wall_vel, dtype=np.float64)
        self.dV = self.h ** 3
        self.ncell = self.n[0] * self.n[1] * self.n[2]
        # compact index of each padded face slot, -1 for pinned wall faces
        self.face_index = []
        self.nface = []
        off = 0
        self.face_offset = []
        for c in range(3):
            idx = -np.ones(self.n[::-1], dtype=np.int64)      # indexed [k, j, i]
            mask = np.ones(self.n[::-1], dtype=bool)
            if self.bc[c] != PERIODIC:
                sl = [slice(None)] * 3
                sl[2 - c] = 0
                mask[tuple(sl)] = False
            cnt = int(mask.sum())
            idx[mask] = np.arange(cnt)
            self.face_index.append(idx)
            self.nface.append(cnt)
            self.face_offset.append(off)
            off += cnt
        self.nv = off

    # ------------------------------------------------------------------ layout
    def padded_to_compact(self, padded: np.ndarray) -> np.ndarray:
        """[3, Nz, Ny, Nx] (or flat 3*N) padded velocity -> compact vector."""
        p = np.asarray(padded).reshape(3, *self.n[::-1])
        out = np.empty(self.nv)
        for c in range(3):
            m = self.face_index[c] >= 0
            out[self.face_offset[c]:self.face_offset[c] + self.nface[c]] = p[c][m]
        return out

    def compact_to_padded(self, v: np.ndarray) -> np.ndarray:
        out = np.zeros((3, *self.n[::-1]))
        for c in range(3):
            m = self.face_index[c] >= 0
            out[c][m] = v[self.face_offset[c]:self.face_offset[c] + self.nface[c]]
        return out.reshape(3, -1)

    def nodes(self, a: int) -> int:
        return self.n[a] + 1 if self.bc[a] != PERIODIC else self.n[a]

    def family_dims(self, fam: int) -> Tuple[int, int, int]:
        c, b = FAMILIES[fam]
        return tuple(self.nodes(a) if (a == b and b != c) else self.n[a] for a in range(3))

    def family_offsets(self) -> np.ndarray:
        sizes = [int(np.prod(self.family_dims(f))) for f in range(9)]
        return np.concatenate([[0], np.cumsum(sizes)])

    @property
    def nW(self) -> int:
        return int(self.family_offsets()[-1])


def _cell_lin(g: Grid, i, j, k):
    return i + g.n[0] * (j + g.n[1] * k)


def _face_col(g: Grid, c: int, pos):
    """Global compact column of velocity component c at padded position pos=(i,j,k) arrays.

    Returns -1 where the slot is not an unknown.  pos entries must be in range.
    """
    i, j, k = pos
    idx = g.face_index[c][k, j, i]
    return np.where(idx >= 0, idx + g.face_offset[c], -1)


def _grid_coords(dims):
    k, j, i = np.meshgrid(np.arange(dims[2]), np.arange(dims[1]), np.arange(dims[0]), indexing="ij")
    return [i.ravel(), j.ravel(), k.ravel()]


def divergence(g: Grid) -> sp.csr_matrix:
    """D: velocity (compact) -> cells.  (Dv)_cell = sum_c (u_c(f+1) - u_c(f)) / h."""
    rows, cols, vals = [], [], []
    pos = _grid_coords(g.n)
    cell = _cell_lin(g, *pos)
    for c in range(3):
        for shift, sgn in ((1, 1.0), (0, -1.0)):
            p = list(pos)
            f = p[c] + shift
            if g.bc[c] == PERIODIC:
                f = f % g.n[c]
                ok = np.ones_like(f, dtype=bool)
            else:
                ok = (f >= 1) & (f <= g.n[c] - 1)
                f = np.clip(f, 0, g.n[c] - 1)
            p[c] = f
            col = _face_col(g, c, p)
            ok &= col >= 0
            rows.append(cell[ok]); cols.append(col[ok]); vals.append(np.full(ok.sum(), sgn / g.h))
    return sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                         shape=(g.ncell, g.nv))


def gradient(g: Grid) -> sp.csr_matrix:
    """G = -D^T (the paper's adjoint relation)."""
    return (-divergence(g).T).tocsr()


def vector_gradient(g: Grid) -> sp.csr_matrix:
    """GT: velocity (compact) -> noise index space W (rows of pinned slots are empty).

    Family (c, c): cell (i,j,k) -> (u_c(f = i_c + 1) - u_c(i_c)) / h.
    Family (c, b): node n along b -> w * (u_c(cell n) - u_c(cell n - 1)) / h, where a
    cell outside a wall axis holds zero velocity and w = sqrt(2) on the two wall nodes
    of a no-slip axis, 0 on those of a free-slip axis.
    """
    offs = g.family_offsets()
    rows, cols, vals = [], [], []
    for fam, (c, b) in enumerate(FAMILIES):
        dims = g.family_dims(fam)
        pos = _grid_coords(dims)
        lin = pos[0] + dims[0] * (pos[1] + dims[1] * pos[2]) + offs[fam]
        if b == c:
            for shift, sgn in ((1, 1.0), (0, -1.0)):
                p = list(pos)
                f = p[c] + shift
                if g.bc[c] == PERIODIC:
                    f = f % g.n[c]; ok = np.ones_like(f, dtype=bool)
                else:
                    ok = (f >= 1) & (f <= g.n[c] - 1); f = np.clip(f, 0, g.n[c] - 1)
                p[c] = f
                col = _face_col(g, c, p)
                ok &= col >= 0
                rows.append(lin[ok]); cols.append(col[ok]); vals.append(np.full(ok.sum(), sgn / g.h))
        else:
            node = pos[b]
            if g.bc[b] != PERIODIC:
                w = np.where((node == 0) | (node == g.n[b]), math.sqrt(2.0) if g.bc[b] == WALL else 0.0, 1.0)
            else:
                w = np.ones(node.shape)
            for shift, sgn in ((0, 1.0), (-1, -1.0)):
                p = list(pos)
                cb = node + shift
                if g.bc[b] == PERIODIC:
                    cb = cb % g.n[b]; ok = np.ones_like(cb, dtype=bool)
                else:
                    ok = (cb >= 0) & (cb <= g.n[b] - 1); cb = np.clip(cb, 0, g.n[b] - 1)
                p[b] = cb
                col = _face_col(g, c, p)
                ok &= col >= 0
                rows.append(lin[ok]); cols.append(col[ok]); vals.append((sgn * w / g.h)[ok])
    return sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                         shape=(g.nW, g.nv))


def tensor_divergence(g: Grid) -> sp.csr_matrix:
    """DT = -GT^T."""
    return (-vector_gradient(g).T).tocsr()


def vector_laplacian(g: Grid) -> sp.csr_matrix:
    """Lm by the ghost-cell stencil (homogeneous part).

    Per axis a, face neighbours along a = c (Dirichlet 0 at wall faces) and
    cell neighbours along a != c (ghost -u across a no-slip wall, i.e. diagonal
    -3/h^2 next to it; ghost +u across a free-slip wall, diagonal -1/h^2);
    periodic axes wrap.
    """
    rows, cols, vals = [], [], []
    for c in range(3):
        pos = _grid_coords(g.n)
        me = _face_col(g, c, pos)
        keep = me >= 0
        pos = [p[keep] for p in pos]
        me = me[keep]
        diag = np.zeros(me.shape)
        for a in range(3):
            for d in (1, -1):
                p = list(pos)
                nb = p[a] + d
                if g.bc[a] == PERIODIC:
                    nb = nb % g.n[a]
                    p[a] = nb
                    col = _face_col(g, c, p)
                    rows.append(me); cols.append(col); vals.append(np.full(me.shape, 1.0 / g.h**2))
                    diag -= 1.0 / g.h**2
                elif a == c:
                    ok = (nb >= 1) & (nb <= g.n[a] - 1)
                    p[a] = np.clip(nb, 0, g.n[a] - 1)
                    col = _face_col(g, c, p)
                    rows.append(me[ok]); cols.append(col[ok]); vals.append(np.full(ok.sum(), 1.0 / g.h**2))
                    diag -= 1.0 / g.h**2
                else:
                    ok = (nb >= 0) & (nb <= g.n[a] - 1)
                    p[a] = np.clip(nb, 0, g.n[a] - 1)
                    col = _face_col(g, c, p)
                    rows.append(me[ok]); cols.append(col[ok]); vals.append(np.full(ok.sum(), 1.0 / g.h**2))
                    # beyond the wall the ghost is -u (no-slip) or +u (free-slip)
                    diag -= np.where(ok, 1.0, 2.0 if g.bc[a] == WALL else 0.0) / g.h**2
        rows.append(me); cols.append(me); vals.append(diag)
    return sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                         shape=(g.nv, g.nv))


def scalar_laplacian(g: Grid) -> sp.csr_matrix:
    """L = D G (Neumann at walls by construction)."""
    return (divergence(g) @ gradient(g)).tocsr()


def moving_wall_rhs(g: Grid) -> np.ndarray:
    """Affine part of -eta*Lm moved to the right-hand side: +2 eta U_w / h^2 on
    tangential faces next to a moving wall (ghost u_g = 2 U_w - u)."""
    out = np.zeros(g.nv)
    for c in range(3):
        pos = _grid_coords(g.n)
        me = _face_col(g, c, pos)
        for a in range(3):
            if a == c or g.bc[a] != WALL:
                continue
            for side, at in ((0, 0), (1, g.n[a] - 1)):
                U = g.wall_vel[a, side, c]
                if U == 0.0:
                    continue
                sel = (pos[a] == at) & (me >= 0)
                np.add.at(out, me[sel], 2.0 * g.eta * U / g.h**2)
    return out


def noise_stress_divergence(g: Grid, W: np.ndarray, kT: float, dt: float) -> np.ndarray:
    """sqrt(2 kT eta / (dV dt)) * DT W, the fluctuating-stress forcing of eq. (DFHD)."""
    scale = math.sqrt(2.0 * kT * g.eta / (g.dV * dt))
    return scale * (tensor_divergence(g) @ W)
