"""The constrained Stokes saddle-point system and its exact solution.

Follows Sec. III.C of the paper (eqs. LangevinD1-D4) and the block matrix of
Algorithm 1.  Sign reading: the printed block matrix of Algorithm 1 carries
-K and -K^T with -F on the right, which would give U = -N F; eqs. D1-D4 are
followed instead, so the operator is

        [ -eta Lm   G   -S   0 ] [ v      ]   [ g + noise + moving-wall terms ]
        [   -D      0    0   0 ] [ pi     ] = [ 0                             ]
        [   -J      0    0   K ] [ lambda ]   [ -slip + J_bc                  ]
        [    0      0   K^T  0 ] [ U      ]   [ F                             ]

(row 3 is J v = K U + slip with J v = J_0 v + J_bc; row 4 is K^T lambda = F).
Unknown order: compact velocity, cell pressure, lambda [nm, 3], U [nb, 6].

Solvers (all reach the exact discrete solution; the residual against the
assembled matrix is the acceptance test):
  * ``solve_direct``: sparse LU of the matrix bordered by the mean-pressure
    constraint (the pressure is defined up to a constant);
  * ``solve_fgmres``: right-preconditioned FGMRES with an oracle-only
    preconditioner (exact per-component fast sine/cosine/Fourier Poisson
    solves in a projection step, plus a per-body dense blob-mobility block).
"""
from __future__ import annotations

import math
from typing import Optional

import numpy as np
import scipy.fft as sfft
import scipy.linalg as sla
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from . import bodies as B
from . import ib
from . import mac
from .mac import Grid, PERIODIC, SLIP, WALL


class Saddle:
    """Assembled operators of one configuration."""

    def __init__(self, g: Grid, q, theta, r_ref, offsets, fluid_only: bool = False):
        self.g = g
        self.q = np.asarray(q, dtype=np.float64).reshape(-1, 3)
        self.theta = np.asarray(theta, dtype=np.float64).reshape(-1, 4)
        self.r_ref = np.asarray(r_ref, dtype=np.float64).reshape(-1, 3)
        self.offsets = np.asarray(offsets, dtype=np.int64)
        self.fluid_only = fluid_only
        self.r = B.marker_positions(self.q, self.theta, self.r_ref, self.offsets)
        self.Lm = mac.vector_laplacian(g)
        self.D = mac.divergence(g)
        self.G = mac.gradient(g)
        self.nv, self.nc = g.nv, g.ncell
        self.nm = 0 if fluid_only else self.r.shape[0]
        self.nb = 0 if fluid_only else self.q.shape[0]
        blocks = [[-g.eta * self.Lm, self.G], [-self.D, None]]
        if not fluid_only:
            self.J = ib.interpolation(g, self.r)
            self.S = (self.J.T / g.dV).tocsr()
            self.K = B.geometric_matrix(self.theta, self.r_ref, self.offsets)
            blocks = [[-g.eta * self.Lm, self.G, -self.S, None],
                      [-self.D, None, None, None],
                      [-self.J, None, None, self.K],
                      [None, None, self.K.T, None]]
        self.A = sp.bmat(blocks, format="csr")
        self.n = self.A.shape[0]
        self.sl_v = slice(0, self.nv)
        self.sl_p = slice(self.nv, self.nv + self.nc)
        self.sl_l = slice(self.nv + self.nc, self.nv + self.nc + 3 * self.nm)
        self.sl_u = slice(self.nv + self.nc + 3 * self.nm, self.n)

    # ------------------------------------------------------------------ rhs
    def rhs(self, FT=None, slip=None, fluid=None, include_bc: bool = True) -> np.ndarray:
        b = np.zeros(self.n)
        if fluid is not None:
            b[self.sl_v] += fluid
        if include_bc:
            b[self.sl_v] += mac.moving_wall_rhs(self.g)
        if not self.fluid_only:
            lam_rhs = np.zeros((self.nm, 3))
            if slip is not None:
                lam_rhs -= np.asarray(slip).reshape(-1, 3)
            if include_bc:
                lam_rhs += ib.interpolation_bc(self.g, self.r)
            b[self.sl_l] = lam_rhs.ravel()
            if FT is not None:
                b[self.sl_u] = np.asarray(FT).ravel()
        return b

    def split(self, x: np.ndarray):
        """(v compact, pi, lambda [nm,3], U [nb,6])."""
        return (x[self.sl_v], x[self.sl_p], x[self.sl_l].reshape(-1, 3), x[self.sl_u].reshape(-1, 6))

    def residual(self, x: np.ndarray, b: np.ndarray) -> float:
        return float(np.linalg.norm(b - self.A @ x) / max(np.linalg.norm(b), 1e-300))

    # -------------------------------------------------------------- solvers
    def solve_direct(self, b: np.ndarray) -> np.ndarray:
        """Sparse LU of [[A, e],[e^T, 0]] with e the pressure-mean indicator."""
        e = np.zeros(self.n)
        e[self.sl_p] = 1.0
        Ab = sp.bmat([[self.A, sp.csr_matrix(e[:, None])], [sp.csr_matrix(e[None, :]), None]], format="csc")
        xb = spla.spsolve(Ab, np.concatenate([b, [0.0]]))
        return xb[:-1]

    def solve_fgmres(self, b: np.ndarray, tol: float = 1e-12, restart: int = 80, max_iter: int = 2000,
                     blob_radius: Optional[float] = None):
        pc = _OraclePreconditioner(self, blob_radius)
        x, info = fgmres(lambda z: self.A @ z, pc.apply, b, tol=tol, restart=restart, max_iter=max_iter)
        return x, info

    def solve(self, b: np.ndarray, tol: float = 1e-12) -> np.ndarray:
        """Exact discrete solution: direct for small systems, FGMRES otherwise."""
        if self.n <= 3000:
            x = self.solve_direct(b)
        else:
            x, _ = self.solve_fgmres(b, tol=tol)
        x = x.copy()
        x[self.sl_p] -= np.mean(x[self.sl_p])
        return x


def fgmres(matvec, precond, b, tol=1e-12, restart=80, max_iter=2000, x0=None):
    """Right-preconditioned flexible GMRES (Saad 1993) with modified Gram-Schmidt.

    Stops when the true residual ||b - A x|| <= tol ||b||; returns (x, info dict).
    """
    n = b.shape[0]
    x = np.zeros(n) if x0 is None else x0.copy()
    bnorm = np.linalg.norm(b)
    if bnorm == 0.0:
        return x, {"iters": 0, "rel_residual": 0.0}
    it = 0
    r = b - matvec(x)
    beta = np.linalg.norm(r)
    while it < max_iter:
        if beta <= tol * bnorm:
            break
        V = np.zeros((restart + 1, n))
        Z = np.zeros((restart, n))
        H = np.zeros((restart + 1, restart))
        V[0] = r / beta
        gvec = np.zeros(restart + 1)
        gvec[0] = beta
        cs = np.zeros(restart)
        sn = np.zeros(restart)
        j_end = 0
        for j in range(restart):
            Z[j] = precond(V[j])
            w = matvec(Z[j])
            for i in range(j + 1):
                H[i, j] = np.dot(V[i], w)
                w -= H[i, j] * V[i]
            H[j + 1, j] = np.linalg.norm(w)
            if H[j + 1, j] > 0:
                V[j + 1] = w / H[j + 1, j]
            for i in range(j):
                t = cs[i] * H[i, j] + sn[i] * H[i + 1, j]
                H[i + 1, j] = -sn[i] * H[i, j] + cs[i] * H[i + 1, j]
                H[i, j] = t
            den = math.hypot(H[j, j], H[j + 1, j])
            cs[j] = H[j, j] / den
            sn[j] = H[j + 1, j] / den
            H[j, j] = den
            H[j + 1, j] = 0.0
            gvec[j + 1] = -sn[j] * gvec[j]
            gvec[j] = cs[j] * gvec[j]
            it += 1
            j_end = j + 1
            if abs(gvec[j + 1]) <= tol * bnorm or it >= max_iter:
                break
        y = sla.solve_triangular(H[:j_end, :j_end], gvec[:j_end])
        x += Z[:j_end].T @ y
        r = b - matvec(x)
        beta = np.linalg.norm(r)
    return x, {"iters": it, "rel_residual": float(beta / bnorm)}


# ---------------------------------------------------------------------------
# Oracle-only preconditioner: exact fast Poisson solves per component.

def _axis_eigs(N: int, h: float, kind: str) -> np.ndarray:
    if kind == "fft":
        k = np.arange(N)
        return -(4.0 / h**2) * np.sin(np.pi * k / N) ** 2
    if kind == "dst1":           # N - 1 unknowns between two Dirichlet faces
        k = np.arange(1, N)
        return -(4.0 / h**2) * np.sin(np.pi * k / (2 * N)) ** 2
    if kind == "dst2":           # N cell centres, odd ghosts
        k = np.arange(1, N + 1)
        return -(4.0 / h**2) * np.sin(np.pi * k / (2 * N)) ** 2
    if kind == "dct2":           # N cell centres, even ghosts (Neumann)
        k = np.arange(N)
        return -(4.0 / h**2) * np.sin(np.pi * k / (2 * N)) ** 2
    raise ValueError(kind)


def _fwd(x, kind, axis):
    if kind == "fft":
        return sfft.fft(x, axis=axis)
    if kind == "dst1":
        return sfft.dst(x, type=1, axis=axis, norm="ortho")
    if kind == "dst2":
        return sfft.dst(x, type=2, axis=axis, norm="ortho")
    return sfft.dct(x, type=2, axis=axis, norm="ortho")


def _inv(x, kind, axis):
    if kind == "fft":
        return sfft.ifft(x, axis=axis)
    if kind == "dst1":
        return sfft.idst(x, type=1, axis=axis, norm="ortho")
    if kind == "dst2":
        return sfft.idst(x, type=2, axis=axis, norm="ortho")
    return sfft.idct(x, type=2, axis=axis, norm="ortho")


class _FastPoisson:
    """Exact inverse of a separable 7-point Laplacian by per-axis transforms."""

    def __init__(self, dims, kinds, h):
        self.dims = dims              # (nx, ny, nz) of the unknown array
        self.kinds = kinds
        eig = np.zeros(dims[::-1])
        for a in range(3):
            shape = [1, 1, 1]
            shape[2 - a] = dims[a]
            eig = eig + _axis_eigs(dims[a] + (1 if kinds[a] == "dst1" else 0), h, kinds[a]).reshape(shape)
        self.eig = eig
        self.singular = np.abs(eig) < 1e-14

    def solve(self, f: np.ndarray) -> np.ndarray:
        """Solve L u = f (L the separable Laplacian); singular modes set to zero."""
        x = f.reshape(self.dims[::-1]).astype(np.complex128 if "fft" in self.kinds else np.float64)
        for a in range(3):
            x = _fwd(x, self.kinds[a], 2 - a)
        x = np.where(self.singular, 0.0, x / np.where(self.singular, 1.0, self.eig))
        for a in range(3):
            x = _inv(x, self.kinds[a], 2 - a)
        return np.real(x).ravel()


def rpy_mobility(x: np.ndarray, a: float, eta: float) -> np.ndarray:
    """Free-space Rotne-Prager-Yamakawa blob mobility (3n x 3n), used only to precondition."""
    n = x.shape[0]
    M = np.zeros((n, 3, n, 3))
    c0 = 1.0 / (6.0 * math.pi * eta * a)
    I = np.eye(3)
    for i in range(n):
        for j in range(n):
            d = x[i] - x[j]
            r = np.linalg.norm(d)
            if i == j:
                M[i, :, j, :] = c0 * I
                continue
            e = np.outer(d, d) / r**2
            if r >= 2 * a:
                M[i, :, j, :] = (1.0 / (8.0 * math.pi * eta * r)) * ((1 + 2 * a * a / (3 * r * r)) * I
                                                                    + (1 - 2 * a * a / (r * r)) * e)
            else:
                M[i, :, j, :] = c0 * ((1 - 9 * r / (32 * a)) * I + (3 * r / (32 * a)) * e)
    return M.reshape(3 * n, 3 * n)


class _OraclePreconditioner:
    """Upper block-triangular: bodies first (RPY block per body), then a projection
    step with exact component solves for the fluid."""

    def __init__(self, s: Saddle, blob_radius: Optional[float]):
        self.s = s
        g = s.g
        self.comp = []
        for c in range(3):
            dims = tuple(g.n[a] - 1 if (a == c and g.bc[a] != PERIODIC) else g.n[a] for a in range(3))
            kinds = tuple("fft" if g.bc[a] == PERIODIC else
                          ("dst1" if a == c else ("dct2" if g.bc[a] == SLIP else "dst2")) for a in range(3))
            self.comp.append(_FastPoisson(dims, kinds, g.h))
        self.pres = _FastPoisson(g.n, tuple("fft" if g.bc[a] == PERIODIC else "dct2" for a in range(3)), g.h)
        self.bodies = []
        if not s.fluid_only:
            a = 1.25 * g.h if blob_radius is None else blob_radius
            d = B.marker_offsets(s.theta, s.r_ref, s.offsets)
            for p in range(s.nb):
                lo, hi = s.offsets[p], s.offsets[p + 1]
                M = rpy_mobility(d[lo:hi], a, g.eta)
                Kp = B.geometric_matrix(s.theta[p:p + 1], s.r_ref[lo:hi], np.array([0, hi - lo])).toarray()
                Mc = sla.cho_factor(M)
                Ninv = Kp.T @ sla.cho_solve(Mc, Kp)
                self.bodies.append((lo, hi, Mc, Kp, np.linalg.inv(Ninv)))

    def _fluid(self, rv, rp):
        g = self.s.g
        vs = np.empty_like(rv)
        for c in range(3):
            sl = slice(g.face_offset[c], g.face_offset[c] + g.nface[c])
            vs[sl] = self.comp[c].solve(-rv[sl] / g.eta)
        div = self.s.D @ vs + rp
        phi = self.pres.solve(div)
        v = vs - self.s.G @ phi
        p = -g.eta * div
        return v, p

    def apply(self, r: np.ndarray) -> np.ndarray:
        s = self.s
        out = np.zeros_like(r)
        rv = r[s.sl_v].copy()
        if not s.fluid_only:
            rl = r[s.sl_l].reshape(-1, 3)
            ru = r[s.sl_u].reshape(-1, 6)
            lam = np.zeros_like(rl)
            U = np.zeros_like(ru)
            for p, (lo, hi, Mc, Kp, N) in enumerate(self.bodies):
                gl = rl[lo:hi].ravel()
                Up = N @ (ru[p] + Kp.T @ sla.cho_solve(Mc, gl))
                lam[lo:hi] = sla.cho_solve(Mc, Kp @ Up - gl).reshape(-1, 3)
                U[p] = Up
            out[s.sl_l] = lam.ravel()
            out[s.sl_u] = U.ravel()
            rv = rv + s.S @ lam.ravel()
        v, p = self._fluid(rv, r[s.sl_p])
        out[s.sl_v] = v
        out[s.sl_p] = p
        return out
