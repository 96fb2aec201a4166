"""Seeded synthetic inputs shared by the oracle, the tests and the benchmark.

This module holds data only: rigid-body marker geometries and seeded draws of
body positions, orientations and forces for the confined-suspension
workloads.  It contains none of the method's arithmetic (no grid operator,
no delta kernel, no solver), so both the CPU oracle and the GPU path may use
it without sharing computation.

Geometries (the paper builds spheres as rigid agglomerates of blobs, Sec. III.B):
  * ``icosahedron(R)``     -- the 12 vertices of a regular icosahedron,
  * ``icosphere42(R)``     -- those 12 plus the 30 edge midpoints, projected
                              back to radius R (one subdivision).

Workloads (all with h = 1 and viscosity 1):
  * ``single_sphere``      -- 32^3 box, no-slip on all faces, one 42-marker
                              sphere of radius 2.5 h near the centre.
  * ``two_spheres``        -- 32x32x64 box, walls, two 42-marker spheres.
  * ``monolayer``          -- 256x128x32, periodic in x, walls in y and z,
                              bottom wall sliding at +0.5 in x, 1024 twelve-
                              marker spheres (radius 1.5 h) in a triangular
                              lattice.
  * ``ensemble``           -- many independent walled boxes of edge
                              16/24/32/48 with 1-4 spheres each.
  * ``many_spheres``       -- 128^3 walled box with 64 spheres.
  * ``boomerang_slit``     -- replicas of one 15-blob L-shaped boomerang in a
                              64x64x16 slit (periodic in x and y, no-slip
                              walls in z), 6-point kernel (App. A).
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional, Sequence, Tuple

import numpy as np

PERIODIC = 0
WALL = 1          # no-slip wall
SLIP = 2          # free-slip wall

GOLDEN = (1.0 + math.sqrt(5.0)) / 2.0


def icosahedron(radius: float) -> np.ndarray:
    """12 icosahedron vertices (0, +-1, +-g) and cyclic shifts, scaled to ``radius``.

    Order: for each cyclic shift s = 0, 1, 2 of the coordinate triple, the four
    sign choices (+,+), (+,-), (-,+), (-,-) of (1, g).
    """
    pts = []
    for s in range(3):
        for sa in (1.0, -1.0):
            for sb in (1.0, -1.0):
                v = [0.0, sa * 1.0, sb * GOLDEN]
                v = v[-s:] + v[:-s] if s else v
                pts.append(v)
    p = np.array(pts, dtype=np.float64)
    p /= np.linalg.norm(p, axis=1, keepdims=True)
    return p * radius


def icosphere42(radius: float) -> np.ndarray:
    """12 vertices + 30 edge midpoints (edges sorted by vertex pair), all at ``radius``."""
    v = icosahedron(1.0)
    d = np.linalg.norm(v[:, None, :] - v[None, :, :], axis=2)
    emin = d[d > 1e-12].min()
    mids = []
    for i in range(12):
        for j in range(i + 1, 12):
            if abs(d[i, j] - emin) < 1e-9:
                m = 0.5 * (v[i] + v[j])
                mids.append(m / np.linalg.norm(m))
    assert len(mids) == 30
    p = np.vstack([v, np.array(mids)])
    return p * radius


def random_unit_quaternions(rng: np.random.Generator, n: int) -> np.ndarray:
    """Uniform random unit quaternions (scalar first) from normalised N(0,1)^4."""
    q = rng.standard_normal((n, 4))
    q /= np.linalg.norm(q, axis=1, keepdims=True)
    return q


@dataclasses.dataclass
class Workload:
    """One confined suspension: grid, boundary conditions and rigid bodies."""
    name: str
    n: Tuple[int, int, int]
    bc: Tuple[int, int, int]
    h: float
    eta: float
    # wall_vel[axis][side][component]: tangential velocity of each wall
    wall_vel: np.ndarray
    r_ref: np.ndarray             # (nm, 3) body-frame marker offsets, concatenated
    offsets: np.ndarray           # (nb + 1,) int32 CSR body -> markers
    q: np.ndarray                 # (nb, 3) body positions
    theta: np.ndarray             # (nb, 4) unit quaternions, scalar first
    FT: np.ndarray                # (nb, 6) forces and torques
    radius: np.ndarray            # (nb,) geometric sphere radius (for forces/rejection)
    kT: float = 0.0
    dt: float = 0.0
    tol: float = 1e-8
    seed: int = 0
    kernel: int = 4               # width of the delta kernel (4 or 6)

    @property
    def nb(self) -> int:
        return int(self.q.shape[0])

    @property
    def nm(self) -> int:
        return int(self.r_ref.shape[0])


def _bodies(shapes: Sequence[np.ndarray]):
    r_ref = np.vstack(shapes).astype(np.float64)
    offs = np.zeros(len(shapes) + 1, dtype=np.int32)
    offs[1:] = np.cumsum([s.shape[0] for s in shapes])
    return r_ref, offs


def _place_nonoverlapping(rng, n_bodies, lo, hi, min_dist, max_tries=100000):
    """Rejection-sample centres uniformly in the box [lo, hi] with pair distance >= min_dist."""
    pts: List[np.ndarray] = []
    tries = 0
    while len(pts) < n_bodies:
        tries += 1
        if tries > max_tries:
            raise RuntimeError("could not place bodies without overlap")
        c = lo + (hi - lo) * rng.random(3)
        if all(np.linalg.norm(c - p) >= min_dist for p in pts):
            pts.append(c)
    return np.array(pts, dtype=np.float64)


def zero_wall_vel() -> np.ndarray:
    return np.zeros((3, 2, 3), dtype=np.float64)


def single_sphere(seed: int = 1901, n: int = 32) -> Workload:
    """One 42-marker sphere (R = 2.5 h) in an n^3 walled box, centre n/2 + U(-2, 2)^3."""
    rng = np.random.default_rng(seed)
    R = 2.5
    r_ref, offs = _bodies([icosphere42(R)])
    q = (n / 2.0 + rng.uniform(-2.0, 2.0, size=3))[None, :]
    theta = random_unit_quaternions(rng, 1)
    FT = rng.standard_normal((1, 6))
    return Workload("single_sphere", (n, n, n), (WALL, WALL, WALL), 1.0, 1.0, zero_wall_vel(),
                    r_ref, offs, q, theta, FT, np.array([R]), tol=1e-8, seed=seed)


def spheres_in_box(seed: int, n: Tuple[int, int, int], n_bodies: int, R: float = 2.5,
                   shape: str = "ico42", gap: float = 1.0, name: str = "spheres_in_box",
                   kT: float = 1.0, dt: float = 0.01, tol: float = 1e-6) -> Workload:
    """``n_bodies`` equal spheres at seeded non-overlapping positions in a walled box.

    Centres are uniform in [R + gap, n - R - gap] per axis with centre distance
    >= 2R + gap; forces and torques are N(0, 1).
    """
    rng = np.random.default_rng(seed)
    geo = icosphere42(R) if shape == "ico42" else icosahedron(R)
    r_ref, offs = _bodies([geo] * n_bodies)
    lo = np.full(3, R + gap)
    hi = np.array(n, dtype=np.float64) - R - gap
    q = _place_nonoverlapping(rng, n_bodies, lo, hi, 2 * R + gap)
    theta = random_unit_quaternions(rng, n_bodies)
    FT = rng.standard_normal((n_bodies, 6))
    return Workload(name, tuple(n), (WALL, WALL, WALL), 1.0, 1.0, zero_wall_vel(),
                    r_ref, offs, q, theta, FT, np.full(n_bodies, R), kT=kT, dt=dt, tol=tol,
                    seed=seed)


def two_spheres(seed: int = 1902) -> Workload:
    """Two 42-marker spheres (R = 2.5 h) tightly confined in a 32x32x64 walled box."""
    return spheres_in_box(seed, (32, 32, 64), 2, name="two_spheres", kT=1.0, dt=0.01, tol=1e-6)


def many_spheres(seed: int = 1905, n: int = 128, n_bodies: int = 64) -> Workload:
    """64 spheres of 42 markers in a 128^3 walled box (the differentiated-solve workload)."""
    return spheres_in_box(seed, (n, n, n), n_bodies, name="many_spheres", tol=1e-12)


def monolayer(seed: int = 1903, n=(256, 128, 32), rows: int = 16, cols: int = 64,
              spacing: float = 4.0, R: float = 1.5, wall_speed: float = 0.5) -> Workload:
    """Quasi-2D colloidal monolayer in a microchannel.

    ``rows`` x ``cols`` twelve-marker spheres on a triangular lattice with
    spacing ``spacing`` (rows sqrt(3)/2 * spacing apart, alternate rows shifted
    by half a spacing), centred in y, at height R + 1 above the bottom wall,
    with seeded U(-0.25, 0.25) jitter in x and y.  Periodic in x, walls in y
    and z; the bottom (z = 0) wall slides at ``wall_speed`` along +x.
    """
    rng = np.random.default_rng(seed)
    nx, ny, nz = n
    dy = spacing * math.sqrt(3.0) / 2.0
    y0 = ny / 2.0 - dy * (rows - 1) / 2.0
    cs = []
    for r in range(rows):
        for c in range(cols):
            x = (c + 0.5 * (r % 2) + 0.25) * spacing
            cs.append([x % nx, y0 + r * dy, R + 1.0])
    q = np.array(cs, dtype=np.float64)
    q[:, :2] += rng.uniform(-0.25, 0.25, size=(q.shape[0], 2))
    nb = q.shape[0]
    r_ref, offs = _bodies([icosahedron(R)] * nb)
    theta = random_unit_quaternions(rng, nb)
    FT = rng.standard_normal((nb, 6))
    wv = zero_wall_vel()
    wv[2, 0, 0] = wall_speed
    return Workload("monolayer", tuple(n), (PERIODIC, WALL, WALL), 1.0, 1.0, wv, r_ref, offs,
                    q, theta, FT, np.full(nb, R), kT=1.0, dt=0.01, tol=1e-6, seed=seed)


def ensemble(seed: int = 1904, n_replicas: int = 256, sizes=(16, 24, 32, 48),
             max_bodies: int = 4) -> List[Workload]:
    """Independent walled replicas: edge drawn from ``sizes``, 1..max_bodies spheres each."""
    rng = np.random.default_rng(seed)
    out = []
    for r in range(n_replicas):
        n = int(rng.choice(sizes))
        nb = int(rng.integers(1, max_bodies + 1))
        sub_seed = int(rng.integers(0, 2**31 - 1))
        w = spheres_in_box(sub_seed, (n, n, n), nb, name=f"replica{r}", kT=1.0, dt=0.01, tol=1e-6)
        out.append(w)
    return out


def small_box(seed: int, n=(12, 12, 12), n_bodies: int = 1, R: float = 1.5, shape: str = "ico12",
              bc=(WALL, WALL, WALL), wall_vel: Optional[np.ndarray] = None, gap: float = 0.6) -> Workload:
    """Tiny configurations for dense brute-force checks."""
    w = spheres_in_box(seed, n, n_bodies, R=R, shape=shape, gap=gap, name="small_box")
    w.bc = tuple(bc)
    if wall_vel is not None:
        w.wall_vel = np.asarray(wall_vel, dtype=np.float64)
    return w


# ---------------------------------------------------------------- App. A boomerang
# Units: the mesh width h, the viscosity eta and kT are 1.  The blob radius of
# the 6-point kernel is a = 1.47 h and the blobs are s = 0.925 a apart; with
# s = 0.3 um this makes h = 0.3 um / (0.925 * 1.47) = 0.2206 um.
BOOMERANG_A = 1.47
BOOMERANG_S = 0.925 * BOOMERANG_A
BOOMERANG_N = (64, 64, 16)
_KB, _T, _G = 1.380649e-23, 300.0, 9.80665            # J/K, K, m/s^2
_H_M = 0.3e-6 / BOOMERANG_S                          # mesh width in metres
_M_E = 1.57e-11 * 1e-6                               # buoyant mass per blob: 1.57e-11 mg, in kg
BOOMERANG_POTENTIAL = dict(
    phi0=4.0,                                        # 4 kT
    d=BOOMERANG_A,                                   # d = a
    b=0.1 * BOOMERANG_A,                             # b = 0.1 a
    weight=_M_E * _G * _H_M / (_KB * _T),            # m_e g in kT / h (about 8.2e-3)
)


def boomerang_shape(s: float = BOOMERANG_S) -> np.ndarray:
    """15 blobs: the cross point at the origin, then 7 along +x and 7 along +y, s apart."""
    pts = [[0.0, 0.0, 0.0]]
    pts += [[k * s, 0.0, 0.0] for k in range(1, 8)]
    pts += [[0.0, k * s, 0.0] for k in range(1, 8)]
    return np.array(pts, dtype=np.float64)


# unit vector in the plane of the boomerang bisecting the right angle at the
# cross point, pointing from the arms towards the cross point (body frame)
BOOMERANG_P = np.array([-1.0, -1.0, 0.0]) / math.sqrt(2.0)


def boomerang_dt(dtau: float, a: float = BOOMERANG_A) -> float:
    """Time step of the dimensionless step dtau = dt kT / (6 pi eta a^3)."""
    return dtau * 6.0 * math.pi * a ** 3


def boomerang_slit(seed: int = 1906, n_replicas: int = 1, dtau: float = 0.036, tol: float = 1e-6,
                   z0: Optional[float] = None) -> List[Workload]:
    """Replicas of one boomerang in the App. A slit, tracking point at the cross point.

    Each replica starts flat (the L in a horizontal plane) at height z0
    (default: mid-slit), at a seeded uniform (x, y) and a seeded rotation
    about z.  Forces are configuration dependent (evaluated each step by the
    caller), so FT is zero here.
    """
    rng = np.random.default_rng(seed)
    nx, ny, nz = BOOMERANG_N
    r_ref, offs = _bodies([boomerang_shape()])
    wv = zero_wall_vel()
    out = []
    for r in range(n_replicas):
        xy = rng.uniform(0.0, 1.0, 2) * np.array([nx, ny], dtype=np.float64)
        alpha = rng.uniform(0.0, 2.0 * math.pi)
        q = np.array([[xy[0], xy[1], nz / 2.0 if z0 is None else z0]])
        theta = np.array([[math.cos(0.5 * alpha), 0.0, 0.0, math.sin(0.5 * alpha)]])
        out.append(Workload("boomerang%d" % r, BOOMERANG_N, (PERIODIC, PERIODIC, WALL), 1.0, 1.0, wv.copy(),
                            r_ref.copy(), offs.copy(), q, theta, np.zeros((1, 6)), np.array([BOOMERANG_S * 7]),
                            kT=1.0, dt=boomerang_dt(dtau), tol=tol, seed=seed, kernel=6))
    return out
