"""Named synthetic configurations shared by the GPU parity tests and the script
that stores the oracle's error gains for them (tests/golden/make_error_gains.py).
Inputs only: seeded geometry, positions, forces and slip; no arithmetic of the
method."""
from __future__ import annotations

import numpy as np

import workloads as W


def solve_configs():
    """Operator-apply and mobility-solve cases: walled, periodic, ragged (partial tiles),
    a one-cell last tile on a periodic axis, the sliding-wall monolayer, and two
    replicas of the benchmark ensemble (the crowded 16^3 box with four spheres that
    sets the length of the batched iteration loop, and a 48^3 box)."""
    out = {
        "single_sphere_32": W.single_sphere(),
        "two_spheres_32x32x64": W.two_spheres(),
        "ragged_10x12x14": W.small_box(21, n=(10, 12, 14), n_bodies=3, R=1.5, shape="ico12"),
    }
    w = W.small_box(22, n=(16, 12, 12), n_bodies=3, R=1.5, shape="ico12")
    w.bc = (W.PERIODIC, W.WALL, W.WALL)
    out["periodic_x_16x12x12"] = w
    # periodic x of 17 cells: the last tile holds one cell, and markers of the body
    # at x = 0.15 h in cell 0 reach cell 15 (tile 3) through the wrap
    w = W.small_box(23, n=(17, 12, 12), n_bodies=2, R=1.5, shape="ico12")
    w.bc = (W.PERIODIC, W.WALL, W.WALL)
    w.q[0, 0] = 0.15 * w.h
    out["periodic_wrap_17x12x12"] = w
    out["monolayer_64x32x16"] = W.monolayer(n=(64, 32, 16), rows=4, cols=16)
    out.update(ensemble_replicas())
    return out


def ensemble_replicas():
    """The first 16^3 replica with four spheres and the first 48^3 replica of the
    256-replica benchmark ensemble, with their ensemble index."""
    ens = W.ensemble()
    k16 = next(k for k, w in enumerate(ens) if w.n[0] == 16 and w.nb == 4)
    k48 = next(k for k, w in enumerate(ens) if w.n[0] == 48)
    a, b = ens[k16], ens[k48]
    a.name, b.name = "ensemble_%d" % k16, "ensemble_%d" % k48
    return {"ensemble16_4spheres": a, "ensemble48": b}


def kernel6_configs():
    """The paper's 6-point kernel on walled, periodic (with a one-cell last tile and a
    wrap), ragged, sliding-wall and ensemble-like boxes."""
    import copy
    base = solve_configs()
    out = {}
    for name in ("ragged_10x12x14", "periodic_wrap_17x12x12", "monolayer_64x32x16", "ensemble16_4spheres"):
        w = copy.deepcopy(base[name])
        w.kernel = 6
        out[name + "_k6"] = w
    w = copy.deepcopy(sem_configs()["two_spheres_16x16x32"])
    w.kernel = 6
    out["two_spheres_16x16x32_k6"] = w
    return out


def slip_configs():
    """Free-slip walls: a closed free-slip box; a box periodic in x with no-slip walls
    in y and free-slip walls in z; a ragged box mixing both wall types; the 6-point
    kernel with free-slip walls."""
    import copy
    out = {}
    w = W.small_box(41, n=(12, 12, 16), n_bodies=3, R=1.5, shape="ico12")
    w.bc = (W.SLIP, W.SLIP, W.SLIP)
    out["slip_box_12x12x16"] = w
    w = W.small_box(42, n=(16, 12, 12), n_bodies=3, R=1.5, shape="ico12")
    w.bc = (W.PERIODIC, W.WALL, W.SLIP)
    out["periodic_x_wall_y_slip_z_16x12x12"] = w
    w = W.small_box(43, n=(10, 12, 14), n_bodies=3, R=1.5, shape="ico12")
    w.bc = (W.SLIP, W.WALL, W.SLIP)
    out["slip_wall_slip_10x12x14"] = w
    w = copy.deepcopy(out["periodic_x_wall_y_slip_z_16x12x12"])
    w.kernel = 6
    out["periodic_x_wall_y_slip_z_16x12x12_k6"] = w
    return out


def sem_configs():
    return {
        "two_spheres_16x16x32": W.spheres_in_box(31, (16, 16, 32), 2, name="two_small"),
        "two_spheres_32x32x64": W.two_spheres(),
        "monolayer_32x16x12_sliding": W.monolayer(n=(32, 16, 12), rows=2, cols=8),
    }


def boomerang_configs():
    """The App. A boomerang in its 64x64x16 slit (6-point kernel): tilted 40 degrees
    about x with the x arm 1.8 h above the bottom wall (its blobs inside the
    exponential range of the wall repulsion), and a replica whose cross point sits
    1.0 h below the top wall (inside the linear range)."""
    import math
    low = W.boomerang_slit(seed=41, n_replicas=1)[0]
    low.q = np.array([[20.3, 37.9, 1.8]])
    a = math.radians(40.0)
    low.theta = np.array([[math.cos(a / 2), math.sin(a / 2), 0.0, 0.0]])
    high = W.boomerang_slit(seed=42, n_replicas=1)[0]
    high.q = np.array([[50.2, 3.7, 15.0]])
    a = math.radians(-25.0)
    b = math.radians(60.0)
    # rotation about -x by 25 degrees, then about z by 60 degrees: arms go downwards
    qx = np.array([math.cos(a / 2), math.sin(a / 2), 0.0, 0.0])
    qz = np.array([math.cos(b / 2), 0.0, 0.0, math.sin(b / 2)])
    w_, x_, y_, z_ = qz
    high.theta = np.array([[w_ * qx[0] - x_ * qx[1], w_ * qx[1] + x_ * qx[0], y_ * qx[0] + z_ * qx[1],
                            z_ * qx[0] - y_ * qx[1]]])
    high.theta /= np.linalg.norm(high.theta)
    return {"boomerang_64x64x16_k6": low, "boomerang_top_64x64x16_k6": high}


def marker_slip(w, seed=17, scale=0.05):
    """A nonzero prescribed slip on every marker (Sec. II eq. rigidBC): a seeded random
    field plus a swirl about a fixed axis through each body's tracking point (the
    surface velocity of an active particle), both of size `scale`, lab frame."""
    rng = np.random.default_rng(seed)
    axis = np.array([0.3, -0.5, 0.8])
    d = w.r_ref / np.maximum(np.linalg.norm(w.r_ref, axis=1, keepdims=True), 1e-12)
    return scale * (rng.standard_normal((w.nm, 3)) + np.cross(axis, d))


def gain_configs():
    """Every configuration whose solves the GPU tests bound through the stored gains."""
    out = dict(solve_configs())
    out.pop("periodic_wrap_17x12x12")          # apply only
    for k, w in sem_configs().items():
        out.setdefault(k, w)
    for k, w in kernel6_configs().items():
        if k != "monolayer_64x32x16_k6":          # apply only
            out[k] = w
    out.update(slip_configs())
    out["boomerang_64x64x16_k6"] = boomerang_configs()["boomerang_64x64x16_k6"]
    return out
