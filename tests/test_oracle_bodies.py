"""Pins of the oracle's rigid-body maps (paper Sec. II and III.B).

* Quaternion rotation matrices agree with Rodrigues' axis-angle formula.
* Rotate(theta, phi) composes the lab-frame rotation exp([phi]_x) on the left.
* K and K^T are mutually adjoint; K^T K of one body has its closed form.
* L_p of the two sphere geometries is the sphere diameter.
* Tile binning is a stable sort by (tile, marker id) (brute-force check).
"""
import math

import numpy as np

import workloads as W
from oracle import bodies as B
from oracle import mac


def _rodrigues(phi):
    a = np.linalg.norm(phi)
    if a == 0:
        return np.eye(3)
    n = phi / a
    C = np.array([[0, -n[2], n[1]], [n[2], 0, -n[0]], [-n[1], n[0], 0]])
    return math.cos(a) * np.eye(3) + math.sin(a) * C + (1 - math.cos(a)) * np.outer(n, n)


def test_rotation_matrix_is_rodrigues():
    rng = np.random.default_rng(0)
    for _ in range(20):
        phi = rng.standard_normal(3)
        a = np.linalg.norm(phi)
        th = np.concatenate([[math.cos(a / 2)], math.sin(a / 2) * phi / a])[None, :]
        R = B.rotation_matrices(th)[0]
        assert np.abs(R - _rodrigues(phi)).max() < 1e-14


def test_rotate_composition():
    rng = np.random.default_rng(1)
    th = W.random_unit_quaternions(rng, 5)
    phi = rng.standard_normal((5, 3))
    th2 = B.rotate(th, phi)
    assert np.allclose(np.linalg.norm(th2, axis=1), 1.0, atol=1e-15)
    for p in range(5):
        lhs = B.rotation_matrices(th2[p:p + 1])[0]
        rhs = _rodrigues(phi[p]) @ B.rotation_matrices(th[p:p + 1])[0]
        assert np.abs(lhs - rhs).max() < 1e-13
    assert np.array_equal(B.rotate(th, np.zeros((5, 3))), th)


def test_K_adjoint_and_closed_form():
    rng = np.random.default_rng(2)
    shapes = [W.icosphere42(2.5), W.icosahedron(1.5), W.icosphere42(1.0)]
    r_ref = np.vstack(shapes)
    offs = np.array([0, 42, 54, 96])
    th = W.random_unit_quaternions(rng, 3)
    U = rng.standard_normal((3, 6))
    lam = rng.standard_normal((96, 3))
    KU = B.apply_K(th, r_ref, offs, U)
    KTl = B.apply_KT(th, r_ref, offs, lam)
    assert abs(np.sum(KU * lam) - np.sum(U * KTl)) < 1e-12
    K = B.geometric_matrix(th, r_ref, offs)
    assert np.abs(K @ U.ravel() - KU.ravel()).max() < 1e-14
    assert np.abs(K.T @ lam.ravel() - KTl.ravel()).max() < 1e-13
    # K^T K of body 0: [[n I, -[sum d]_x], [[sum d]_x, sum(|d|^2 I - d d^T)]]
    d = B.marker_offsets(th, r_ref, offs)[:42]
    KtK = (K.T @ K).toarray()[:6, :6]
    sd = d.sum(axis=0)
    C = np.array([[0, -sd[2], sd[1]], [sd[2], 0, -sd[0]], [-sd[1], sd[0], 0]])
    I = sum(np.dot(x, x) * np.eye(3) - np.outer(x, x) for x in d)
    ref = np.block([[42 * np.eye(3), -C], [C, I]])
    assert np.abs(KtK - ref).max() < 1e-12


def test_body_length_and_geometry():
    s42 = W.icosphere42(2.5)
    s12 = W.icosahedron(1.5)
    assert np.allclose(np.linalg.norm(s42, axis=1), 2.5)
    offs = np.array([0, 42, 54])
    L = B.body_length(np.vstack([s42, s12]), offs)
    assert abs(L[0] - 5.0) < 1e-12 and abs(L[1] - 3.0) < 1e-12
    # minimum marker spacing of the 42-point sphere ~ 1.37 h at R = 2.5 h
    dd = np.linalg.norm(s42[:, None] - s42[None], axis=2) + np.eye(42) * 99
    assert 1.3 < dd.min() < 1.45


def test_tiles_stable_sort():
    g = mac.Grid((16, 12, 20), (0, 1, 1))
    rng = np.random.default_rng(3)
    r = rng.uniform(0.01, 1.0, size=(300, 3)) * np.array(g.n)
    r[:7, 0] -= 16.0          # periodic axis: wrapped
    tile, perm = B.marker_tiles(g, r)
    td = B.tile_dims(g)
    for i in range(300):
        c = [int(math.floor(r[i, a] / g.h)) % g.n[a] for a in range(3)]
        t = c[0] // 4 + td[0] * (c[1] // 4 + td[1] * (c[2] // 4))
        assert tile[i] == t
    ref = sorted(range(300), key=lambda i: (tile[i], i))
    assert perm.tolist() == ref


def test_K_rotation_sense_matches_marker_motion():
    """(K U)_i must be the velocity with which marker i actually moves when body p
    turns with angular velocity omega (Sec. II; K of Sec. III.B): the central
    difference of r_i(q, Rotate(theta, +eps omega)) and r_i(q, Rotate(theta, -eps
    omega)) over 2 eps equals K [0, omega] to O(eps^2).  Adjointness holds for either
    sign of the cross product, and the K^T K closed form on a body with sum d = 0 does
    not see it, so this is what fixes the rotation sense.  Bodies whose marker offsets
    do not sum to zero (the sphere shifted off its tracking point) are included."""
    rng = np.random.default_rng(7)
    shapes = [W.icosphere42(2.5) + np.array([0.4, -0.2, 0.9]), W.icosahedron(1.5), W.icosahedron(1.0) * 0.7]
    r_ref = np.vstack(shapes)
    offs = np.array([0, 42, 54, 66])
    q = rng.standard_normal((3, 3)) * 3.0
    th = W.random_unit_quaternions(rng, 3)
    omega = rng.standard_normal((3, 3))
    eps = 1e-5
    rp = B.marker_positions(q, B.rotate(th, eps * omega), r_ref, offs)
    rm = B.marker_positions(q, B.rotate(th, -eps * omega), r_ref, offs)
    vel = (rp - rm) / (2 * eps)
    U = np.concatenate([np.zeros((3, 3)), omega], axis=1)
    KU = B.apply_K(th, r_ref, offs, U)
    assert np.abs(vel - KU).max() < 1e-8 * np.abs(KU).max()
    # a translation moves every marker of its body rigidly
    U = np.concatenate([rng.standard_normal((3, 3)), np.zeros((3, 3))], axis=1)
    assert np.abs(B.apply_K(th, r_ref, offs, U) - U[B.body_of_marker(offs), :3]).max() == 0.0
