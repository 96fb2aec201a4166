"""Pins of the oracle's caller-side forces (eq. Usoft, constant force) and of
its Gibbs-Boltzmann reference for the App. A boomerang.

The profile is pinned by its closed-form properties, forces and torques by
central differences of the energy, the quadrature route by a one-dimensional
Boltzmann integral and the Haar angle law, and the Metropolis chain and the
exact sampler by the quadrature.
"""
import math

import numpy as np
import pytest
from scipy import integrate

import workloads as W
from oracle.bodies import rotate
from oracle.gibbs import angle_with_z, gb_marginals, gb_samples, haar_quaternions, metropolis, slit_energy
from oracle.mac import Grid, PERIODIC, WALL, SLIP
from oracle.potentials import body_energy, body_forces, soft_profile

PHI0, D, B = 4.0, 1.47, 0.147


def test_soft_profile_closed_form():
    eps = 1e-9
    v_in, s_in = soft_profile(D - eps, PHI0, D, B)
    v_out, s_out = soft_profile(D + eps, PHI0, D, B)
    assert abs(v_in - PHI0) < 1e-6 and abs(v_out - PHI0) < 1e-6          # continuous at r = d
    assert abs(s_in + PHI0 / B) < 1e-12 and abs(s_out + PHI0 / B) < 1e-6  # C^1: slope -phi0/b both sides
    v, _ = soft_profile(D + B * math.log(2.0), PHI0, D, B)
    assert abs(v - PHI0 / 2) < 1e-12                                      # half strength one b ln 2 out
    v0, _ = soft_profile(0.0, PHI0, D, B)
    assert abs(v0 - PHI0 * (1.0 + D / B)) < 1e-12                         # linear branch at the face
    r = np.linspace(D, D + 3.0, 7)
    v1, _ = soft_profile(r, PHI0, D, B)
    v2, _ = soft_profile(r + B, PHI0, D, B)
    assert np.allclose(v2 / v1, math.exp(-1.0), rtol=1e-13)               # exponential tail, length b
    # derivative against a central difference on both branches
    for x in (0.3, 1.0, 1.6, 2.4):
        h = 1e-6
        fd = (soft_profile(x + h, PHI0, D, B)[0] - soft_profile(x - h, PHI0, D, B)[0]) / (2 * h)
        assert abs(fd - soft_profile(x, PHI0, D, B)[1]) < 1e-6 * PHI0 / B


def _bodies_case(rng):
    g = Grid((12, 10, 8), (PERIODIC, WALL, SLIP), 1.0, 1.0)
    r_ref = np.vstack([W.boomerang_shape(0.6), W.icosahedron(1.2)])
    offs = np.array([0, 15, 27], dtype=np.int32)
    q = np.array([[3.0, 2.4, 2.2], [8.0, 6.0, 5.6]]) + rng.uniform(-0.3, 0.3, (2, 3))
    th = haar_quaternions(rng, 2)
    return g, r_ref, offs, q, th


def test_forces_are_minus_energy_gradient():
    rng = np.random.default_rng(3)
    g, r_ref, offs, q, th = _bodies_case(rng)
    fc = np.array([0.01, -0.02, -0.05])
    args = (PHI0, D, B, fc)
    FT = body_forces(g, q, th, r_ref, offs, *args)
    h = 1e-6
    for p in range(2):
        for k in range(3):
            dq = np.zeros_like(q); dq[p, k] = h
            fd = (body_energy(g, q + dq, th, r_ref, offs, *args)[p]
                  - body_energy(g, q - dq, th, r_ref, offs, *args)[p]) / (2 * h)
            assert abs(FT[p, k] + fd) < 1e-6 * (1.0 + abs(fd)), (p, k, FT[p, k], fd)
            phi = np.zeros((2, 3)); phi[p, k] = h
            fd = (body_energy(g, q, rotate(th, phi), r_ref, offs, *args)[p]
                  - body_energy(g, q, rotate(th, -phi), r_ref, offs, *args)[p]) / (2 * h)
            assert abs(FT[p, 3 + k] + fd) < 1e-6 * (1.0 + abs(fd)), (p, k, FT[p, 3 + k], fd)
    # the periodic axis carries no wall force; the constant force alone along x
    assert np.allclose(FT[:, 0], [15 * fc[0], 12 * fc[0]], atol=1e-14)


def test_constant_force_only():
    rng = np.random.default_rng(4)
    g, r_ref, offs, q, th = _bodies_case(rng)
    fc = np.array([0.0, 0.0, -1.0])
    FT = body_forces(g, q, th, r_ref, offs, 0.0, D, B, fc)
    from oracle.bodies import marker_offsets
    dd = marker_offsets(th, r_ref, offs)
    assert np.allclose(FT[0, :3], 15 * fc) and np.allclose(FT[1, :3], 12 * fc)
    assert np.allclose(FT[0, 3:], np.cross(dd[:15], fc).sum(0), atol=1e-13)


def test_single_blob_height_marginal_is_1d_boltzmann():
    Lz, w = 16.0, 0.3
    edges = np.linspace(0.0, Lz, 17)
    ph, pa, se_h, _ = gb_marginals(np.zeros((1, 3)), np.array([1.0, 0.0, 0.0]), Lz, PHI0, D, B, w, edges,
                                   np.linspace(0, np.pi, 5), m=200, nz=8000, batches=2)
    dens = lambda z: math.exp(-(soft_profile(z, PHI0, D, B)[0] + soft_profile(Lz - z, PHI0, D, B)[0] + w * z))
    Z = integrate.quad(dens, 0.0, Lz, points=[D, Lz - D], limit=200)[0]
    ref = [integrate.quad(dens, a, b_, limit=200)[0] / Z for a, b_ in zip(edges[:-1], edges[1:])]
    assert np.allclose(ph, ref, atol=2e-6), np.max(np.abs(ph - np.array(ref)))
    assert np.all(se_h < 1e-12)                        # no orientation dependence: exact
    # the angle of any body vector is sin-distributed: bin mass (cos a - cos b)/2
    ea = np.linspace(0, np.pi, 5)
    exp_a = 0.5 * (np.cos(ea[:-1]) - np.cos(ea[1:]))
    assert np.allclose(pa, exp_a, atol=0.06)


def test_haar_angle_law():
    rng = np.random.default_rng(5)
    th = haar_quaternions(rng, 200000)
    ang = angle_with_z(th, np.array([0.3, -0.4, 0.5]))
    ea = np.linspace(0, np.pi, 13)
    h, _ = np.histogram(ang, ea)
    exp_a = 0.5 * (np.cos(ea[:-1]) - np.cos(ea[1:]))
    sig = np.sqrt(exp_a * (1 - exp_a) / th.shape[0])
    assert np.all(np.abs(h / th.shape[0] - exp_a) < 5 * sig)


def _boomerang_case():
    p = W.BOOMERANG_POTENTIAL
    return W.boomerang_shape(), float(W.BOOMERANG_N[2]), p["phi0"], p["d"], p["b"], p["weight"]


def test_slit_energy_outside_is_infinite():
    r_ref, Lz, phi0, d, b, w = _boomerang_case()
    assert np.isinf(slit_energy(np.array([[-0.1, 3.0]]), Lz, phi0, d, b, w)[0])
    assert np.isinf(slit_energy(np.array([[Lz, 3.0]]), Lz, phi0, d, b, w)[0])
    assert np.isfinite(slit_energy(np.array([[0.1, 3.0]]), Lz, phi0, d, b, w)[0])


@pytest.fixture(scope="module")
def boomerang_reference():
    r_ref, Lz, phi0, d, b, w = _boomerang_case()
    ze = np.linspace(0.0, Lz, 17)
    ae = np.linspace(0.0, np.pi, 13)
    ph, pa, se_h, se_a = gb_marginals(r_ref, W.BOOMERANG_P, Lz, phi0, d, b, w, ze, ae, m=8000, nz=800,
                                     batches=8)
    return ze, ae, ph, pa, se_h, se_a


def test_boomerang_marginals_shape(boomerang_reference):
    ze, ae, ph, pa, se_h, se_a = boomerang_reference
    assert abs(ph.sum() - 1.0) < 1e-12 and abs(pa.sum() - 1.0) < 1e-12
    # heights within about a blob radius of a wall are strongly suppressed
    assert ph[0] < 1e-3 and ph[-1] < 1e-3
    # gravity: more mass in the lower half
    assert ph[:8].sum() > ph[8:].sum()
    assert np.all(se_h < 0.02) and np.all(se_a < 0.02)


def test_exact_samples_match_quadrature(boomerang_reference):
    ze, ae, ph, pa, se_h, se_a = boomerang_reference
    r_ref, Lz, phi0, d, b, w = _boomerang_case()
    z, th = gb_samples(r_ref, Lz, phi0, d, b, w, 20000, seed=11)
    n = z.shape[0]
    hz, _ = np.histogram(z, ze)
    ha, _ = np.histogram(angle_with_z(th, W.BOOMERANG_P), ae)
    for hist, ref, se in ((hz / n, ph, se_h), (ha / n, pa, se_a)):
        sig = np.sqrt(ref * (1 - ref) / n + se ** 2) + 1e-4
        assert np.all(np.abs(hist - ref) < 5 * sig), (hist, ref)


def test_metropolis_matches_quadrature(boomerang_reference):
    ze, ae, ph, pa, se_h, se_a = boomerang_reference
    r_ref, Lz, phi0, d, b, w = _boomerang_case()
    zs, ths, acc = metropolis(r_ref, Lz, phi0, d, b, w, Lz / 2, np.array([1.0, 0, 0, 0]), 60000,
                              seed=2, sz=0.6, srot=0.35, thin=20)
    assert 0.2 < acc < 0.9
    zs, ths = zs[300:], ths[300:]                      # burn-in
    # batch means: 10 batches of consecutive samples give the Monte-Carlo error of the mean height
    mean_ref = float(np.sum(ph * 0.5 * (ze[:-1] + ze[1:])))
    bm = np.array([c.mean() for c in np.array_split(zs, 10)])
    err = bm.std(ddof=1) / math.sqrt(10)
    assert abs(zs.mean() - mean_ref) < 4 * err + 0.05, (zs.mean(), mean_ref, err)
    ang = angle_with_z(ths, W.BOOMERANG_P)
    ma = float(np.sum(pa * 0.5 * (ae[:-1] + ae[1:])))
    bm = np.array([c.mean() for c in np.array_split(ang, 10)])
    err = bm.std(ddof=1) / math.sqrt(10)
    assert abs(ang.mean() - ma) < 4 * err + 0.02, (ang.mean(), ma, err)
