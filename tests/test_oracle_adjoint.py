"""Pins of the oracle's gradient of L = sum |U_p|^2 through the mobility solve.

* Central finite differences (eps 1e-5, solves at 1e-12) along 8 seeded random
  directions in (forces/torques, positions, rotations) agree with the
  adjoint formula, with the 4-point and with the 6-point kernel (whose
  derivative enters through the kernel gradient in J).
* dL/dF = 2 N U with N assembled column by column (N symmetric).
"""
import numpy as np
import pytest

import workloads as W
from oracle import adjoint, mac
from oracle.saddle import Saddle


@pytest.mark.parametrize("kernel", [4, 6])
def test_gradient_vs_finite_differences(kernel):
    w = W.small_box(4, n=(10, 10, 12), n_bodies=2, R=1.5, shape="ico12")
    g = mac.Grid(w.n, w.bc, w.h, w.eta, kernel=kernel)
    s, x = adjoint.solve_U(g, w.r_ref, w.offsets, w.q, w.theta, w.FT)
    U = s.split(x)[3]
    dF, dq, dphi = adjoint.mobility_vjp(g, w.r_ref, w.offsets, w.q, w.theta, w.FT, 2 * U)
    rng = np.random.default_rng(1901)
    pairs = []
    for _ in range(8):
        a = rng.standard_normal((2, 6))
        b = rng.standard_normal((2, 3))
        c = rng.standard_normal((2, 3))
        fd = adjoint.finite_difference(g, w.r_ref, w.offsets, w.q, w.theta, w.FT, a, b, c)
        an = np.sum(dF * a) + np.sum(dq * b) + np.sum(dphi * c)
        pairs.append((fd, an))
    # the solves' 1e-12 tolerance leaves ~1e-12 |L| / eps of noise in a difference
    # quotient; it is measured against the typical directional derivative
    scale = np.mean([abs(an) for _, an in pairs])
    for fd, an in pairs:
        assert abs(fd - an) <= 1e-6 * max(abs(fd), scale)


def test_force_gradient_is_2NU():
    w = W.small_box(7, n=(8, 8, 10), n_bodies=1, R=1.5, shape="ico12")
    g = mac.Grid(w.n, w.bc, w.h, w.eta)
    s = Saddle(g, w.q, w.theta, w.r_ref, w.offsets)
    N = np.zeros((6, 6))
    for k in range(6):
        e = np.zeros(6)
        e[k] = 1.0
        N[:, k] = s.split(s.solve(s.rhs(FT=e, include_bc=False)))[3].ravel()
    U = N @ w.FT.ravel()
    dF, _, _ = adjoint.mobility_vjp(g, w.r_ref, w.offsets, w.q, w.theta, w.FT, 2 * U.reshape(1, 6))
    assert np.abs(dF.ravel() - 2 * N @ U).max() < 1e-9 * np.abs(2 * N @ U).max()
