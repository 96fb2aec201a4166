"""Pins of the oracle's staggered-grid operators (paper Sec. III.A).

Checked against what the mathematics fixes, not against the oracle itself:
adjoint relations G = -D^T and Lm = DT GT (the ghost-cell Laplacian built
independently), closed-form sine/cosine eigenpairs, and a manufactured
divergence-free Stokes solution recovered by a solve; no-slip (1), free-slip
(2) and periodic (0) axes in combination.  Closed-form flows: plane Poiseuille
between no-slip walls, plane Couette between sliding walls, and a shear-free
cosine mode between free-slip walls.
"""
import math

import numpy as np
import pytest

from oracle import mac, saddle

BCS = [(1, 1, 1), (0, 1, 1), (1, 0, 1), (0, 0, 1), (1, 0, 0), (2, 2, 2), (1, 2, 0), (0, 2, 1), (2, 1, 2)]


@pytest.mark.parametrize("bc", BCS)
def test_adjoint_relations(bc):
    g = mac.Grid((5, 6, 4), bc, h=0.7)
    D, G = mac.divergence(g), mac.gradient(g)
    GT, DT = mac.vector_gradient(g), mac.tensor_divergence(g)
    assert abs(G + D.T).max() == 0.0
    assert abs(DT + GT.T).max() == 0.0
    Lm = mac.vector_laplacian(g)
    # ghost-cell stencil == DT GT (discrete fluctuation-dissipation balance)
    assert abs(Lm - DT @ GT).max() < 1e-12
    assert abs(Lm - Lm.T).max() < 1e-12
    # D and G entries are exactly +-1/h
    assert np.allclose(np.abs(D.data), 1.0 / g.h)


def _mode_1d(N, kind, k, h):
    if kind == "face_wall":      # faces 1..N-1 (compact), Dirichlet at 0, N
        f = np.arange(1, N)
        return np.sin(np.pi * k * f / N), -(4 / h**2) * math.sin(math.pi * k / (2 * N)) ** 2
    if kind == "cell_wall":      # cells, odd ghosts
        j = np.arange(N)
        return np.sin(np.pi * k * (j + 0.5) / N), -(4 / h**2) * math.sin(math.pi * k / (2 * N)) ** 2
    if kind == "cell_neumann":
        j = np.arange(N)
        return np.cos(np.pi * k * (j + 0.5) / N), -(4 / h**2) * math.sin(math.pi * k / (2 * N)) ** 2
    j = np.arange(N)             # periodic
    return np.cos(2 * np.pi * k * j / N), -(4 / h**2) * math.sin(math.pi * k / N) ** 2


@pytest.mark.parametrize("bc", BCS)
def test_vector_laplacian_eigenpairs(bc):
    g = mac.Grid((6, 5, 7), bc, h=1.3)
    Lm = mac.vector_laplacian(g)
    rng = np.random.default_rng(3)
    for c in range(3):
        for _ in range(3):
            vec = np.ones(1)
            lam = 0.0
            for a in (2, 1, 0):      # build [k][j][i] -> x fastest via kron
                N = g.n[a]
                if g.bc[a] == mac.PERIODIC:
                    kind, k = "periodic", int(rng.integers(0, N))
                elif a == c:
                    kind, k = "face_wall", int(rng.integers(1, N))
                elif g.bc[a] == mac.SLIP:       # even ghosts: cosine modes
                    kind, k = "cell_neumann", int(rng.integers(0, N))
                else:
                    kind, k = "cell_wall", int(rng.integers(1, N + 1))
                m, l = _mode_1d(N, kind, k, g.h)
                vec = np.kron(vec, m)
                lam += l
            full = np.zeros(g.nv)
            full[g.face_offset[c]:g.face_offset[c] + g.nface[c]] = vec
            out = Lm @ full
            assert np.abs(out - lam * full).max() < 1e-12 * max(1.0, abs(lam))


@pytest.mark.parametrize("bc", BCS)
def test_scalar_laplacian_eigenpairs(bc):
    g = mac.Grid((6, 5, 4), bc)
    L = mac.scalar_laplacian(g)
    rng = np.random.default_rng(5)
    for _ in range(4):
        vec = np.ones(1)
        lam = 0.0
        for a in (2, 1, 0):
            N = g.n[a]
            kind = "periodic" if g.bc[a] == mac.PERIODIC else "cell_neumann"
            m, l = _mode_1d(N, kind, int(rng.integers(0, N)), g.h)
            vec = np.kron(vec, m)
            lam += l
        assert np.abs(L @ vec - lam * vec).max() < 1e-12


def _curl_field(g, rng):
    """Divergence-free padded velocity: discrete curl of a random edge potential
    that vanishes on wall node planes (so the normal velocity on walls is 0)."""
    nx, ny, nz = g.n
    nodes = [g.nodes(a) for a in range(3)]

    def pot(dims, wall_axes):
        p = rng.standard_normal(dims[::-1])
        for a in wall_axes:
            if g.bc[a] != mac.PERIODIC:
                sl = [slice(None)] * 3
                sl[2 - a] = 0
                p[tuple(sl)] = 0.0
                sl[2 - a] = dims[a] - 1
                p[tuple(sl)] = 0.0
        return p

    # psi_z on z-edges (node x, node y, cell z), psi_y on y-edges, psi_x on x-edges
    pz = pot((nodes[0], nodes[1], nz), (0, 1))
    py = pot((nodes[0], ny, nodes[2]), (0, 2))
    px = pot((nx, nodes[1], nodes[2]), (1, 2))

    def dnode(p, axis, N):
        """difference p[n+1] - p[n] along an edge-node axis -> N values (wraps if periodic)."""
        ax = 2 - axis
        if p.shape[ax] == N:       # periodic: N nodes
            return np.roll(p, -1, axis=ax) - p
        return np.diff(p, axis=ax)

    ux = np.zeros((nz, ny, nx)); uy = np.zeros((nz, ny, nx)); uz = np.zeros((nz, ny, nx))
    # u_x = d psi_z / dy - d psi_y / dz  at (face x, cell y, cell z)
    ux += dnode(pz, 1, ny)[:, :, :nx] - dnode(py, 2, nz)[:, :, :nx]
    uy += dnode(px, 2, nz)[:, :ny, :] - dnode(pz, 0, nx)[:, :ny, :]
    uz += dnode(py, 0, nx)[:nz, :, :] - dnode(px, 1, ny)[:nz, :, :]
    return np.stack([ux, uy, uz]).reshape(3, -1) / g.h


@pytest.mark.parametrize("bc", [(1, 1, 1), (0, 1, 1), (0, 0, 1), (2, 1, 2), (0, 2, 1)])
def test_manufactured_stokes(bc):
    g = mac.Grid((8, 6, 10), bc, h=1.0, eta=1.7)
    rng = np.random.default_rng(7)
    vpad = _curl_field(g, rng)
    v = g.padded_to_compact(vpad)
    # the potential vanishes on wall planes, so the dropped wall slots carry nothing
    assert np.allclose(g.compact_to_padded(v), vpad)
    D = mac.divergence(g)
    assert np.abs(D @ v).max() < 1e-12
    pi = rng.standard_normal(g.ncell)
    pi -= pi.mean()
    f = -g.eta * (mac.vector_laplacian(g) @ v) + mac.gradient(g) @ pi
    s = saddle.Saddle(g, np.zeros((0, 3)), np.zeros((0, 4)), np.zeros((0, 3)), np.zeros(1, dtype=int),
                      fluid_only=True)
    b = s.rhs(fluid=f, include_bc=False)
    x = s.solve_direct(b)
    assert np.abs(x[s.sl_v] - v).max() < 1e-9
    p = x[s.sl_p] - x[s.sl_p].mean()
    assert np.abs(p - pi).max() < 1e-9
    xf, info = s.solve_fgmres(b, tol=1e-12)
    assert info["rel_residual"] < 1e-12
    assert np.abs(xf[s.sl_v] - v).max() < 1e-9


@pytest.mark.parametrize("nz", [8, 16])
def test_plane_poiseuille_closed_form(nz):
    """Uniform force F along x between no-slip walls at z = 0 and z = L, periodic x, y.

    Every interior row of the discrete momentum equation holds for the parabola
    F z (L - z) / (2 eta) (the second difference of a quadratic is exact); at the first
    and last cell the odd reflection about the wall places the ghost at -u_0, which
    misses the parabola's value by F h^2 / (4 eta), and the error that this drives is
    the constant F h^2 / (8 eta).  So the discrete solution is the parabola plus that
    constant at every x face, with no flow across and a uniform pressure: second-order
    accuracy of the wall treatment, with its exact error constant."""
    h, eta, F = 0.5, 1.3, 0.7
    g = mac.Grid((4, 3, nz), (0, 0, 1), h=h, eta=eta)
    f = np.zeros((3, nz, 3, 4))
    f[0] = F
    s = saddle.Saddle(g, np.zeros((0, 3)), np.zeros((0, 4)), np.zeros((0, 3)), np.zeros(1, dtype=int),
                      fluid_only=True)
    x = s.solve_direct(s.rhs(fluid=g.padded_to_compact(f), include_bc=False))
    v = g.compact_to_padded(x[s.sl_v]).reshape(3, nz, 3, 4)
    L = nz * h
    z = (np.arange(nz) + 0.5) * h
    expect = F * z * (L - z) / (2 * eta) + F * h * h / (8 * eta)
    assert np.abs(v[0] - expect[:, None, None]).max() < 1e-10 * expect.max()
    assert np.abs(v[1:]).max() < 1e-12
    p = x[s.sl_p]
    assert np.abs(p - p.mean()).max() < 1e-10


def test_noise_index_space_counts():
    g = mac.Grid((4, 5, 6), (0, 1, 1))
    dims = [g.family_dims(f) for f in range(9)]
    assert dims[0] == (4, 5, 6)                 # xx on cells
    assert dims[3] == (4, 6, 6)                 # xy: nodes along y (wall: N+1)
    assert dims[5] == (4, 5, 6)                 # yx: nodes along x (periodic: N)
    assert g.nW == sum(int(np.prod(d)) for d in dims)


def test_moving_wall_rhs():
    wv = np.zeros((3, 2, 3))
    wv[2, 0, 0] = 0.5                           # bottom z wall slides along +x
    g = mac.Grid((4, 4, 5), (0, 1, 1), eta=2.0, wall_vel=wv)
    r = mac.moving_wall_rhs(g)
    ux = g.compact_to_padded(r)[0].reshape(5, 4, 4)
    assert np.allclose(ux[0], 2 * 2.0 * 0.5)
    assert np.allclose(ux[1:], 0.0)
    assert np.allclose(g.compact_to_padded(r)[1:], 0.0)


@pytest.mark.parametrize("wall_axis,comp", [(2, 0), (1, 2), (0, 1)])
def test_plane_couette_closed_form(wall_axis, comp):
    """Plane Couette flow: walls normal to `wall_axis` sliding with tangential
    velocities U_lo and U_hi along `comp`, the other two axes periodic, no body.  With
    the tangential ghost u_g = 2 U_w - u (Sec. III.A; the sliding wall of the monolayer,
    Sec. VI) the linear profile U_lo + (U_hi - U_lo) x / L at the face centres is the
    exact discrete solution: its second differences vanish inside, and its value at the
    mirror point of the first cell is exactly 2 U_w minus its value in that cell.  So
    the affine right-hand side from the sliding walls must reproduce it to round-off,
    with no cross flow and a uniform pressure; and interpolation with the sliding-wall
    term J_bc (Sec. III.B) returns the same line at every marker, wall neighbours
    included, because the 4-point kernel reproduces linear functions."""
    from oracle import ib
    n = [4, 4, 4]
    n[wall_axis] = 12
    bc = [mac.PERIODIC] * 3
    bc[wall_axis] = mac.WALL
    h, eta = 0.5, 1.7
    Ulo, Uhi = 0.8, -0.3
    wv = np.zeros((3, 2, 3))
    wv[wall_axis, 0, comp] = Ulo
    wv[wall_axis, 1, comp] = Uhi
    g = mac.Grid(tuple(n), tuple(bc), h=h, eta=eta, wall_vel=wv)
    s = saddle.Saddle(g, np.zeros((0, 3)), np.zeros((0, 4)), np.zeros((0, 3)), np.zeros(1, dtype=int),
                      fluid_only=True)
    x = s.solve_direct(s.rhs(include_bc=True))
    v = g.compact_to_padded(x[s.sl_v]).reshape(3, n[2], n[1], n[0])
    L = n[wall_axis] * h
    coord = (np.arange(n[wall_axis]) + 0.5) * h
    line = Ulo + (Uhi - Ulo) * coord / L
    shape = [1, 1, 1]
    shape[2 - wall_axis] = n[wall_axis]
    assert np.abs(v[comp] - line.reshape(shape)).max() < 1e-12
    for c in range(3):
        if c != comp:
            assert np.abs(v[c]).max() < 1e-12
    p = x[s.sl_p]
    assert np.abs(p - p.mean()).max() < 1e-11
    # interpolation with the affine wall term reproduces the line at markers anywhere
    rng = np.random.default_rng(4)
    r = rng.uniform(0.02, 0.98, size=(40, 3)) * np.array(n) * h
    r[:5, wall_axis] = rng.uniform(0.01, 0.3, 5) * h          # next to the lower wall
    r[5:10, wall_axis] = L - rng.uniform(0.01, 0.3, 5) * h    # next to the upper wall
    Jv = (ib.interpolation(g, r) @ x[s.sl_v]).reshape(-1, 3) + ib.interpolation_bc(g, r)
    expect = Ulo + (Uhi - Ulo) * r[:, wall_axis] / L
    assert np.abs(Jv[:, comp] - expect).max() < 1e-12
    assert np.abs(np.delete(Jv, comp, axis=1)).max() < 1e-12


@pytest.mark.parametrize("k", [0, 1, 3])
def test_free_slip_channel_closed_form(k):
    """Free-slip walls at z = 0 and z = L (zero tangential stress: even ghosts), x and
    y periodic, body force f_x = F cos(pi k z / L) at the x faces.  The discrete
    solution is the same cosine, divided by eta times its eigenvalue
    (4/h^2) sin^2(pi k / (2 N)) -- a no-slip wall (odd ghosts) would have sine modes
    instead.  k = 0 (uniform forcing) has no steady state between free-slip walls;
    there the singular mode is checked to be in the operator's kernel."""
    h, eta, F, nz = 0.5, 1.3, 0.7, 12
    g = mac.Grid((4, 3, nz), (mac.PERIODIC, mac.PERIODIC, mac.SLIP), h=h, eta=eta)
    Lm = mac.vector_laplacian(g)
    z = (np.arange(nz) + 0.5) * h
    L = nz * h
    prof = np.cos(math.pi * k * z / L)
    f = np.zeros((3, nz, 3, 4))
    f[0] = F * prof[:, None, None]
    fc = g.padded_to_compact(f)
    lam = (4.0 / h ** 2) * math.sin(math.pi * k / (2 * nz)) ** 2
    if k == 0:
        assert np.abs(Lm @ fc).max() < 1e-12           # uniform shear-free flow is a null mode
        return
    s = saddle.Saddle(g, np.zeros((0, 3)), np.zeros((0, 4)), np.zeros((0, 3)), np.zeros(1, dtype=int),
                      fluid_only=True)
    x, info = s.solve_fgmres(s.rhs(fluid=fc, include_bc=False), tol=1e-13)
    v = g.compact_to_padded(x[s.sl_v]).reshape(3, nz, 3, 4)
    expect = F * prof / (eta * lam)
    assert np.abs(v[0] - expect[:, None, None]).max() < 1e-10 * np.abs(expect).max()
    assert np.abs(v[1:]).max() < 1e-12
    # the no-slip rule would not reproduce it
    gw = mac.Grid((4, 3, nz), (mac.PERIODIC, mac.PERIODIC, mac.WALL), h=h, eta=eta)
    assert np.abs(mac.vector_laplacian(gw) @ g.padded_to_compact(f) + lam * fc).max() > 1e-3 * lam * F
