"""Plain FP64 CPU oracle for the RB-FIB mobility-solve hot path.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path (the HIP library and
its Python binding) may import, call or link anything in this package; only
the tests, the smoke check and the benchmark's CPU-baseline leg do.

Every discrete operator is assembled as an explicit SciPy sparse matrix in a
compact unknown layout (only true unknowns, wall faces excluded), so that
adjointness and structure are checked as exact matrix identities.  Solves
reach the exact discrete solution either by a dense/sparse direct solve
(tiny grids) or by an oracle-only right-preconditioned FGMRES to 1e-12 whose
result is always re-checked against the assembled operator.

Modules, with the part of the paper each follows (Sprinkle, Donev, Bhalla &
Patankar, "Brownian dynamics of fully confined suspensions of rigid particles
without Green's functions"):

  mac      staggered grid, D, G, tensor DT/GT, vector Laplacian   (Sec. III.A)
  ib       delta kernel, spreading S, interpolation J, walls      (Sec. III.B)
  bodies   quaternions, marker positions, K and K^T, tiles        (Sec. II, III.B)
  saddle   constrained system, RHS, direct and FGMRES solves      (Sec. III.C, Alg. 1)
  rng      Philox4x32-10 counter RNG and Box-Muller normals       (random inputs)
  sem      Split-Euler-Maruyama step with RFD drift               (Sec. IV, Alg. 1)
  adjoint  gradient of a loss of the rigid velocities             (differentiated solve)
"""
