"""Shared test plumbing: workloads -> library structs and oracle grids, and the
conversion between the oracle's compact unknowns and the library's padded
state vector.  Layout conversion only; no arithmetic of the method."""
from __future__ import annotations

import numpy as np

from oracle import mac


def oracle_grid(w) -> mac.Grid:
    return mac.Grid(w.n, w.bc, w.h, w.eta, w.wall_vel, kernel=getattr(w, "kernel", 4))


def pack_state(g: mac.Grid, v, p, lam, U) -> np.ndarray:
    """Oracle pieces (compact velocity, pressure, lambda, U) -> padded state vector."""
    vp = g.compact_to_padded(v).reshape(-1)
    return np.concatenate([vp, np.asarray(p).ravel(), np.asarray(lam).ravel(), np.asarray(U).ravel()])


def unpack_state(g: mac.Grid, x: np.ndarray, nm: int, nb: int):
    N = g.ncell
    v = g.padded_to_compact(x[:3 * N])
    p = x[3 * N:4 * N]
    lam = x[4 * N:4 * N + 3 * nm].reshape(-1, 3)
    U = x[4 * N + 3 * nm:4 * N + 3 * nm + 6 * nb].reshape(-1, 6)
    return v, p, lam, U


def oracle_to_padded(s, x_oracle: np.ndarray) -> np.ndarray:
    v, p, lam, U = s.split(x_oracle)
    return pack_state(s.g, v, p, lam, U)


def padded_to_oracle(s, x_pad: np.ndarray) -> np.ndarray:
    v, p, lam, U = unpack_state(s.g, x_pad, s.nm, s.nb)
    return np.concatenate([v, p, lam.ravel(), U.ravel()])


def lib_context(rb, ws, **opt_kw):
    """Build a library context for one workload or a list of them."""
    if not isinstance(ws, (list, tuple)):
        ws = [ws]
    grids = [rb.make_grid(w.n, w.bc, w.h, w.eta, w.wall_vel) for w in ws]
    opt_kw.setdefault("kernel", getattr(ws[0], "kernel", 4))
    if opt_kw["kernel"] == 6:
        opt_kw.setdefault("blob_radius", 1.4)     # the 6-point blob is larger (1.47 h)
    opts = rb.rbfib_default_opts(**opt_kw)
    return rb.rbfib_create_batch(grids, [w.r_ref for w in ws], [w.offsets for w in ws], opts)


def dev(t):
    import torch
    return torch.as_tensor(np.ascontiguousarray(t), dtype=torch.float64).cuda()


# ------------------------------------------------------------------ error bounds
_GAINS = None


def error_gains(name: str) -> np.ndarray:
    """gain_k = ||A^+ e_{U,k}||_2 for configuration `name`, written by the oracle
    (tests/golden/make_error_gains.py): a solve whose residual has 2-norm rho has
    |U_k - U*_k| <= gain_k rho."""
    global _GAINS
    if _GAINS is None:
        import json
        import os
        with open(os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "error_gains.json")) as fh:
            _GAINS = json.load(fh)
    return np.asarray(_GAINS[name]["gain"], dtype=np.float64)


# Largest gain from the residuals of the two solves that feed the drift of a SEM step
# (the random-finite-difference solve and the unconstrained Stokes solve) to the
# final velocities, relative to the gain of the final solve's own residual: their
# errors reach U through differences of K, K^T, J and S over Q+- divided by delta,
# which are O(1) multiples of the solution error (at most the largest marker offset
# times |W|, a few units), and for the unconstrained solve through the inverse
# Laplacian (up to ~L^2 / (3 pi^2) h^2 for an L-cell box, ~35 at L = 32).
SEM_DRIFT_GAIN = 100.0


def sem_error_bound(name: str, norms, tol: float, final_rel_residual: float) -> np.ndarray:
    """Per-component bound on |U_gpu - U_oracle| for one SEM step: the final solve's
    residual (final_rel_residual ||b_3||) times its gain, plus the drift solves'
    residuals (at most tol ||b_1||, tol ||b_2||) times SEM_DRIFT_GAIN times it."""
    b1, b2, b3 = norms
    rho = final_rel_residual * b3 + SEM_DRIFT_GAIN * tol * (b1 + b2)
    return error_gains(name).reshape(-1, 6) * rho
