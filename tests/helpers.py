"""Shared test plumbing: workloads -> library structs and oracle grids, and the
conversion between the oracle's compact unknowns and the library's padded
state vector.  Layout conversion only; no arithmetic of the method."""
from __future__ import annotations

import numpy as np

from oracle import mac


def oracle_grid(w) -> mac.Grid:
    return mac.Grid(w.n, w.bc, w.h, w.eta, w.wall_vel)


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
    opts = rb.rbfib_default_opts(**opt_kw)
    return rb.rbfib_create_batch(grids, [w.r_ref for w in ws], [w.offsets for w in ws], opts)


def dev(t):
    import torch
    return torch.as_tensor(np.ascontiguousarray(t), dtype=torch.float64).cuda()
