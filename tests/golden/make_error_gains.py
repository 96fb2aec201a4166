"""Writes tests/golden/error_gains.json: for each named test configuration, the
oracle's gain from a solve residual to the error of each rigid-body velocity.

For the saddle system A x = b (eqs. D1-D4; A symmetric at h = 1, its only null
vector the constant pressure, to which every residual is orthogonal), a computed
x with residual r = b - A x has error A^+ r, so the error of velocity component k
obeys
    |U_k - U*_k| = |y_k . r| <= ||y_k||_2 ||r||_2 ,   y_k = A^+ e_{U,k}
(Cauchy-Schwarz).  y_k is the solution of the mobility problem with a unit force
or torque on coordinate k and mean-free pressure, so gain_k = ||y_k||_2 needs one
exact oracle solve per body coordinate.  Only the oracle is called.

Run from the repository root:  python tests/golden/make_error_gains.py [names...]
"""
import json
import os
import sys
import time
from concurrent.futures import ProcessPoolExecutor

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

OUT = os.path.join(ROOT, "tests", "golden", "error_gains.json")


def _gain(args):
    name, k = args
    from oracle import mac
    from oracle.saddle import Saddle
    from tests.parity_configs import gain_configs
    w = gain_configs()[name]
    g = mac.Grid(w.n, w.bc, w.h, w.eta, w.wall_vel, kernel=w.kernel)
    assert g.h == 1.0, "the gains use A^T = A, which holds at h = 1"
    s = Saddle(g, w.q, w.theta, w.r_ref, w.offsets)
    e = np.zeros(6 * w.nb)
    e[k] = 1.0
    y = s.solve(s.rhs(FT=e.reshape(w.nb, 6), include_bc=False), tol=1e-12)
    res = s.residual(y, s.rhs(FT=e.reshape(w.nb, 6), include_bc=False))
    return name, k, float(np.linalg.norm(y)), res


def _init_worker():
    from threadpoolctl import threadpool_limits
    threadpool_limits(limits=1)


def main(names=None):
    from tests.parity_configs import gain_configs
    cfg = gain_configs()
    names = names or list(cfg)
    try:
        with open(OUT) as fh:
            data = json.load(fh)
    except OSError:
        data = {}
    jobs = [(n, k) for n in names for k in range(6 * cfg[n].nb)]
    t0 = time.time()
    out = {n: [None] * (6 * cfg[n].nb) for n in names}
    worst = {n: 0.0 for n in names}
    with ProcessPoolExecutor(max_workers=min(8, os.cpu_count() or 1), initializer=_init_worker) as ex:
        for n, k, gk, res in ex.map(_gain, jobs, chunksize=1):
            out[n][k] = gk
            worst[n] = max(worst[n], res)
    for n in names:
        w = cfg[n]
        data[n] = {"workload": w.name, "grid": list(w.n), "bodies": w.nb, "markers": w.nm,
                   "gain": [round(v, 12) for v in out[n]],
                   "max_oracle_residual": worst[n]}
        print("%-28s nb=%4d max gain %.4f (%.0f s)" % (n, w.nb, max(out[n]), time.time() - t0), flush=True)
    with open(OUT, "w") as fh:
        json.dump(data, fh, indent=1, sort_keys=True)
        fh.write("\n")


if __name__ == "__main__":
    main(sys.argv[1:] or None)
