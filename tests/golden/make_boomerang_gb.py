"""Writes tests/golden/boomerang_gb.json: the Gibbs-Boltzmann marginals of the
App. A boomerang in its 64x64x16 slit (cross-point height and the angle of
p-hat with the z axis), from the oracle's quadrature route (oracle/gibbs.py):
independent seeded batches of Haar orientations, each with the height
integral on a fine trapezoid grid, spread over worker processes.  Only the
oracle is called.

Run from the repository root:  python tests/golden/make_boomerang_gb.py
"""
import json
import os
import sys
import time
from concurrent.futures import ProcessPoolExecutor

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

OUT = os.path.join(ROOT, "tests", "golden", "boomerang_gb.json")
WORKERS, PER_WORKER, BATCHES, NZ = 8, 50000, 5, 3200
Z_EDGES = np.linspace(0.0, 16.0, 33)          # 0.5 h bins across the slit
A_EDGES = np.linspace(0.0, np.pi, 19)         # 10 degree bins


def _part(i):
    import workloads as W
    from oracle.gibbs import gb_marginals
    p = W.BOOMERANG_POTENTIAL
    return gb_marginals(W.boomerang_shape(), W.BOOMERANG_P, float(W.BOOMERANG_N[2]), p["phi0"], p["d"], p["b"],
                        p["weight"], Z_EDGES, A_EDGES, m=PER_WORKER, seed=1000 + i, nz=NZ, batches=BATCHES)


def _init_worker():
    from threadpoolctl import threadpool_limits
    threadpool_limits(limits=1)


def main():
    import workloads as W
    t0 = time.time()
    with ProcessPoolExecutor(max_workers=WORKERS, initializer=_init_worker) as ex:
        parts = list(ex.map(_part, range(WORKERS)))
    ph = np.mean([p[0] for p in parts], axis=0)
    pa = np.mean([p[1] for p in parts], axis=0)
    se_h = np.sqrt(np.sum([p[2] ** 2 for p in parts], axis=0)) / WORKERS
    se_a = np.sqrt(np.sum([p[3] ** 2 for p in parts], axis=0)) / WORKERS
    zc = 0.5 * (Z_EDGES[1:] + Z_EDGES[:-1])
    data = {
        "what": "Gibbs-Boltzmann marginals of the App. A boomerang (oracle quadrature)",
        "potential": W.BOOMERANG_POTENTIAL, "spacing": W.BOOMERANG_S, "slit": list(W.BOOMERANG_N),
        "p_body": W.BOOMERANG_P.tolist(), "orientations": WORKERS * PER_WORKER, "height_nodes": NZ + 1,
        "z_edges": Z_EDGES.tolist(), "angle_edges": A_EDGES.tolist(),
        "p_height": [round(v, 12) for v in ph], "p_angle": [round(v, 12) for v in pa],
        "se_height": [float("%.3e" % v) for v in se_h], "se_angle": [float("%.3e" % v) for v in se_a],
        "mean_height_bin_centres": float(np.sum(ph * zc)),
    }
    with open(OUT, "w") as fh:
        json.dump(data, fh, indent=1)
        fh.write("\n")
    print("wrote %s in %.0f s; max se %.2e / %.2e" % (OUT, time.time() - t0, se_h.max(), se_a.max()))


if __name__ == "__main__":
    main()
