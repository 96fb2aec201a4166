"""Launch-geometry autotuner of librbfib: an offline sweep on the target GPU.

For each workload class it times batched Split-Euler-Maruyama launches (the
library's real hot path: three solves per replica with the FP32 multigrid
preconditioner) under candidate launch geometries and keeps the fastest:

  krylov_chunk  Krylov vector elements per workgroup of the projection and update
                passes (512, 1024, 2048)
  spread_p      (tile, marker) pairs staged per LDS round of spreading (16, 32, 64)
  spread_grid   workgroups of the spreading grid-stride loop
  mg_npt        grid points per thread of the multigrid and cell kernels (1, 4)
  apply_kc      z planes per workgroup of the z-marching fluid apply (0: the
                two-cells-per-thread apply; 4, 8, 16)

by coordinate descent in that order (each candidate timed twice, the faster
kept), and writes the table that context creation reads (tuning.txt beside the
library, or the file named by RBFIB_TUNING): one line per class,

    cells_lo cells_hi reps_lo reps_hi krylov_chunk spread_grid spread_p mg_npt apply_kc

followed by a comment with the measured seconds per launch of the defaults and
of the choice.  Run from the repository root on the GPU it is for:

    python paper_1901_06427_amd/autotune.py [--out FILE] [--classes a,b,...]
"""
import argparse
import os
import sys
import tempfile
import time

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

BIG = 9223372036854775807

# workload classes: how to build a representative batch, how many launches to time,
# and the (inclusive) ranges of total cells and replicas the table line covers
CLASSES = {
    "ensemble": dict(build="ensemble", launches=3, cells=(4000000, BIG), reps=(16, 1000000)),
    "large_single": dict(build="monolayer", launches=2, cells=(500000, BIG), reps=(1, 15)),
    "small_single": dict(build="two_spheres", launches=12, cells=(0, 499999), reps=(1, 15)),
}

SPACE = [("krylov_chunk", (512, 1024, 2048)), ("spread_p", (16, 32, 64)),
         ("spread_grid", (1024, 4096, 16384, 65536)), ("mg_npt", (1, 4)), ("apply_kc", (0, 4, 8, 16))]
DEFAULT = {"krylov_chunk": 1024, "spread_grid": 65536, "spread_p": 32, "mg_npt": 0, "apply_kc": 0}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def _workloads(kind):
    import workloads as W
    if kind == "ensemble":
        return W.ensemble()
    if kind == "monolayer":
        return [W.monolayer()]
    return [W.two_spheres()]


def _line(cfg, cells=(0, BIG), reps=(1, 1000000)):
    return "%d %d %d %d %d %d %d %d %d" % (cells[0], cells[1], reps[0], reps[1], cfg["krylov_chunk"],
                                           cfg["spread_grid"], cfg["spread_p"], cfg["mg_npt"], cfg["apply_kc"])


def time_geometry(ws, cfg, launches, table_dir):
    """Seconds per batched SEM launch of workloads ws under launch geometry cfg."""
    import numpy as np
    import torch
    import paper_1901_06427_amd as rb
    path = os.path.join(table_dir, "candidate.txt")
    with open(path, "w") as fh:
        fh.write(_line(cfg) + "\n")
    os.environ["RBFIB_TUNING"] = path
    grids = [rb.make_grid(w.n, w.bc, w.h, w.eta, w.wall_vel) for w in ws]
    ctx = rb.rbfib_create_batch(grids, [w.r_ref for w in ws], [w.offsets for w in ws],
                                rb.rbfib_default_opts(tol=1e-6, precond_fp32=1))
    got = rb.rbfib_launch_geometry(ctx)
    assert all(got[k] == cfg[k] for k in ("krylov_chunk", "spread_grid", "spread_p", "apply_kc")), (got, cfg)
    cat = lambda key: torch.as_tensor(np.concatenate([getattr(w, key) for w in ws]), dtype=torch.float64).cuda()
    q0, th0, FT = cat("q"), cat("theta"), cat("FT")
    U = torch.empty((sum(w.nb for w in ws), 6), dtype=torch.float64, device="cuda")
    best = float("inf")
    for rep in range(2):
        q, th = q0.clone(), th0.clone()
        rb.rbfib_sem_step(ctx, q, th, FT, 1.0, 0.01, 77, 0, U)          # warm-up (graph capture)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for k in range(launches):
            rb.rbfib_sem_step(ctx, q, th, FT, 1.0, 0.01, 77, 1 + k, U)
        torch.cuda.synchronize()
        best = min(best, (time.perf_counter() - t0) / launches)
    ctx.close()
    return best


def tune_class(name, spec, table_dir):
    ws = _workloads(spec["build"])
    cur = dict(DEFAULT)
    base = time_geometry(ws, cur, spec["launches"], table_dir)
    log("%s: defaults %.4f s per launch" % (name, base))
    best_t = base
    for key, values in SPACE:
        for v in values:
            if v == cur[key]:
                continue
            cand = dict(cur)
            cand[key] = v
            t = time_geometry(ws, cand, spec["launches"], table_dir)
            log("  %s %s=%d: %.4f s" % (name, key, v, t))
            if t < best_t:
                best_t, cur = t, cand
    log("%s: chose %s, %.4f s per launch (defaults %.4f)" % (name, cur, best_t, base))
    return cur, base, best_t


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--out", default=os.path.join(HERE, "tuning.txt"))
    ap.add_argument("--classes", default=",".join(CLASSES))
    args = ap.parse_args()
    lines = ["# launch geometry of librbfib, written by paper_1901_06427_amd/autotune.py on the GPU it ran on",
             "# cells_lo cells_hi reps_lo reps_hi krylov_chunk spread_grid spread_p mg_npt apply_kc"]
    with tempfile.TemporaryDirectory() as tmp:
        for name in args.classes.split(","):
            spec = CLASSES[name]
            cfg, base, best = tune_class(name, spec, tmp)
            lines.append("%s  # %s: %.4f s per SEM launch (defaults %.4f s)" % (
                _line(cfg, spec["cells"], spec["reps"]), name, best, base))
    os.environ.pop("RBFIB_TUNING", None)
    with open(args.out, "w") as fh:
        fh.write("\n".join(lines) + "\n")
    print("\n".join(lines), flush=True)


if __name__ == "__main__":
    main()
