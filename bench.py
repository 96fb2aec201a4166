"""Benchmark of the RB-FIB mobility-solve hot path on one MI355X.

Workload (default): two 42-marker spheres of radius 2.5 h tightly confined in a
32 x 32 x 64 walled box, kT = 1, dt = 0.01, soft steric repulsion between the
spheres and with the walls, fluctuating stress on cells and edges, and one
Split-Euler-Maruyama step per benchmark step (Algorithm 1: two constrained
mobility solves and one unconstrained Stokes solve, each to a relative
residual of 1e-6).  Inputs are seeded and synthetic, and resident in GPU
memory before the timed region.

The JSON line reports constrained mobility solves per second with the FP32
multigrid preconditioner (the headline), the same workload with the FP64
preconditioner ("plain_fp64"), a roofline object for the dominant kernel
(timed with HIP events inside the library on its own stream), and the FP64
CPU oracle timed on a bounded sample of the same workload.
"""
import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

METRIC = "RB-FIB mobility solves/s at 1e-6 residual, batched+FP32-PC vs plain; HBM GB/s"
HBM_PEAK_GBS = 8000.0


def log(*a):
    print(*a, file=sys.stderr, flush=True)


# ----------------------------------------------------------------- workload forces
def soft_forces_torch(q, radius, n, h, kT):
    """Soft steric repulsion Phi(r) = Phi0 (1 + (d - r)/b) for r < d and
    Phi0 exp((d - r)/b) for r >= d, Phi0 = 4 kT, b = 0.1 R; pairs use d = 2R on
    centre distances, walls use d = R on the distance from a centre to each
    wall.  Caller-side forces (not part of the mobility solve)."""
    import torch
    phi0 = 4.0 * kT
    b = 0.1 * radius
    nb = q.shape[0]
    F = torch.zeros((nb, 6), dtype=q.dtype, device=q.device)

    def mag(r, d):
        return torch.where(r < d, torch.full_like(r, phi0) / b, (phi0 / b) * torch.exp((d - r) / b))

    if nb > 1:
        dq = q[:, None, :] - q[None, :, :]
        r = torch.linalg.norm(dq, dim=2) + torch.eye(nb, dtype=q.dtype, device=q.device) * 1e9
        f = mag(r, 2 * radius)[:, :, None] * dq / r[:, :, None]
        F[:, :3] += f.sum(dim=1)
    L = torch.tensor([n[0] * h, n[1] * h, n[2] * h], dtype=q.dtype, device=q.device)
    lo = q
    hi = L[None, :] - q
    F[:, :3] += mag(lo, radius) - mag(hi, radius)
    return F


def soft_forces_np(q, radius, n, h, kT):
    phi0 = 4.0 * kT
    b = 0.1 * radius

    def mag(r, d):
        return np.where(r < d, phi0 / b, (phi0 / b) * np.exp((d - r) / b))

    nb = q.shape[0]
    F = np.zeros((nb, 6))
    if nb > 1:
        dq = q[:, None, :] - q[None, :, :]
        r = np.linalg.norm(dq, axis=2) + np.eye(nb) * 1e9
        F[:, :3] += np.sum(mag(r, 2 * radius)[:, :, None] * dq / r[:, :, None], axis=1)
    L = np.array(n, dtype=float) * h
    F[:, :3] += mag(q, radius) - mag(L[None, :] - q, radius)
    return F


# ----------------------------------------------------------------- GPU run
def run_gpu(w, steps, warmup, fp32, seed=2024, timing=False):
    import torch
    import paper_1901_06427_amd as rb
    from tests.helpers import lib_context
    ctx = lib_context(rb, w, tol=w.tol, precond_fp32=fp32, min_body_dist=0.0)
    q = torch.as_tensor(w.q, dtype=torch.float64).cuda().contiguous()
    th = torch.as_tensor(w.theta, dtype=torch.float64).cuda().contiguous()
    U = torch.empty((w.nb, 6), dtype=torch.float64, device="cuda")
    R = float(w.radius[0])
    step_id = 0
    iters = 0
    rejected = 0

    def one():
        nonlocal step_id, iters, rejected
        F = soft_forces_torch(q, R, w.n, w.h, w.kT)
        info = rb.rbfib_sem_step(ctx, q, th, F, w.kT, w.dt, seed, step_id, U)
        step_id += 1
        iters += sum(i.iters for i in info)
        rejected += sum(1 for i in info if i.status == rb.RBFIB_EREJECT)

    for _ in range(warmup):
        one()
    iters = 0
    rejected = 0
    if timing:
        rb.rbfib_enable_timing(ctx, True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        one()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    stats = {}
    if timing:
        for which, name in ((0, "mac_saddle_apply"), (1, "mg_smooth_level0")):
            avg_ms, nbytes, launches = rb.rbfib_kernel_stats(ctx, which)
            stats[name] = (avg_ms, nbytes, launches)
    out = {"seconds": t1 - t0, "steps": steps, "iters": iters, "rejected": rejected, "stats": stats}
    ctx.close()
    return out


# ----------------------------------------------------------------- CPU oracle baseline
def run_cpu_baseline(w, budget_s=20.0, seed=2024):
    """The oracle's SEM step as it stands (FP64, solves to 1e-12), single thread."""
    from threadpoolctl import threadpool_limits
    from oracle import mac, sem
    g = mac.Grid(w.n, w.bc, w.h, w.eta, w.wall_vel)
    q, th = w.q.copy(), w.theta.copy()
    R = float(w.radius[0])
    n_steps = 0
    with threadpool_limits(limits=1):
        t0 = time.perf_counter()
        while True:
            F = soft_forces_np(q, R, w.n, w.h, w.kT)
            res = sem.sem_step(g, w.r_ref, w.offsets, q, th, F, w.kT, w.dt, seed, n_steps)
            q, th = res.q, res.theta
            n_steps += 1
            if time.perf_counter() - t0 > budget_s:
                break
        t1 = time.perf_counter()
    return {"steps": n_steps, "seconds": t1 - t0}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=40)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--plain-steps", type=int, default=None)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-budget", type=float, default=20.0)
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py measures one GPU: every box here has a single MI355X, and the hot path "
              "(one confined suspension per device) is not sharded across GPUs; run with --gpus 1.",
              file=sys.stderr)
        sys.exit(2)

    import torch
    import workloads as W
    w = W.two_spheres()
    log("workload two_spheres: grid", w.n, "bodies", w.nb, "markers", w.nm)

    fast = run_gpu(w, args.steps, args.warmup, fp32=1, timing=True)
    plain = run_gpu(w, args.plain_steps or max(5, args.steps // 2), 2, fp32=0)
    solves_per_step = 2
    value = solves_per_step * fast["steps"] / fast["seconds"]
    plain_value = solves_per_step * plain["steps"] / plain["seconds"]
    log("fp32-pc: %.1f solves/s, %.1f iters/step; fp64-pc: %.1f solves/s" %
        (value, fast["iters"] / fast["steps"], plain_value))

    # roofline of the dominant kernel class (by measured total time)
    st = fast["stats"]
    best = max(st.items(), key=lambda kv: kv[1][0] * kv[1][2])
    name, (avg_ms, nbytes, launches) = best
    achieved = nbytes / (avg_ms * 1e-3) / 1e9 if avg_ms > 0 else 0.0
    roofline = {"bound": "hbm", "kernel": name, "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": None,
                "avg_us": round(avg_ms * 1e3, 2), "bytes_per_launch": nbytes, "launches": launches}
    others = {k: {"avg_us": round(v[0] * 1e3, 2), "launches": v[2],
                  "GB/s": round(v[1] / (v[0] * 1e-3) / 1e9, 1) if v[0] > 0 else 0.0} for k, v in st.items()}

    cpu = None
    if not args.no_cpu_baseline:
        cb = run_cpu_baseline(w, args.cpu_budget)
        cpu = {"value": round(solves_per_step * cb["steps"] / cb["seconds"], 4), "unit": "mobility solves/s",
               "cores": 1, "kind": "oracle",
               "sample": "%d SEM steps of the same workload (FP64 oracle, solves to 1e-12, 1 thread)" % cb["steps"]}

    ms_per_step = 1e3 * fast["seconds"] / fast["steps"]
    line = {
        "metric": METRIC,
        "value": round(value, 3),
        "unit": "mobility solves/s",
        "n_gpus": 1,
        "steps": fast["steps"],
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "two_spheres_32x32x64_sem", "grid": list(w.n), "bodies": w.nb, "markers": w.nm,
                   "kT": w.kT, "dt": w.dt, "tol": w.tol, "precond": "fp32 multigrid", "solves_per_step": 2,
                   "fgmres_iters_per_step": round(fast["iters"] / fast["steps"], 2),
                   "rejected_steps": fast["rejected"]},
        "plain_fp64": {"value": round(plain_value, 3), "unit": "mobility solves/s",
                       "fgmres_iters_per_step": round(plain["iters"] / plain["steps"], 2),
                       "ratio_fp32pc_over_plain": round(value / plain_value, 3)},
        "roofline": roofline,
        "kernels": others,
        "cpu_baseline": cpu,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
