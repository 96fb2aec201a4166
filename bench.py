"""Benchmark of the RB-FIB mobility-solve hot path on one MI355X.

Headline workload: an ensemble of 256 independent walled boxes (edge drawn from
16/24/32/48 cells, h = 1, viscosity 1) holding 1-4 spheres of 42 markers and
radius 2.5 h each, kT = 1, dt = 0.01, soft steric repulsion, fluctuating
stress on cells and edges.  One benchmark step advances every replica by one
Split-Euler-Maruyama step (Algorithm 1: two constrained mobility solves and
one unconstrained Stokes solve per replica, each to a relative residual of
1e-6) in one batched launch sequence with the FP32 multigrid preconditioner
and captured HIP graphs.  "plain_fp64" solves the same replicas one at a time
with the FP64 preconditioner on the same GPU; "two_spheres" is the 32x32x64
two-sphere box of the paper's tight-cavity example, one replica;
"single_sphere_32" times deterministic mobility solves of one sphere in a walled
32^3 box to 1e-8 with both preconditioner precisions; "monolayer_1024" times SEM steps of the 1024-sphere sliding-wall monolayer with
the FP32 and the FP64 multigrid; "adjoint_128" times the forward solve and the
vector-Jacobian product on the 128^3 box with 64 spheres.

Inputs are seeded and synthetic, and resident in GPU memory before the timed
region.  The roofline object is for the kernel class that dominates the
headline's graph-mode launches (the basis update of a two-step Arnoldi block),
timed with HIP events inside the library on its own stream in a short eager
run; the CPU
baseline is the FP64 oracle's SEM step on a bounded sample of replicas.
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


# ----------------------------------------------------------------- GPU runs
class Ensemble:
    """Concatenated replicas plus per-body data for the caller-side forces."""

    def __init__(self, ws):
        import torch
        self.ws = ws
        self.nb = sum(w.nb for w in ws)
        self.q = torch.as_tensor(np.concatenate([w.q for w in ws]), dtype=torch.float64).cuda().contiguous()
        self.th = torch.as_tensor(np.concatenate([w.theta for w in ws]), dtype=torch.float64).cuda().contiguous()
        rep = np.concatenate([np.full(w.nb, r) for r, w in enumerate(ws)])
        box = np.concatenate([np.tile(np.array(w.n, dtype=float) * w.h, (w.nb, 1)) for w in ws])
        self.rep = torch.as_tensor(rep).cuda()
        self.box = torch.as_tensor(box, dtype=torch.float64).cuda()
        self.R = float(ws[0].radius[0])
        self.kT = ws[0].kT
        self.dt = ws[0].dt

    def forces(self):
        """Soft steric forces, pairs only within a replica (see soft_forces_torch)."""
        import torch
        q = self.q
        phi0 = 4.0 * self.kT
        b = 0.1 * self.R

        def mag(r, d):
            return torch.where(r < d, torch.full_like(r, phi0) / b, (phi0 / b) * torch.exp((d - r) / b))

        F = torch.zeros((self.nb, 6), dtype=q.dtype, device=q.device)
        F[:, :3] += mag(q, self.R) - mag(self.box - q, self.R)
        # bodies of one replica are contiguous: loop over the (<= 4) partner offsets
        for o in range(1, 4):
            if o >= self.nb:
                break
            same = self.rep[o:] == self.rep[:-o]
            d = q[:-o] - q[o:]
            r = torch.linalg.norm(d, dim=1).clamp_min(1e-12)
            f = torch.where(same[:, None], mag(r, 2 * self.R)[:, None] * d / r[:, None], torch.zeros_like(d))
            F[:-o, :3] += f
            F[o:, :3] -= f
        return F


MG_FUSED = 0
RESTART = 0       # 0: the library default
SWEEPS = 0        # 0: the library default
OMEGA = 0.0       # 0: the library default
PSWEEPS = 0       # 0: the library default
BLOB = 0.0        # 0: the library default
BOTTOM = -1       # -1: the library default
CHEBY = -1.0      # < 0: the library default
EXTRA_OPTS = {}   # further rbfib_opts fields (--opt name=value)


def lib_context(rb, ws, **opt_kw):
    """A batched library context for workloads ws (the GPU leg builds its contexts
    through the binding alone; nothing under oracle/ is imported here)."""
    grids = [rb.make_grid(w.n, w.bc, w.h, w.eta, w.wall_vel) for w in ws]
    opts = rb.rbfib_default_opts(**opt_kw)
    return rb.rbfib_create_batch(grids, [w.r_ref for w in ws], [w.offsets for w in ws], opts)


def run_gpu(ws, steps, warmup, fp32, seed=2024, timing=False, graphs=True, tol=None, keep_first_U=False):
    """`steps` timed SEM launches after `warmup` untimed ones.  Replica r draws from
    seed + r; launch k uses step counter k.  keep_first_U: the velocities of launch 0
    (a warm-up launch from the initial configuration) are copied to the host after
    it, outside the timed region."""
    import torch
    import paper_1901_06427_amd as rb
    E = Ensemble(ws)
    ctx = lib_context(rb, ws, tol=ws[0].tol if tol is None else tol, precond_fp32=fp32,
                      use_graphs=int(graphs and not timing),
                      mg_fused=MG_FUSED, **({"restart": RESTART} if RESTART else {}),
                      **({"mg_sweeps": SWEEPS} if SWEEPS else {}), **({"mg_omega": OMEGA} if OMEGA else {}),
                      **({"mg_sweeps_p": PSWEEPS} if PSWEEPS else {}), **({"blob_radius": BLOB} if BLOB else {}),
                      **({"mg_bottom": BOTTOM} if BOTTOM >= 0 else {}),
                      **({"mg_cheby": CHEBY} if CHEBY >= 0 else {}), **EXTRA_OPTS)
    U = torch.empty((E.nb, 6), dtype=torch.float64, device="cuda")
    step_id = 0
    iters = 0
    rejected = 0

    def one():
        nonlocal step_id, iters, rejected
        info = rb.rbfib_sem_step(ctx, E.q, E.th, E.forces(), E.kT, E.dt, seed, step_id, U)
        step_id += 1
        iters += sum(i.iters for i in info)
        rejected += sum(1 for i in info if i.status == rb.RBFIB_EREJECT)

    first_U = None
    for k in range(warmup):
        one()
        if k == 0 and keep_first_U:
            first_U = U.cpu().numpy().copy()
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
        for which, name in TIMED_CLASSES:
            avg_ms, nbytes, launches = rb.rbfib_kernel_stats(ctx, which)
            if launches:
                stats[name] = (avg_ms, nbytes, launches)
    ctx.close()
    return {"seconds": t1 - t0, "steps": steps, "iters": iters, "rejected": rejected, "stats": stats,
            "replicas": len(ws), "first_U": first_U}


def run_plain(ws, warmup=1, seed=2024, tol=None):
    """The same replicas one at a time, FP64 preconditioner, one SEM step each (replica
    k of the ensemble draws from seed + k, as in the batched launches)."""
    total = 0.0
    iters = 0
    for k, w in enumerate(ws):
        r = run_gpu([w], 1, warmup, fp32=0, seed=seed + k, graphs=True, tol=tol)
        total += r["seconds"]
        iters += r["iters"]
    return {"seconds": total, "steps": len(ws), "iters": iters}


def _dev(a):
    import torch
    return torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float64).cuda()


TIMED_CLASSES = ((0, "mac_saddle_apply"), (1, "mg_smooth_level0"), (2, "mg_down_level0"), (3, "mg_up_level0"),
                 (4, "krylov_dots"), (5, "krylov_update"), (6, "spread"))


def class_rates(rb, ctx, run):
    """Per-class launches, mean duration and algorithmic GB/s (HIP events inside the
    library, eager context) over one call of run()."""
    import torch
    rb.rbfib_enable_timing(ctx, True)
    run()
    torch.cuda.synchronize()
    out = {}
    for which, name in TIMED_CLASSES:
        avg_ms, nbytes, launches = rb.rbfib_kernel_stats(ctx, which)
        if launches:
            out[name] = {"avg_us": round(avg_ms * 1e3, 2), "launches": launches,
                         "GB/s": round(nbytes / (avg_ms * 1e-3) / 1e9, 1) if avg_ms > 0 else 0.0}
    return out


def run_monolayer(steps, seed=2024):
    """The 1024-sphere monolayer (256x128x32, periodic x, walls y and z, sliding bottom
    wall): SEM steps with the FP32 multigrid inside FP64 FGMRES and with the all-FP64
    preconditioner, from the same configuration with the same random numbers.  Step 0
    of each is untimed and its velocities are compared between the two; steps 1..steps
    are timed."""
    import torch
    import paper_1901_06427_amd as rb
    import workloads as W
    w = W.monolayer()
    out, U0 = {}, {}
    for fp32 in (1, 0):
        ctx = lib_context(rb, [w], tol=w.tol, precond_fp32=fp32, **({"mg_bottom": BOTTOM} if BOTTOM >= 0 else {}))
        q, th, FT = _dev(w.q), _dev(w.theta), _dev(w.FT)
        U = torch.empty((w.nb, 6), dtype=torch.float64, device="cuda")
        rb.rbfib_sem_step(ctx, q, th, FT, w.kT, w.dt, seed, 0, U)
        U0[fp32] = U.cpu().numpy()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        iters = 0
        for k in range(1, steps + 1):
            info = rb.rbfib_sem_step(ctx, q, th, FT, w.kT, w.dt, seed, k, U)
            iters += info[0].iters
        torch.cuda.synchronize()
        sec = (time.perf_counter() - t0) / steps
        ctx.close()
        out["fp32_pc" if fp32 else "fp64_pc"] = {"ms_per_step": round(1e3 * sec, 2), "solves_per_s": round(2 / sec, 3),
                                                 "fgmres_iters_per_step": round(iters / steps, 1)}
    d = float(np.abs(U0[1] - U0[0]).max() / np.abs(U0[0]).max())
    # kernel-class rates of one eager SEM step with the FP32 multigrid
    ctx = lib_context(rb, [w], tol=w.tol, precond_fp32=1, use_graphs=0,
                      **({"mg_bottom": BOTTOM} if BOTTOM >= 0 else {}))
    q, th, FT = _dev(w.q), _dev(w.theta), _dev(w.FT)
    U = torch.empty((w.nb, 6), dtype=torch.float64, device="cuda")
    out["kernels_fp32_pc"] = class_rates(rb, ctx, lambda: rb.rbfib_sem_step(ctx, q, th, FT, w.kT, w.dt, seed, 1, U))
    ctx.close()
    out.update({"grid": list(w.n), "bodies": w.nb, "markers": w.nm, "tol": w.tol, "timed_steps": steps,
                "U_rel_diff_fp32_vs_fp64_pc": d,
                "speedup_fp32_pc": round(out["fp64_pc"]["ms_per_step"] / out["fp32_pc"]["ms_per_step"], 3)})
    return out


def run_single_sphere(solves=20, tol=1e-8):
    """One 42-marker sphere in a walled 32^3 box: deterministic mobility solves
    (forces and torques only) to tol, with the FP32 multigrid and with the all-FP64
    preconditioner; two untimed solves first."""
    import torch
    import paper_1901_06427_amd as rb
    import workloads as W
    w = W.single_sphere()
    out = {"grid": list(w.n), "bodies": w.nb, "markers": w.nm, "tol": tol, "timed_solves": solves}
    for fp32 in (1, 0):
        ctx = lib_context(rb, [w], tol=tol, precond_fp32=fp32)
        q, th, FT = _dev(w.q), _dev(w.theta), _dev(w.FT)
        U = torch.empty((w.nb, 6), dtype=torch.float64, device="cuda")
        for _ in range(2):
            rb.rbfib_solve_mobility(ctx, q, th, FT, U)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        iters, res = 0, 0.0
        for _ in range(solves):
            info = rb.rbfib_solve_mobility(ctx, q, th, FT, U)
            iters += info[0].iters
            res = max(res, info[0].rel_residual)
        torch.cuda.synchronize()
        sec = (time.perf_counter() - t0) / solves
        ctx.close()
        out["fp32_pc" if fp32 else "fp64_pc"] = {"solves_per_s": round(1.0 / sec, 2), "ms_per_solve": round(1e3 * sec, 3),
                                                 "fgmres_iters_per_solve": round(iters / solves, 1),
                                                 "max_rel_residual": res}
    return out


def run_adjoint(tol=1e-10, reps=2):
    """The differentiated solve: 64 spheres of 42 markers in a 128^3 walled box; the
    forward mobility solve and the vector-Jacobian product (forward re-solve plus the
    adjoint solve, then the gradient kernels), FP32 multigrid, best of reps."""
    import torch
    import paper_1901_06427_amd as rb
    import workloads as W
    w = W.many_spheres()
    ctx = lib_context(rb, [w], tol=tol, precond_fp32=1)
    q, th, FT = _dev(w.q), _dev(w.theta), _dev(w.FT)
    U = torch.empty((w.nb, 6), dtype=torch.float64, device="cuda")
    Ubar = _dev(np.random.default_rng(5).standard_normal((w.nb, 6)))
    dFT, dq, dphi = (torch.empty((w.nb, k), dtype=torch.float64, device="cuda") for k in (6, 3, 3))
    best_f = best_b = float("inf")
    it_f = it_b = 0
    for _ in range(reps):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        inf = rb.rbfib_solve_mobility(ctx, q, th, FT, U, include_bc=False, allow=())
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        infb = rb.rbfib_mobility_vjp(ctx, q, th, FT, Ubar, dFT, dq, dphi, allow=())
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        best_f, best_b = min(best_f, t1 - t0), min(best_b, t2 - t1)
        it_f, it_b = inf[0].iters, infb[0].iters
    ctx.close()
    # kernel-class rates of one eager forward solve plus vector-Jacobian product
    ctx = lib_context(rb, [w], tol=tol, precond_fp32=1, use_graphs=0)

    def fwd_bwd():
        rb.rbfib_solve_mobility(ctx, q, th, FT, U, include_bc=False, allow=())
        rb.rbfib_mobility_vjp(ctx, q, th, FT, Ubar, dFT, dq, dphi, allow=())
    rates = class_rates(rb, ctx, fwd_bwd)
    ctx.close()
    return {"grid": list(w.n), "bodies": w.nb, "markers": w.nm, "tol": tol,
            "forward_ms": round(1e3 * best_f, 2), "forward_iters": it_f,
            "vjp_ms": round(1e3 * best_b, 2), "vjp_iters": it_b,
            "forward_plus_backward_ms": round(1e3 * (best_f + best_b), 2), "kernels": rates}


# ----------------------------------------------------------------- CPU oracle baseline
_CPU_ENS = None


def _cpu_init():
    from threadpoolctl import threadpool_limits
    threadpool_limits(limits=1)


def _cpu_step(k, seed=2024):
    """One oracle SEM step on replica k of the default ensemble (worker process), with
    the random numbers the GPU's first launch draws for that replica (seed + k, step
    counter 0) and the same forces; returns (k, U)."""
    global _CPU_ENS
    import workloads as W
    from oracle import mac, sem
    if _CPU_ENS is None:
        _CPU_ENS = W.ensemble()
    w = _CPU_ENS[k]
    g = mac.Grid(w.n, w.bc, w.h, w.eta, w.wall_vel)
    F = soft_forces_np(w.q, float(w.radius[0]), w.n, w.h, w.kT)
    res = sem.sem_step(g, w.r_ref, w.offsets, w.q, w.theta, F, w.kT, w.dt, seed + k, 0)
    return k, res.U


def run_cpu_baseline(n_replicas, budget_s=20.0):
    """The oracle's SEM step as it stands (FP64, solves to 1e-12), one single-threaded
    process per host core (at most 16), replicas taken in ensemble order until the
    time budget is used.  Runs before anything touches the GPU.  Returns the oracle's
    velocities of the replicas it finished (the reference for the GPU's error)."""
    import multiprocessing as mp
    cores = max(1, min(16, os.cpu_count() or 1))
    ctx = mp.get_context("spawn")
    U = {}
    with ctx.Pool(cores, initializer=_cpu_init) as pool:
        pool.map(_cpu_step, [0] * cores, chunksize=1)       # import and build once per worker, untimed
        done = 0
        t0 = time.perf_counter()
        for k, Uk in pool.imap_unordered(_cpu_step, range(n_replicas), chunksize=1):
            done += 1
            U[k] = Uk
            if time.perf_counter() - t0 > budget_s:
                break
        t1 = time.perf_counter()
        pool.terminate()
    return {"steps": done, "seconds": t1 - t0, "cores": cores, "U": U}


def oracle_error(U_gpu, U_ref, ws):
    """Largest and median over the replicas of max |U_gpu - U_oracle| / max |U_oracle|
    (one SEM step, every velocity component of the replica's bodies)."""
    if U_gpu is None or not U_ref:
        return None
    b0 = np.cumsum([0] + [w.nb for w in ws])
    errs = []
    for k, Ur in sorted(U_ref.items()):
        Ug = U_gpu[b0[k]:b0[k + 1]]
        errs.append(float(np.abs(Ug - Ur).max() / max(np.abs(Ur).max(), 1e-300)))
    return {"max": float(max(errs)), "median": float(np.median(errs)), "replicas": len(errs)}


def copy_ceiling():
    """Achieved device-to-device copy bandwidth (read + write bytes / time) of 1 GiB
    arrays, timed with events on torch's stream, which the copy runs on."""
    import torch
    a = torch.ones(128 * 1024 * 1024, dtype=torch.float64, device="cuda")
    b = torch.empty_like(a)
    for _ in range(3):
        b.copy_(a)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(10):
        b.copy_(a)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / 10
    del a, b
    return 2 * 128 * 1024 * 1024 * 8 / (ms * 1e-3) / 1e9


COUNTERS = os.path.join(ROOT, "profiles", "ensemble_256_sem_hbm_counters.md")
KERNEL_SOURCES = ("paper_1901_06427_amd/csrc/grid.hip", "paper_1901_06427_amd/csrc/krylov.hip",
                  "paper_1901_06427_amd/csrc/common.h", "paper_1901_06427_amd/csrc/ib.hip")


def _code_tokens(text):
    """Source text without comments, whitespace runs outside literals collapsed to one
    space: what the compiler sees, so that editing a comment does not mark the
    counters stale."""
    out, i, n = [], 0, len(text)

    def space():
        if out and out[-1] != " ":
            out.append(" ")

    while i < n:
        c = text[i]
        if text.startswith("//", i):
            j = text.find("\n", i)
            i = n if j < 0 else j
        elif text.startswith("/*", i):
            j = text.find("*/", i + 2)
            i = n if j < 0 else j + 2
            space()
        elif c in "\"'":
            j = i + 1
            while j < n and text[j] != c:
                j += 2 if text[j] == "\\" else 1
            out.append(text[i:j + 1])
            i = j + 1
        elif c.isspace():
            space()
            i += 1
        else:
            out.append(c)
            i += 1
    return "".join(out).strip()


def kernel_source_hash():
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, f), encoding="utf-8") as fh:
            h.update(_code_tokens(fh.read()).encode())
    return h.hexdigest()[:16]


def measured_traffic(kernel):
    """HBM bytes per launch of a kernel class from the committed counter summary
    (FETCH_SIZE and WRITE_SIZE, each scaled by the counts of a calibration
    kernel of known size); None when the kernel sources changed since."""
    try:
        with open(COUNTERS) as fh:
            for line in fh:
                f = line.split()
                if len(f) == 6 and f[0] == "traffic:" and f[1] == kernel and f[4] == "sources":
                    return float(f[2]) if f[5] == kernel_source_hash() else None
    except OSError:
        return None
    return None


# The kernel class with the largest share of kernel time in the headline's graph-mode
# launches (rocprofv3 kernel trace of `bench.py --batched-only`): the basis update of a
# two-step Arnoldi block.  Its launches are timed with HIP events in an eager launch.
ROOFLINE_CLASS = "krylov_update"


def roofline_of(stats, ensemble_default=True):
    name = ROOFLINE_CLASS if ROOFLINE_CLASS in stats else max(stats.items(), key=lambda kv: kv[1][0] * kv[1][2])[0]
    avg_ms, nbytes, launches = stats[name]
    achieved = nbytes / (avg_ms * 1e-3) / 1e9 if avg_ms > 0 else 0.0
    traffic = measured_traffic(name) if ensemble_default else None
    roof = {"bound": "hbm", "kernel": name, "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic, "avg_us": round(avg_ms * 1e3, 2),
            "bytes_per_launch": nbytes, "launches": launches}
    others = {k: {"avg_us": round(v[0] * 1e3, 2), "launches": v[2],
                  "GB/s": round(v[1] / (v[0] * 1e-3) / 1e9, 1) if v[0] > 0 else 0.0} for k, v in stats.items()}
    return roof, others


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2, help="timed batched SEM launches")
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--replicas", type=int, default=256)
    ap.add_argument("--plain-replicas", type=int, default=24, help="replicas timed one at a time")
    ap.add_argument("--two-spheres-steps", type=int, default=20)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--tight-tol", type=float, default=1e-10,
                    help="second batched-vs-plain comparison at this tolerance (0: skip)")
    ap.add_argument("--tight-steps", type=int, default=3, help="timed batched launches at the tight tolerance")
    ap.add_argument("--cpu-budget", type=float, default=20.0)
    ap.add_argument("--monolayer-steps", type=int, default=3,
                    help="timed SEM steps of the 1024-sphere monolayer per preconditioner precision (0: skip)")
    ap.add_argument("--no-adjoint", action="store_true", help="skip the 128^3 differentiated solve")
    ap.add_argument("--copy-probe", action="store_true",
                    help="run one elementwise kernel reading and writing 256 MiB first (counter calibration)")
    ap.add_argument("--timing-only", action="store_true",
                    help="only the eager timed run of the ensemble (one SEM launch, no masking of converged "
                         "replicas, no graphs): the command the hardware-counter profiles are taken on")
    ap.add_argument("--mg-bottom", type=int, default=-1,
                    help="LDS budget in KB of the bottom multigrid kernel, 0 off (-1: library default)")
    ap.add_argument("--mg-cheby", type=float, default=-1.0,
                    help="lower end of the Chebyshev smoothing interval, 0 constant weights (-1: library default)")
    ap.add_argument("--opt", action="append", default=[], metavar="NAME=VALUE",
                    help="set any other solver option field (repeatable)")
    ap.add_argument("--restart", type=int, default=0, help="FGMRES restart length (0: library default)")
    ap.add_argument("--mg-sweeps", type=int, default=0, help="damped-Jacobi sweeps per level (0: library default)")
    ap.add_argument("--mg-omega", type=float, default=0.0, help="Jacobi damping (0: library default)")
    ap.add_argument("--mg-sweeps-p", type=int, default=0, help="pressure-cycle sweeps (0: library default)")
    ap.add_argument("--blob-radius", type=float, default=0.0,
                    help="blob radius of the body-block preconditioner, units of h (0: library default)")
    ap.add_argument("--batched-only", action="store_true",
                    help="only the batched ensemble launches (the command the graph-mode trace is taken on)")
    ap.add_argument("--two-spheres-only", action="store_true",
                    help="only the SEM steps of the 32x32x64 two-sphere box (its kernel trace)")
    ap.add_argument("--monolayer-only", action="store_true",
                    help="only the SEM steps of the 1024-sphere monolayer")
    ap.add_argument("--single-sphere-only", action="store_true",
                    help="only the mobility solves of one sphere in a 32^3 box")
    ap.add_argument("--adjoint-only", action="store_true",
                    help="only the 128^3 differentiated solve")
    ap.add_argument("--mg-fused", type=int, default=0, choices=(0, 1, 2),
                    help="multigrid level kernels: 0 separate (default), 1 fused where the level fills the "
                         "device, 2 fused on every level")
    args = ap.parse_args()
    global MG_FUSED, RESTART, SWEEPS, OMEGA, PSWEEPS, BLOB, BOTTOM, CHEBY, EXTRA_OPTS
    MG_FUSED = args.mg_fused
    RESTART = args.restart
    BOTTOM = args.mg_bottom
    CHEBY = args.mg_cheby
    for kv in args.opt:
        k, v = kv.split("=", 1)
        EXTRA_OPTS[k] = float(v) if any(ch in v for ch in ".eE") else int(v)
    SWEEPS = args.mg_sweeps
    OMEGA = args.mg_omega
    PSWEEPS = args.mg_sweeps_p
    BLOB = args.blob_radius
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py measures one GPU: every box here has a single MI355X, and the replicas of the "
              "ensemble share one device; run with --gpus 1.", file=sys.stderr)
        sys.exit(2)

    cpu = None
    cb = None
    if args.two_spheres_only or args.monolayer_only or args.single_sphere_only or args.adjoint_only:
        import workloads as W
        out = {}
        if args.single_sphere_only:
            out["single_sphere_32"] = run_single_sphere()
        if args.two_spheres_only:
            two = run_gpu([W.two_spheres()], args.two_spheres_steps, 2, fp32=1)
            out["two_spheres"] = {"value": round(2 * two["steps"] / two["seconds"], 3), "unit": "mobility solves/s",
                                  "ms_per_step": round(1e3 * two["seconds"] / two["steps"], 3),
                                  "fgmres_iters_per_step": round(two["iters"] / two["steps"], 1),
                                  "us_per_iter": round(1e6 * two["seconds"] / two["iters"], 1)}
        if args.monolayer_only:
            out["monolayer_1024"] = run_monolayer(max(1, args.monolayer_steps))
        if args.adjoint_only:
            out["adjoint_128"] = run_adjoint()
        out["mg_bottom"] = BOTTOM
        print(json.dumps(out), flush=True)
        return

    if not args.no_cpu_baseline and not args.timing_only and not args.batched_only:
        cb = run_cpu_baseline(args.replicas, args.cpu_budget)
        cpu = {"value": round(2 * cb["steps"] / cb["seconds"], 4), "unit": "mobility solves/s",
               "cores": cb["cores"], "kind": "oracle",
               "sample": "one SEM step on each of %d ensemble replicas in ensemble order (FP64 oracle, solves "
                         "to 1e-12, the random numbers of the GPU's first launch), %d single-threaded "
                         "processes, %.1f s" % (cb["steps"], cb["cores"], cb["seconds"])}
        log("cpu oracle: %.3f solves/s on %d processes" % (cpu["value"], cb["cores"]))

    import torch
    import workloads as W
    if args.copy_probe:
        # one elementwise kernel that reads 256 MiB and writes 256 MiB: the
        # calibration dispatch for the FETCH_SIZE / WRITE_SIZE counters
        a = torch.ones(32 * 1024 * 1024, dtype=torch.float64, device="cuda")
        b = torch.empty_like(a)
        torch.cuda.synchronize()
        torch.mul(a, 2.0, out=b)
        torch.cuda.synchronize()
        del a, b
    ens = W.ensemble(n_replicas=args.replicas)
    log("ensemble: %d replicas, %d bodies, %d markers" % (len(ens), sum(w.nb for w in ens), sum(w.nm for w in ens)))
    if args.timing_only:
        timing = run_gpu(ens, 1, 0, fp32=1, timing=True)
        roofline, kernels = roofline_of(timing["stats"], args.replicas == 256 and MG_FUSED == 0)
        print(json.dumps({"timing_only": True, "roofline": roofline, "kernels": kernels,
                          "kernel_sources": kernel_source_hash()}), flush=True)
        return

    batched = run_gpu(ens, args.steps, args.warmup, fp32=1, keep_first_U=args.warmup > 0)
    solves = 2 * batched["replicas"] * batched["steps"]
    value = solves / batched["seconds"]
    log("batched fp32-pc: %.1f solves/s (%.2f s per launch)" % (value, batched["seconds"] / batched["steps"]))
    if args.batched_only:
        print(json.dumps({"batched_only": True, "value": round(value, 3), "steps": batched["steps"],
                          "fgmres_iters_per_launch": batched["iters"] / batched["steps"]}), flush=True)
        return
    U_oracle = cb["U"] if cpu is not None else None
    err = oracle_error(batched["first_U"], U_oracle, ens)
    if err:
        log("batched at tol %.0e: U error vs oracle max %.2e median %.2e over %d replicas"
            % (ens[0].tol, err["max"], err["median"], err["replicas"]))

    plain = run_plain(ens[:args.plain_replicas])
    plain_value = 2 * plain["steps"] / plain["seconds"]
    log("plain fp64-pc, one replica at a time: %.1f solves/s" % plain_value)

    # the same comparison at a tolerance tight enough for the velocities to agree with
    # the oracle to ~1e-6 (the relative residual is dominated by the fluctuating
    # forcing, so 1e-6 of it leaves U with a larger relative error)
    tight = None
    if args.tight_tol > 0:
        bt = run_gpu(ens, max(1, min(args.steps, args.tight_steps)), 1, fp32=1, tol=args.tight_tol,
                     keep_first_U=True)
        vt = 2 * bt["replicas"] * bt["steps"] / bt["seconds"]
        pt = run_plain(ens[:args.plain_replicas], tol=args.tight_tol)
        pvt = 2 * pt["steps"] / pt["seconds"]
        et = oracle_error(bt["first_U"], U_oracle, ens)
        tight = {"tol": args.tight_tol, "batched": round(vt, 3), "plain_fp64": round(pvt, 3),
                 "ratio_batched_over_plain": round(vt / pvt, 3), "steps": bt["steps"],
                 "fgmres_iters_per_launch": round(bt["iters"] / bt["steps"], 1), "oracle_err": et}
        log("tol %.0e: batched %.1f, plain %.1f solves/s; U error vs oracle %s" % (args.tight_tol, vt, pvt, et))

    timing = run_gpu(ens, 1, 0, fp32=1, timing=True)
    roofline, kernels = roofline_of(timing["stats"], args.replicas == 256 and MG_FUSED == 0)
    roofline["copy_ceiling_GBps"] = round(copy_ceiling(), 1)

    w2 = W.two_spheres()
    two = run_gpu([w2], args.two_spheres_steps, 2, fp32=1)
    two_value = 2 * two["steps"] / two["seconds"]
    log("two spheres: %.1f solves/s" % two_value)

    single = run_single_sphere()
    log("single sphere 32^3: %.1f solves/s (fp32 pc), %.1f (fp64 pc)" % (
        single["fp32_pc"]["solves_per_s"], single["fp64_pc"]["solves_per_s"]))
    mono = run_monolayer(args.monolayer_steps) if args.monolayer_steps > 0 else None
    if mono:
        log("monolayer: fp32-pc %.1f ms/step, fp64-pc %.1f ms/step, U rel diff %.2e" % (
            mono["fp32_pc"]["ms_per_step"], mono["fp64_pc"]["ms_per_step"], mono["U_rel_diff_fp32_vs_fp64_pc"]))
    adj = run_adjoint() if not args.no_adjoint else None
    if adj:
        log("128^3 adjoint: forward %.1f ms, vjp %.1f ms" % (adj["forward_ms"], adj["vjp_ms"]))
    import paper_1901_06427_amd as rb
    gctx = lib_context(rb, ens, tol=1e-6, precond_fp32=1)
    geometry = rb.rbfib_launch_geometry(gctx)
    gctx.close()

    n_cells = sum(int(np.prod(w.n)) for w in ens)
    line = {
        "metric": METRIC,
        "value": round(value, 3),
        "unit": "mobility solves/s",
        "n_gpus": 1,
        "steps": batched["steps"],
        "warmup": args.warmup,
        "ms_per_step": round(1e3 * batched["seconds"] / batched["steps"], 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "ensemble_256_walled_boxes_sem", "replicas": len(ens),
                   "edges": [16, 24, 32, 48], "cells": n_cells, "bodies": sum(w.nb for w in ens),
                   "markers": sum(w.nm for w in ens), "kT": 1.0, "dt": 0.01, "tol": 1e-6,
                   "precond": "fp32 multigrid", "solves_per_step_per_replica": 2,
                   "fgmres_iters_per_launch": round(batched["iters"] / batched["steps"], 1),
                   "rejected": batched["rejected"], "launch_geometry": geometry},
        "oracle_err": err,
        "plain_fp64": {"value": round(plain_value, 3), "unit": "mobility solves/s",
                       "sample": "first %d replicas, one SEM step each, solved one at a time" % plain["steps"],
                       "ratio_batched_over_plain": round(value / plain_value, 3)},
        "tight_tolerance": tight,
        "two_spheres": {"value": round(two_value, 3), "unit": "mobility solves/s", "grid": [32, 32, 64],
                        "ms_per_step": round(1e3 * two["seconds"] / two["steps"], 3),
                        "fgmres_iters_per_step": round(two["iters"] / two["steps"], 1)},
        "single_sphere_32": single,
        "monolayer_1024": mono,
        "adjoint_128": adj,
        "roofline": roofline,
        "kernels": kernels,
        "cpu_baseline": cpu,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
