"""Launch geometries the autotuner may choose (Krylov chunk, spreading pairs per
LDS round and grid, multigrid points per thread), forced through a table file
(RBFIB_TUNING) at context creation: the context reports the geometry it took, the
apply still matches the oracle to 1e-10, a solve stays within its residual bound,
and a batch still equals its replicas solved alone bit for bit (every geometry
keeps a fixed summation order)."""
import os

import numpy as np
import pytest

import workloads as W
from oracle.saddle import Saddle
from tests.helpers import dev, error_gains, lib_context, oracle_grid, oracle_to_padded, padded_to_oracle
from tests.parity_configs import ensemble_replicas

pytestmark = pytest.mark.gpu

GEOMETRIES = [(512, 65536, 32, 0), (2048, 65536, 32, 0), (1024, 1024, 16, 1), (1024, 4096, 64, 4),
              (512, 16384, 64, 1)]


@pytest.fixture(scope="module")
def rb():
    import paper_1901_06427_amd as rb
    return rb


@pytest.fixture
def table(tmp_path):
    def write(geo):
        p = tmp_path / "tuning.txt"
        p.write_text("# forced geometry\n0 9223372036854775807 1 1000000 %d %d %d %d\n" % geo)
        os.environ["RBFIB_TUNING"] = str(p)
    yield write
    os.environ.pop("RBFIB_TUNING", None)


@pytest.mark.parametrize("geo", GEOMETRIES)
def test_geometry_apply_solve_batch(rb, table, geo):
    import torch
    table(geo)
    w = ensemble_replicas()["ensemble16_4spheres"]
    print("geometry", geo, flush=True)
    ctx = lib_context(rb, w, tol=1e-8, precond_fp32=1)
    got = rb.rbfib_launch_geometry(ctx)
    assert (got["krylov_chunk"], got["spread_grid"], got["spread_p"]) == geo[:3]
    assert got["mg_npt"] == (geo[3] if geo[3] else 1)
    s = Saddle(oracle_grid(w), w.q, w.theta, w.r_ref, w.offsets)
    x = np.random.default_rng(2).standard_normal(s.n)
    yd = torch.empty(ctx.L, dtype=torch.float64, device="cuda")
    rb.rbfib_apply_saddle(ctx, dev(w.q), dev(w.theta), dev(oracle_to_padded(s, x)), yd)
    y, yr = padded_to_oracle(s, yd.cpu().numpy()), s.A @ x
    for sl in (s.sl_v, s.sl_p, s.sl_l, s.sl_u):
        assert np.abs(y[sl] - yr[sl]).max() <= 1e-10 * np.abs(yr[sl]).max()
    b = s.rhs(FT=w.FT)
    U = torch.empty((w.nb, 6), dtype=torch.float64, device="cuda")
    xo = torch.empty(ctx.L, dtype=torch.float64, device="cuda")
    info = rb.rbfib_solve_mobility(ctx, dev(w.q), dev(w.theta), dev(w.FT), U, x_out=xo, allow=())
    res = s.residual(padded_to_oracle(s, xo.cpu().numpy()), b)
    x_ref, _ = s.solve_fgmres(b, tol=1e-12)
    bound = error_gains("ensemble16_4spheres").reshape(-1, 6) * (res + s.residual(x_ref, b)) * np.linalg.norm(b)
    print("  iters", info[0].iters, "residual", res, flush=True)
    assert res <= 1.05e-8
    assert np.all(np.abs(U.cpu().numpy() - s.split(x_ref)[3]) <= bound * (1 + 1e-6) + 1e-15)
    ctx.close()
    # a batch of mixed replicas equals the replicas alone under the same geometry
    reps = [W.spheres_in_box(101, (16, 16, 16), 1, name="r0"), W.spheres_in_box(102, (24, 24, 24), 3, name="r1"),
            W.spheres_in_box(104, (16, 16, 16), 4, R=1.5, shape="ico12", name="r3")]
    cb = lib_context(rb, reps, tol=1e-7, precond_fp32=1)
    cat = lambda k: dev(np.concatenate([getattr(r, k) for r in reps]))
    Ub = torch.empty((sum(r.nb for r in reps), 6), dtype=torch.float64, device="cuda")
    rb.rbfib_solve_mobility(cb, cat("q"), cat("theta"), cat("FT"), Ub, allow=())
    Ub = Ub.cpu().numpy()
    cb.close()
    b0 = 0
    for r in reps:
        c1 = lib_context(rb, r, tol=1e-7, precond_fp32=1)
        U1 = torch.empty((r.nb, 6), dtype=torch.float64, device="cuda")
        rb.rbfib_solve_mobility(c1, dev(r.q), dev(r.theta), dev(r.FT), U1, allow=())
        assert np.array_equal(Ub[b0:b0 + r.nb], U1.cpu().numpy())
        b0 += r.nb
        c1.close()
