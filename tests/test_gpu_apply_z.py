"""The z-marching fluid apply (launch geometry apply_kc > 0: x-y tiles of 16 x 16
cells marching through apply_kc planes, neighbours in LDS) against the
two-cells-per-thread apply (apply_kc = 0), forced through a table file
(RBFIB_TUNING) at context creation.

Both gather the same values and evaluate the same cell arithmetic, so the saddle
apply must be bit-identical, and so must a whole mobility solve with the FP32
preconditioner (whose FGMRES applies A to FP32 vectors).  Covered: walls on every
axis, periodic x (a 17-cell axis whose wrap crosses into another tile), a periodic
z axis (planes wrap), ragged tiles, a sliding wall, free-slip walls, a batch of
mixed replicas, and chunk lengths that do and do not divide the z extent.  The
apply also matches the oracle to 1e-10 per block.
"""
import copy
import os

import numpy as np
import pytest

import workloads as W
from oracle.saddle import Saddle
from tests.helpers import dev, lib_context, oracle_grid, oracle_to_padded, padded_to_oracle
from tests.parity_configs import slip_configs, solve_configs

pytestmark = pytest.mark.gpu

BIG = 9223372036854775807


def _configs():
    base = solve_configs()
    out = {k: base[k] for k in ("ragged_10x12x14", "periodic_wrap_17x12x12", "monolayer_64x32x16",
                                "ensemble16_4spheres", "ensemble48")}
    w = copy.deepcopy(base["ragged_10x12x14"])
    w.bc = (W.WALL, W.WALL, W.PERIODIC)
    out["periodic_z_10x12x14"] = w
    out["slip_wall_slip_10x12x14"] = slip_configs()["slip_wall_slip_10x12x14"]
    return out


CONFIGS = _configs()


@pytest.fixture(scope="module")
def rb():
    import paper_1901_06427_amd as rb
    return rb


@pytest.fixture
def table(tmp_path):
    def write(kc):
        p = tmp_path / "tuning.txt"
        p.write_text("# forced z-apply planes\n0 %d 1 1000000 1024 65536 32 0 %d\n" % (BIG, kc))
        os.environ["RBFIB_TUNING"] = str(p)
    yield write
    os.environ.pop("RBFIB_TUNING", None)


def _apply(rb, w, x_pad):
    import torch
    ctx = lib_context(rb, w, tol=1e-8)
    y = torch.empty(ctx.L, dtype=torch.float64, device="cuda")
    rb.rbfib_apply_saddle(ctx, dev(w.q), dev(w.theta), dev(x_pad), y)
    kc = rb.rbfib_launch_geometry(ctx)["apply_kc"]
    ctx.close()
    return y.cpu().numpy(), kc


@pytest.mark.parametrize("name", list(CONFIGS))
def test_z_apply_bit_identical(rb, table, name):
    w = CONFIGS[name]
    print("z apply", name, flush=True)
    s = Saddle(oracle_grid(w), w.q, w.theta, w.r_ref, w.offsets)
    x = np.random.default_rng(7).standard_normal(s.n)
    xp = oracle_to_padded(s, x)
    table(0)
    y0, kc = _apply(rb, w, xp)
    assert kc == 0
    yr = s.A @ x
    y = padded_to_oracle(s, y0)
    for sl in (s.sl_v, s.sl_p, s.sl_l, s.sl_u):
        assert np.abs(y[sl] - yr[sl]).max() <= 1e-10 * np.abs(yr[sl]).max()
    for kc in (1, 3, 8, 64):
        table(kc)
        yk, got = _apply(rb, w, xp)
        assert got == kc
        assert np.array_equal(yk, y0), (name, kc, np.abs(yk - y0).max())


def test_z_apply_solve_and_batch_identical(rb, table):
    """FP32-preconditioned solves (FP32 vectors into the apply) of a mixed batch:
    the same velocities bit for bit with and without the z-marching apply."""
    import torch
    reps = [W.spheres_in_box(101, (16, 16, 16), 1, name="r0"), W.spheres_in_box(102, (24, 24, 24), 3, name="r1"),
            W.spheres_in_box(104, (16, 16, 16), 4, R=1.5, shape="ico12", name="r3"),
            CONFIGS["periodic_wrap_17x12x12"]]
    cat = lambda k: dev(np.concatenate([getattr(r, k) for r in reps]))
    out = {}
    for kc in (0, 8):
        table(kc)
        ctx = lib_context(rb, reps, tol=1e-8, precond_fp32=1)
        assert rb.rbfib_launch_geometry(ctx)["apply_kc"] == kc
        U = torch.empty((sum(r.nb for r in reps), 6), dtype=torch.float64, device="cuda")
        info = rb.rbfib_solve_mobility(ctx, cat("q"), cat("theta"), cat("FT"), U, allow=())
        out[kc] = (U.cpu().numpy(), [i.iters for i in info])
        ctx.close()
    print("iters", out[0][1], out[8][1], flush=True)
    assert out[0][1] == out[8][1]
    assert np.array_equal(out[0][0], out[8][0])
