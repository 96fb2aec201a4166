"""The allocation-free apply against the context-based apply, through the C ABI.

rbfib_apply_saddle_noalloc keeps every table in the library's fixed device array
instead of a context's workspace and runs the same kernels, so on the same
configuration and state vector it returns what rbfib_apply_saddle returns (checked
to the FP64 apply bar, 1e-10 relative per block, and reported bit for bit), on two
calls in a row, the second with a smaller grid and fewer markers, so that state a
larger call leaves in the array cannot leak into a smaller one; and inputs beyond
its stated limits are refused before any work.
"""
import numpy as np
import pytest

import workloads as W
from oracle.saddle import Saddle
from tests.helpers import dev, lib_context, oracle_grid, oracle_to_padded, padded_to_oracle

pytestmark = pytest.mark.gpu


def _case(rb, w, seed):
    import torch
    g = oracle_grid(w)
    s = Saddle(g, w.q, w.theta, w.r_ref, w.offsets)
    x = np.random.default_rng(seed).standard_normal(s.n)
    xd = dev(oracle_to_padded(s, x))
    ctx = lib_context(rb, w)
    y_ctx = torch.full((ctx.L,), float("nan"), dtype=torch.float64, device="cuda")
    rb.rbfib_apply_saddle(ctx, dev(w.q), dev(w.theta), xd, y_ctx)
    torch.cuda.synchronize()
    ctx.close()
    y_na = torch.full_like(y_ctx, float("nan"))
    grid = rb.make_grid(w.n, w.bc, w.h, w.eta, w.wall_vel)
    rb.rbfib_apply_saddle_noalloc(grid, w.r_ref, w.offsets, dev(w.q), dev(w.theta), xd, y_na)
    torch.cuda.synchronize()
    a, b = y_na.cpu().numpy(), y_ctx.cpu().numpy()
    print("  bit-identical to rbfib_apply_saddle:", bool(np.array_equal(a, b)), flush=True)
    pa, pb, yr = padded_to_oracle(s, a), padded_to_oracle(s, b), s.A @ x
    for sl in (s.sl_v, s.sl_p, s.sl_l, s.sl_u):
        if sl.stop > sl.start:
            assert np.abs(pa[sl] - pb[sl]).max() <= 1e-10 * np.abs(pb[sl]).max()
            assert np.abs(pa[sl] - yr[sl]).max() <= 1e-10 * np.abs(yr[sl]).max()
    assert np.all(np.isfinite(a))


def test_noalloc_apply_matches_context_apply_twice():
    import paper_1901_06427_amd as rb
    big = W.small_box(22, n=(32, 24, 20), n_bodies=6, R=1.5, shape="ico12")
    big.bc = (W.PERIODIC, W.WALL, W.WALL)
    wv = np.zeros((3, 2, 3))
    wv[2, 0, 0] = 0.5
    big.wall_vel = wv
    small = W.small_box(21, n=(10, 12, 14), n_bodies=2, R=1.5, shape="ico12")
    for name, w, seed in (("32x24x20, 6 bodies", big, 1), ("10x12x14, 2 bodies", small, 2)):
        print("noalloc apply", name, flush=True)
        _case(rb, w, seed)


def test_noalloc_apply_rejects_beyond_limits():
    import torch
    import paper_1901_06427_amd as rb
    w = W.small_box(21, n=(10, 12, 14), n_bodies=2, R=1.5, shape="ico12")
    x = torch.zeros(4 * 10 * 12 * 14 + 3 * w.nm + 6 * w.nb, dtype=torch.float64, device="cuda")
    y = torch.empty_like(x)
    grid = rb.make_grid((512, 256, 128), w.bc)            # 2^24 cells: beyond 2^23
    with pytest.raises(rb.RBFIBError) as e:
        rb.rbfib_apply_saddle_noalloc(grid, w.r_ref, w.offsets, dev(w.q), dev(w.theta), x, y)
    assert e.value.code == rb.RBFIB_EINVAL
    many = np.tile(W.icosahedron(1.0), (700, 1))            # 8400 markers: beyond 8192
    offs = np.arange(0, 8401, 12, dtype=np.int32)
    grid = rb.make_grid((10, 12, 14), w.bc)
    with pytest.raises(rb.RBFIBError) as e:
        rb.rbfib_apply_saddle_noalloc(grid, many, offs, dev(np.zeros((700, 3))), dev(np.tile(w.theta[:1], (700, 1))),
                                      x, y)
    assert e.value.code == rb.RBFIB_EINVAL
