"""Python binding of librbfib.so, the MI355X hot path of the RB-FIB method.

Argument marshalling only: every step of the computation runs in the HIP
library.  Functions carry the C names (``rbfib_create``, ``rbfib_apply_saddle``,
``rbfib_solve_mobility``, ``rbfib_sem_step``, ...) and take torch tensors that
live on the GPU (FP64, contiguous); PyTorch provides device memory and the
stream only.  Importing this module raises if the library has not been built
(``python paper_1901_06427_amd/build.py``): there is no CPU fallback.
"""
from __future__ import annotations

import ctypes
import os
from typing import List, Optional, Sequence

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIBPATH = os.path.join(HERE, "librbfib.so")

RBFIB_OK = 0
RBFIB_EINVAL = -1
RBFIB_EREJECT = -2
RBFIB_ENOCONV = -3
RBFIB_ENUMERIC = -4
RBFIB_EDEVICE = -5
RBFIB_ENOMEM = -6
PERIODIC = 0
WALL = 1
SLIP = 2

EXPORTS = [
    "rbfib_default_opts", "rbfib_strerror", "rbfib_last_error", "rbfib_create", "rbfib_create_batch",
    "rbfib_destroy", "rbfib_set_opts", "rbfib_state_size", "rbfib_layout", "rbfib_markers",
    "rbfib_apply_saddle", "rbfib_precondition", "rbfib_solve_mobility", "rbfib_fluctuating_stress",
    "rbfib_sem_step", "rbfib_mobility_vjp", "rbfib_kernel_stats", "rbfib_enable_timing",
    "rbfib_apply_saddle_noalloc", "rbfib_launch_geometry", "rbfib_body_forces",
    "rbfib_sem_rk2_predict", "rbfib_sem_rk2_correct", "rbfib_sem_ab2_step",
]


class rbfib_grid(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int * 3), ("bc", ctypes.c_int * 3), ("h", ctypes.c_double),
                ("eta", ctypes.c_double), ("wall_vel", ctypes.c_double * 18)]


class rbfib_potential(ctypes.Structure):
    _fields_ = [("phi0", ctypes.c_double), ("d", ctypes.c_double), ("b", ctypes.c_double),
                ("fconst", ctypes.c_double * 3)]


class rbfib_bodies(ctypes.Structure):
    _fields_ = [("nb", ctypes.c_int), ("nm", ctypes.c_int), ("marker_offset", ctypes.POINTER(ctypes.c_int)),
                ("r_ref", ctypes.POINTER(ctypes.c_double))]


class rbfib_opts(ctypes.Structure):
    _fields_ = [("tol", ctypes.c_double), ("restart", ctypes.c_int), ("max_iter", ctypes.c_int),
                ("precond_fp32", ctypes.c_int), ("mg_sweeps", ctypes.c_int), ("mg_sweeps_p", ctypes.c_int),
                ("mg_omega", ctypes.c_double),
                ("blob_radius", ctypes.c_double), ("rfd_delta", ctypes.c_double),
                ("min_body_dist", ctypes.c_double), ("check_every", ctypes.c_int), ("use_graphs", ctypes.c_int),
                ("mg_fused", ctypes.c_int), ("mg_bottom", ctypes.c_int),
                ("mg_cheby", ctypes.c_double), ("krylov_s", ctypes.c_int),
                ("mg_first2", ctypes.c_int), ("kernel", ctypes.c_int),
                ("no_drift", ctypes.c_int)]


class rbfib_info(ctypes.Structure):
    _fields_ = [("iters", ctypes.c_int), ("rel_residual", ctypes.c_double), ("status", ctypes.c_int)]


def _load():
    if not os.path.exists(LIBPATH):
        raise ImportError("librbfib.so is not built; run `python paper_1901_06427_amd/build.py` "
                          "(the RB-FIB hot path has no CPU fallback)")
    # PyTorch ships its own HIP runtime with the same soname; loading torch first
    # makes the library bind to that one runtime instead of a second copy.
    import torch  # noqa: F401
    lib = ctypes.CDLL(LIBPATH)
    P = ctypes.c_void_p
    I = ctypes.c_int
    D = ctypes.c_double
    U64 = ctypes.c_uint64
    sig = {
        "rbfib_default_opts": (None, [ctypes.POINTER(rbfib_opts)]),
        "rbfib_strerror": (ctypes.c_char_p, [I]),
        "rbfib_last_error": (ctypes.c_char_p, []),
        "rbfib_create": (I, [ctypes.POINTER(rbfib_grid), ctypes.POINTER(rbfib_bodies), ctypes.POINTER(rbfib_opts),
                             P, ctypes.POINTER(P)]),
        "rbfib_create_batch": (I, [I, ctypes.POINTER(rbfib_grid), ctypes.POINTER(rbfib_bodies),
                                   ctypes.POINTER(rbfib_opts), P, ctypes.POINTER(P)]),
        "rbfib_destroy": (None, [P]),
        "rbfib_set_opts": (I, [P, ctypes.POINTER(rbfib_opts)]),
        "rbfib_state_size": (ctypes.c_longlong, [P]),
        "rbfib_layout": (I, [P, ctypes.POINTER(ctypes.c_longlong)]),
        "rbfib_markers": (I, [P, P, P, P, P, P]),
        "rbfib_apply_saddle": (I, [P, P, P, P, P]),
        "rbfib_apply_saddle_noalloc": (I, [ctypes.POINTER(rbfib_grid), ctypes.POINTER(rbfib_bodies), P, P, P, P, P]),
        "rbfib_precondition": (I, [P, P, P, P, P]),
        "rbfib_solve_mobility": (I, [P, P, P, P, P, I, P, P, ctypes.POINTER(rbfib_info)]),
        "rbfib_fluctuating_stress": (I, [P, D, D, U64, U64, P]),
        "rbfib_sem_step": (I, [P, P, P, P, P, D, D, U64, U64, P, ctypes.POINTER(rbfib_info)]),
        "rbfib_mobility_vjp": (I, [P, P, P, P, P, P, P, P, P, ctypes.POINTER(rbfib_info)]),
        "rbfib_kernel_stats": (I, [P, I, ctypes.POINTER(D), ctypes.POINTER(D), ctypes.POINTER(ctypes.c_longlong)]),
        "rbfib_enable_timing": (I, [P, I]),
        "rbfib_launch_geometry": (I, [P, ctypes.POINTER(ctypes.c_int)]),
        "rbfib_body_forces": (I, [P, P, P, ctypes.POINTER(rbfib_potential), P]),
        "rbfib_sem_rk2_predict": (I, [P, P, P, P, P, D, D, D, U64, U64, P, P, ctypes.POINTER(rbfib_info)]),
        "rbfib_sem_rk2_correct": (I, [P, P, P, P, P, P, ctypes.POINTER(rbfib_info)]),
        "rbfib_sem_ab2_step": (I, [P, P, P, P, P, D, D, U64, U64, P, I, P, ctypes.POINTER(rbfib_info)]),
    }
    for name, (res, args) in sig.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    return lib


_lib = _load()


class RBFIBError(RuntimeError):
    def __init__(self, code: int, where: str):
        self.code = code
        msg = _lib.rbfib_strerror(code).decode()
        detail = _lib.rbfib_last_error().decode()
        super().__init__("%s failed: %s (%d)%s" % (where, msg, code, (" -- " + detail) if detail else ""))


def _check(code: int, where: str, allow=()):
    if code != RBFIB_OK and code not in allow:
        raise RBFIBError(code, where)
    return code


def _ptr(t) -> Optional[int]:
    if t is None:
        return None
    import torch
    if not (t.is_cuda and t.dtype == torch.float64 and t.is_contiguous()):
        raise ValueError("expected a contiguous float64 CUDA tensor")
    return t.data_ptr()


def _iptr(t) -> Optional[int]:
    if t is None:
        return None
    import torch
    if not (t.is_cuda and t.dtype == torch.int32 and t.is_contiguous()):
        raise ValueError("expected a contiguous int32 CUDA tensor")
    return t.data_ptr()


def rbfib_default_opts(**kw) -> rbfib_opts:
    o = rbfib_opts()
    _lib.rbfib_default_opts(ctypes.byref(o))
    for k, v in kw.items():
        setattr(o, k, v)
    return o


def make_grid(n, bc, h=1.0, eta=1.0, wall_vel=None) -> rbfib_grid:
    g = rbfib_grid()
    for a in range(3):
        g.n[a] = int(n[a])
        g.bc[a] = int(bc[a])
    g.h = float(h)
    g.eta = float(eta)
    wv = np.zeros(18) if wall_vel is None else np.asarray(wall_vel, dtype=np.float64).ravel()
    for i in range(18):
        g.wall_vel[i] = float(wv[i])
    return g


class Context:
    """Owns an rbfib_ctx (one replica or a batch) and the host copies it was built from."""

    def __init__(self, grids: Sequence[rbfib_grid], r_refs: Sequence[np.ndarray], offsets: Sequence[np.ndarray],
                 opts: Optional[rbfib_opts] = None, stream=None):
        import torch
        self.nrep = len(grids)
        self._keep = []
        garr = (rbfib_grid * self.nrep)(*grids)
        barr = (rbfib_bodies * self.nrep)()
        self.nb = 0
        self.nm = 0
        for r in range(self.nrep):
            rr = np.ascontiguousarray(r_refs[r], dtype=np.float64).reshape(-1, 3)
            off = np.ascontiguousarray(offsets[r], dtype=np.int32)
            self._keep += [rr, off]
            barr[r].nb = int(len(off) - 1)
            barr[r].nm = int(rr.shape[0])
            barr[r].marker_offset = off.ctypes.data_as(ctypes.POINTER(ctypes.c_int))
            barr[r].r_ref = rr.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
            self.nb += barr[r].nb
            self.nm += barr[r].nm
        self.opts = opts if opts is not None else rbfib_default_opts()
        if stream is None:
            stream = torch.cuda.current_stream().cuda_stream
        self.stream = stream
        h = ctypes.c_void_p()
        _check(_lib.rbfib_create_batch(self.nrep, garr, barr, ctypes.byref(self.opts), ctypes.c_void_p(stream),
                                       ctypes.byref(h)), "rbfib_create_batch")
        self.h = h
        self.L = int(_lib.rbfib_state_size(h))
        lay = (ctypes.c_longlong * (4 * self.nrep))()
        _check(_lib.rbfib_layout(h, lay), "rbfib_layout")
        self.layout = np.array(list(lay), dtype=np.int64).reshape(self.nrep, 4)

    def close(self):
        if getattr(self, "h", None):
            _lib.rbfib_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def rbfib_create(grid: rbfib_grid, r_ref, offsets, opts=None, stream=None) -> Context:
    return Context([grid], [r_ref], [offsets], opts, stream)


def rbfib_create_batch(grids, r_refs, offsets, opts=None, stream=None) -> Context:
    return Context(grids, r_refs, offsets, opts, stream)


def rbfib_destroy(ctx: Context):
    ctx.close()


def rbfib_set_opts(ctx: Context, opts: rbfib_opts):
    _check(_lib.rbfib_set_opts(ctx.h, ctypes.byref(opts)), "rbfib_set_opts")
    ctx.opts = opts


def rbfib_markers(ctx: Context, q, theta, r=None, tile=None, perm=None):
    _check(_lib.rbfib_markers(ctx.h, _ptr(q), _ptr(theta), _ptr(r), _iptr(tile), _iptr(perm)), "rbfib_markers")


def rbfib_apply_saddle(ctx: Context, q, theta, x, y):
    _check(_lib.rbfib_apply_saddle(ctx.h, _ptr(q), _ptr(theta), _ptr(x), _ptr(y)), "rbfib_apply_saddle")


def rbfib_apply_saddle_noalloc(grid: rbfib_grid, r_ref, offsets, q, theta, x, y, stream=None):
    """y = A x for one replica without a context (the library allocates nothing)."""
    import torch
    rr = np.ascontiguousarray(r_ref, dtype=np.float64).reshape(-1, 3)
    off = np.ascontiguousarray(offsets, dtype=np.int32)
    bd = rbfib_bodies()
    bd.nb = int(len(off) - 1)
    bd.nm = int(rr.shape[0])
    bd.marker_offset = off.ctypes.data_as(ctypes.POINTER(ctypes.c_int))
    bd.r_ref = rr.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    if stream is None:
        stream = torch.cuda.current_stream().cuda_stream
    _check(_lib.rbfib_apply_saddle_noalloc(ctypes.byref(grid), ctypes.byref(bd), _ptr(q), _ptr(theta), _ptr(x),
                                           _ptr(y), ctypes.c_void_p(stream)), "rbfib_apply_saddle_noalloc")


def rbfib_precondition(ctx: Context, q, theta, r, z):
    _check(_lib.rbfib_precondition(ctx.h, _ptr(q), _ptr(theta), _ptr(r), _ptr(z)), "rbfib_precondition")


def _infos(n):
    return (rbfib_info * n)()


def rbfib_solve_mobility(ctx: Context, q, theta, FT, U, slip=None, x_out=None, include_bc=True,
                         allow=(RBFIB_ENOCONV,)) -> List[rbfib_info]:
    info = _infos(ctx.nrep)
    code = _lib.rbfib_solve_mobility(ctx.h, _ptr(q), _ptr(theta), _ptr(FT), _ptr(slip), int(include_bc), _ptr(U),
                                     _ptr(x_out), info)
    _check(code, "rbfib_solve_mobility", allow)
    return list(info)


def rbfib_fluctuating_stress(ctx: Context, kT: float, dt: float, seed: int, step: int, f):
    _check(_lib.rbfib_fluctuating_stress(ctx.h, float(kT), float(dt), int(seed), int(step), _ptr(f)),
           "rbfib_fluctuating_stress")


def rbfib_sem_step(ctx: Context, q, theta, FT, kT: float, dt: float, seed: int, step: int, U, slip=None,
                   allow=(RBFIB_EREJECT, RBFIB_ENOCONV)) -> List[rbfib_info]:
    info = _infos(ctx.nrep)
    code = _lib.rbfib_sem_step(ctx.h, _ptr(q), _ptr(theta), _ptr(FT), _ptr(slip), float(kT), float(dt), int(seed),
                               int(step), _ptr(U), info)
    _check(code, "rbfib_sem_step", allow)
    return list(info)


def rbfib_body_forces(ctx: Context, q, theta, phi0: float, d: float, b: float, fconst, FT) -> None:
    """FT [nb, 6] = soft wall repulsion (eq. Usoft) plus a constant force per marker, summed per body."""
    pot = rbfib_potential(float(phi0), float(d), float(b), (ctypes.c_double * 3)(*[float(v) for v in fconst]))
    _check(_lib.rbfib_body_forces(ctx.h, _ptr(q), _ptr(theta), ctypes.byref(pot), _ptr(FT)), "rbfib_body_forces")


def rbfib_sem_rk2_predict(ctx: Context, q, theta, FT, kT: float, dt: float, seed: int, step: int, q_pred, theta_pred,
                          alpha: float = 1.0, slip=None, allow=(RBFIB_EREJECT, RBFIB_ENOCONV)) -> List[rbfib_info]:
    info = _infos(ctx.nrep)
    code = _lib.rbfib_sem_rk2_predict(ctx.h, _ptr(q), _ptr(theta), _ptr(FT), _ptr(slip), float(kT), float(dt),
                                      float(alpha), int(seed), int(step), _ptr(q_pred), _ptr(theta_pred), info)
    _check(code, "rbfib_sem_rk2_predict", allow)
    return list(info)


def rbfib_sem_rk2_correct(ctx: Context, q, theta, FT_pred, U=None, slip_pred=None,
                          allow=(RBFIB_EREJECT, RBFIB_ENOCONV)) -> List[rbfib_info]:
    info = _infos(ctx.nrep)
    code = _lib.rbfib_sem_rk2_correct(ctx.h, _ptr(q), _ptr(theta), _ptr(FT_pred), _ptr(slip_pred), _ptr(U), info)
    _check(code, "rbfib_sem_rk2_correct", allow)
    return list(info)


def rbfib_sem_ab2_step(ctx: Context, q, theta, FT, kT: float, dt: float, seed: int, step: int, U_det_prev,
                       have_prev: bool, U=None, slip=None, allow=(RBFIB_EREJECT, RBFIB_ENOCONV)) -> List[rbfib_info]:
    info = _infos(ctx.nrep)
    code = _lib.rbfib_sem_ab2_step(ctx.h, _ptr(q), _ptr(theta), _ptr(FT), _ptr(slip), float(kT), float(dt), int(seed),
                                   int(step), _ptr(U_det_prev), 1 if have_prev else 0, _ptr(U), info)
    _check(code, "rbfib_sem_ab2_step", allow)
    return list(info)


def rbfib_mobility_vjp(ctx: Context, q, theta, FT, Ubar, dFT, dq, dphi, dtheta=None,
                       allow=(RBFIB_ENOCONV,)) -> List[rbfib_info]:
    info = _infos(ctx.nrep)
    code = _lib.rbfib_mobility_vjp(ctx.h, _ptr(q), _ptr(theta), _ptr(FT), _ptr(Ubar), _ptr(dFT), _ptr(dq),
                                   _ptr(dphi), _ptr(dtheta), info)
    _check(code, "rbfib_mobility_vjp", allow)
    return list(info)


def _mobility_function():
    import torch

    class MobilitySolve(torch.autograd.Function):
        """U = N(q, theta) F through rbfib_solve_mobility; backward through
        rbfib_mobility_vjp (gradients for q, theta and F)."""

        @staticmethod
        def forward(fctx, lib_ctx, q, theta, FT):
            q, theta, FT = q.contiguous(), theta.contiguous(), FT.contiguous()
            U = torch.empty_like(FT)
            rbfib_solve_mobility(lib_ctx, q, theta, FT, U, include_bc=False, allow=())
            fctx.lib_ctx = lib_ctx
            fctx.save_for_backward(q, theta, FT)
            return U

        @staticmethod
        def backward(fctx, Ubar):
            q, theta, FT = fctx.saved_tensors
            dFT = torch.empty_like(FT)
            dq = torch.empty_like(q)
            dphi = torch.empty_like(q)
            dth = torch.empty_like(theta)
            rbfib_mobility_vjp(fctx.lib_ctx, q, theta, FT, Ubar.contiguous(), dFT, dq, dphi, dth, allow=())
            return None, dq, dth, dFT

    return MobilitySolve


_MOBILITY = None


def mobility_solve(ctx: Context, q, theta, FT):
    """Differentiable U = N(q, theta) F (torch.autograd.Function over the C ABI)."""
    global _MOBILITY
    if _MOBILITY is None:
        _MOBILITY = _mobility_function()
    return _MOBILITY.apply(ctx, q, theta, FT)


def rbfib_enable_timing(ctx: Context, on: bool = True):
    _check(_lib.rbfib_enable_timing(ctx.h, int(on)), "rbfib_enable_timing")


def rbfib_kernel_stats(ctx: Context, which: int):
    a = ctypes.c_double()
    b = ctypes.c_double()
    n = ctypes.c_longlong()
    _check(_lib.rbfib_kernel_stats(ctx.h, int(which), ctypes.byref(a), ctypes.byref(b), ctypes.byref(n)),
           "rbfib_kernel_stats")
    return a.value, b.value, n.value


def rbfib_launch_geometry(ctx: Context) -> dict:
    out = (ctypes.c_int * 5)()
    _check(_lib.rbfib_launch_geometry(ctx.h, out), "rbfib_launch_geometry")
    return {"krylov_chunk": out[0], "spread_grid": out[1], "spread_p": out[2], "mg_npt": out[3],
            "apply_kc": out[4]}


def library_path() -> str:
    return LIBPATH
