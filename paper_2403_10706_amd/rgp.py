"""Thin ctypes binding of librgp (argument marshalling only; every step runs in the HIP library).

Tensors are PyTorch device tensors used as plain device buffers; the current PyTorch stream is
passed to the library.  Names follow the C ABI in ``include/rgp.h``.  Loading fails loudly when
the library has not been built: there is no fallback.
"""
from __future__ import annotations

import ctypes
import dataclasses
import math
import os
from typing import Optional, Sequence, Tuple

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "librgp.so")

RGP_OK = 0
STATUS = {0: "ok", -1: "invalid argument", -2: "grid extents out of range",
          -3: "unsupported dtype combination", -4: "an input image holds a non-finite value",
          -5: "a level started outside the barrier", -6: "no Armijo trial step was accepted",
          -7: "HIP runtime error", -8: "workspace missing or too small"}
# Device-side failures of a correction, reported in stats[2] (never returned by a call).
ENONFINITE, EBARRIER, ELINESEARCH = -4, -5, -6
F64, F32, BF16 = 0, 1, 2
SOLVERS = {"gn": 0, "lbfgs": 1, "admm": 2}
OP_OT_INIT, OP_LOSS_GRAD, OP_GN_HVP, OP_PCG_SOLVE, OP_CORRECT, OP_APPLY_CORRECTION = range(6)
STAT_FIELDS = 12
STAT_HEADER = 4
STAT_NAMES = ("J", "D", "S", "P", "gnorm", "gq", "pcg_iters", "pcg_relres", "gamma", "trials",
              "accepted", "reserved")


class RGPError(RuntimeError):
    def __init__(self, fn: str, code: int, hip: int = 0):
        msg = f"{fn} failed: {STATUS.get(code, code)}"
        if code == -7:
            msg += f" (hip error {hip})"
        super().__init__(msg)
        self.code = code


class Grid(ctypes.Structure):
    _fields_ = [("m", ctypes.c_int64 * 3), ("pe", ctypes.c_int32), ("reserved", ctypes.c_int32),
                ("h", ctypes.c_double * 3)]


class SolverOpts(ctypes.Structure):
    _fields_ = [("alpha", ctypes.c_double), ("beta", ctypes.c_double),
                ("levels", ctypes.c_int32), ("gn_iters", ctypes.c_int32),
                ("pcg_iters", ctypes.c_int32), ("ls_max_trials", ctypes.c_int32),
                ("pcg_rtol", ctypes.c_double), ("armijo_c", ctypes.c_double),
                ("ot_eps", ctypes.c_double), ("ot_guard", ctypes.c_int32),
                ("use_b_init", ctypes.c_int32), ("ot_blur", ctypes.c_int32),
                ("solver", ctypes.c_int32), ("lbfgs_memory", ctypes.c_int32),
                ("batch_march", ctypes.c_int32), ("admm_rho0", ctypes.c_double)]


EXPORTS = ("rgp_status_string", "rgp_last_hip_error", "rgp_default_opts", "rgp_workspace_size",
           "rgp_ot_init", "rgp_loss_grad", "rgp_gn_hvp", "rgp_pcg_solve",
           "rgp_apply_correction", "rgp_correct", "rgp_correct_plan", "rgp_plan_launch",
           "rgp_plan_destroy", "rgp_timing_start", "rgp_timing_stop", "rgp_loss_grad_images",
           "rgp_batch_workspace_size", "rgp_correct_batch_plan", "rgp_autotune", "rgp_blur_field",
           "rgp_loss_grad_noalloc", "rgp_correct_batch", "rgp_correct_lsq", "rgp_restrict_image",
           "rgp_restrict_image_adjoint")

# rgp_kernel_kind
KERNEL_PCG_STEP, KERNEL_LOSS_GRAD, KERNEL_TRIAL, KERNEL_HVP, KERNEL_OT, KERNEL_SHIFT, \
    KERNEL_BLUR = range(7)
KERNEL_NAMES = ("pcg_step", "loss_grad", "trial", "hvp", "ot", "shift", "blur", "dht", "block_pcg",
                "lbfgs", "lsq")


class TimingRecord(ctypes.Structure):
    _fields_ = [("kernel", ctypes.c_int32), ("tag", ctypes.c_int32), ("grid", ctypes.c_uint32),
                ("pad", ctypes.c_uint32), ("cells", ctypes.c_int64), ("nodes", ctypes.c_int64),
                ("ms", ctypes.c_double)]

_lib = None


def load(path: str = LIB_PATH) -> ctypes.CDLL:
    """Load librgp.so (built in-tree by ``paper_2403_10706_amd.build``)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"librgp.so not found at {path}; build it with "
                           "`python -m paper_2403_10706_amd.build`")
    lib = ctypes.CDLL(path)
    vp, i32, f64, sz = ctypes.c_void_p, ctypes.c_int32, ctypes.c_double, ctypes.c_size_t
    gp = ctypes.POINTER(Grid)
    op = ctypes.POINTER(SolverOpts)
    lib.rgp_status_string.restype = ctypes.c_char_p
    lib.rgp_status_string.argtypes = [ctypes.c_int]
    lib.rgp_last_hip_error.restype = ctypes.c_int
    lib.rgp_default_opts.argtypes = [op]
    lib.rgp_default_opts.restype = None
    lib.rgp_workspace_size.argtypes = [ctypes.c_int, gp, ctypes.c_int, op, ctypes.POINTER(sz)]
    lib.rgp_ot_init.argtypes = [gp, ctypes.c_int, vp, vp, ctypes.c_int, vp, f64, i32, vp, vp, sz, vp]
    lib.rgp_loss_grad.argtypes = [gp, ctypes.c_int, vp, vp, ctypes.c_int, vp, f64, f64, vp, vp, vp,
                                  vp, vp, sz, vp]
    lib.rgp_loss_grad_noalloc.argtypes = [gp, ctypes.c_int, vp, vp, ctypes.c_int, vp, f64, f64,
                                          vp, vp, vp, vp, vp]
    lib.rgp_gn_hvp.argtypes = [gp, ctypes.c_int, vp, vp, f64, vp, vp, vp, vp, sz, vp]
    lib.rgp_pcg_solve.argtypes = [gp, ctypes.c_int, vp, vp, f64, vp, vp, i32, f64, vp, vp, vp, sz,
                                  vp]
    lib.rgp_apply_correction.argtypes = [gp, ctypes.c_int, vp, vp, ctypes.c_int, vp, vp, vp, vp]
    lib.rgp_correct.argtypes = [gp, ctypes.c_int, vp, vp, ctypes.c_int, op, vp, vp, vp, vp, vp, vp,
                                sz, vp]
    lib.rgp_correct_plan.argtypes = [gp, ctypes.c_int, vp, vp, ctypes.c_int, op, vp, vp, vp, vp,
                                     vp, vp, sz, vp, ctypes.POINTER(ctypes.c_void_p)]
    lib.rgp_plan_launch.argtypes = [vp, vp]
    lib.rgp_plan_destroy.argtypes = [vp]
    lib.rgp_timing_start.argtypes = [i32]
    lib.rgp_loss_grad_images.argtypes = [gp, ctypes.c_int, vp, vp, ctypes.c_int, vp, vp, vp, vp]
    lib.rgp_batch_workspace_size.argtypes = [i32, gp, ctypes.c_int, op, ctypes.POINTER(sz)]
    lib.rgp_autotune.argtypes = [gp, ctypes.c_int, op, vp, sz, vp, ctypes.POINTER(i32)]
    lib.rgp_correct_batch_plan.argtypes = [i32, gp, ctypes.c_int, vp, vp, ctypes.c_int, op, vp, vp,
                                           vp, vp, vp, sz, vp, ctypes.POINTER(ctypes.c_void_p)]
    lib.rgp_correct_batch.argtypes = [i32, gp, ctypes.c_int, vp, vp, ctypes.c_int, op, vp, vp, vp,
                                      vp, vp, sz, vp]
    lib.rgp_correct_lsq.argtypes = [gp, ctypes.c_int, vp, vp, ctypes.c_int, vp, i32, f64, vp, vp,
                                    vp]
    lib.rgp_timing_stop.argtypes = [ctypes.POINTER(TimingRecord), i32, ctypes.POINTER(i32)]
    lib.rgp_blur_field.argtypes = [gp, ctypes.c_int, vp, vp, vp]
    lib.rgp_restrict_image.argtypes = [gp, ctypes.c_int, vp, ctypes.c_int, vp, vp]
    lib.rgp_restrict_image_adjoint.argtypes = [gp, ctypes.c_int, vp, vp, i32, vp]
    for name in ("rgp_restrict_image", "rgp_restrict_image_adjoint", "rgp_blur_field", "rgp_ot_init", "rgp_loss_grad", "rgp_gn_hvp", "rgp_pcg_solve",
                 "rgp_apply_correction", "rgp_correct", "rgp_workspace_size", "rgp_correct_plan",
                 "rgp_loss_grad_noalloc", "rgp_correct_batch", "rgp_correct_lsq",
                 "rgp_plan_launch", "rgp_plan_destroy", "rgp_timing_start", "rgp_timing_stop",
                 "rgp_loss_grad_images", "rgp_batch_workspace_size", "rgp_correct_batch_plan",
                 "rgp_autotune"):
        getattr(lib, name).restype = ctypes.c_int
    _lib = lib
    return lib


def _check(fn: str, code: int):
    if code != RGP_OK:
        raise RGPError(fn, code, load().rgp_last_hip_error())


_DT = {torch.float64: F64, torch.float32: F32, torch.bfloat16: BF16}


def dtype_code(t: torch.dtype) -> int:
    if t not in _DT:
        raise TypeError(f"unsupported dtype {t}")
    return _DT[t]


def make_grid(shape: Sequence[int], pe: int, h: Sequence[float] = (1.0, 1.0, 1.0)) -> Grid:
    g = Grid()
    for d in range(3):
        g.m[d] = int(shape[d])
        g.h[d] = float(h[d])
    g.pe = int(pe)
    return g


def field_shape(shape: Sequence[int], pe: int) -> Tuple[int, int, int]:
    s = [int(x) for x in shape]
    s[pe] += 1
    return tuple(s)


def _stream_ptr(stream) -> ctypes.c_void_p:
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


def _ptr(t: Optional[torch.Tensor]):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _dev_check(*ts):
    for t in ts:
        if t is not None:
            if not t.is_cuda:
                raise ValueError("librgp works on device tensors only")
            if not t.is_contiguous():
                raise ValueError("tensors must be C-contiguous")


def workspace_size(op: int, shape, pe, h, real_dtype, opts: Optional[SolverOpts] = None) -> int:
    n = ctypes.c_size_t(0)
    g = make_grid(shape, pe, h)
    _check("rgp_workspace_size", load().rgp_workspace_size(
        op, ctypes.byref(g), dtype_code(real_dtype), None if opts is None else ctypes.byref(opts),
        ctypes.byref(n)))
    return int(n.value)


class Workspace:
    """Device workspace cache: one buffer per (device, stream), grown on demand.  Calls that
    share a workspace must not overlap, so calls on different streams get different buffers; a
    buffer is allocated on, and only ever used from, its own stream."""

    def __init__(self):
        self._buf = {}

    def get(self, nbytes: int, device, stream=None) -> torch.Tensor:
        dev = torch.device(device)
        if stream is None:
            stream = torch.cuda.current_stream(dev)
        key = (dev, int(stream.cuda_stream))
        buf = self._buf.get(key)
        if buf is None or buf.numel() < nbytes:
            # zero-filled once, as the library asks of a new workspace; allocated while `stream`
            # is current, so torch's allocator orders its reuse after that stream's work
            with torch.cuda.stream(stream):
                buf = torch.zeros(max(int(nbytes), 256), dtype=torch.uint8, device=dev)
            self._buf[key] = buf
        return buf


_WS = Workspace()


def _ws(op, shape, pe, h, real_dtype, device, opts=None, ws=None, stream=None):
    need = workspace_size(op, shape, pe, h, real_dtype, opts)
    if ws is None:
        ws = _WS.get(need, device, stream)
    if ws.numel() < need:
        raise ValueError(f"workspace too small ({ws.numel()} < {need} bytes)")
    return ws, need


def ot_init(I_plus: torch.Tensor, I_minus: torch.Tensor, pe: int, h=(1.0, 1.0, 1.0), *,
            real_dtype=None, eps: float = 1e-3, guard: bool = True, out=None, ws=None, stream=None):
    """Column-wise 1D OT initial field (see rgp_ot_init).  Returns (b0, n_guarded device tensor)."""
    _dev_check(I_plus, I_minus)
    real_dtype = real_dtype or (torch.float64 if I_plus.dtype == torch.float64 else torch.float32)
    shape = tuple(I_plus.shape)
    if out is None:
        out = torch.empty(field_shape(shape, pe), dtype=real_dtype, device=I_plus.device)
    ng = torch.zeros(1, dtype=torch.int64, device=I_plus.device)
    wsb, need = _ws(OP_OT_INIT, shape, pe, h, real_dtype, I_plus.device, ws=ws, stream=stream)
    g = make_grid(shape, pe, h)
    _check("rgp_ot_init", load().rgp_ot_init(
        ctypes.byref(g), dtype_code(I_plus.dtype), _ptr(I_plus), _ptr(I_minus),
        dtype_code(real_dtype), _ptr(out), float(eps), int(bool(guard)), _ptr(ng), _ptr(wsb),
        wsb.numel(), _stream_ptr(stream)))
    return out, ng


def blur_field(b: torch.Tensor, shape, pe: int, *, out=None, stream=None):
    """Optional 3x3x3 Gaussian blur (sigma 1 voxel, periodic) of a field on the grid of image
    shape `shape` (see rgp_blur_field).  Returns the blurred field (a new tensor unless `out`)."""
    _dev_check(b)
    if tuple(b.shape) != field_shape(tuple(shape), pe):
        raise ValueError(f"field shape {tuple(b.shape)} != {field_shape(tuple(shape), pe)}")
    if out is None:
        out = torch.empty_like(b)
    g = make_grid(tuple(shape), pe)
    _check("rgp_blur_field", load().rgp_blur_field(ctypes.byref(g), dtype_code(b.dtype), _ptr(b),
                                                   _ptr(out), _stream_ptr(stream)))
    return out


def loss_grad(I_plus, I_minus, b, pe, h=(1.0, 1.0, 1.0), alpha=300.0, beta=1e-4, *,
              want_grad=True, want_hess=True, ws=None, stream=None):
    """Objective (device tensor [J, D, S, P] in FP64), gradient and banded GN Hessian."""
    _dev_check(I_plus, I_minus, b)
    shape = tuple(I_plus.shape)
    if tuple(b.shape) != field_shape(shape, pe):
        raise ValueError(f"field shape {tuple(b.shape)} != {field_shape(shape, pe)}")
    dev = b.device
    jdsp = torch.empty(4, dtype=torch.float64, device=dev)
    grad = torch.empty_like(b) if want_grad else None
    hd = torch.empty_like(b) if want_hess else None
    ho = torch.empty_like(b) if want_hess else None
    wsb, _ = _ws(OP_LOSS_GRAD, shape, pe, h, b.dtype, dev, ws=ws, stream=stream)
    g = make_grid(shape, pe, h)
    _check("rgp_loss_grad", load().rgp_loss_grad(
        ctypes.byref(g), dtype_code(I_plus.dtype), _ptr(I_plus), _ptr(I_minus),
        dtype_code(b.dtype), _ptr(b), float(alpha), float(beta), _ptr(jdsp), _ptr(grad), _ptr(hd),
        _ptr(ho), _ptr(wsb), wsb.numel(), _stream_ptr(stream)))
    return jdsp, grad, hd, ho


def loss_grad_noalloc(I_plus, I_minus, b, pe, h=(1.0, 1.0, 1.0), alpha=300.0, beta=1e-4, *,
                      jdsp=None, grad=None, hdiag=None, hoff=None, stream=None):
    """rgp_loss_grad_noalloc into caller-given outputs (any of them None): no workspace, and
    nothing is allocated here when every wanted output is given.  Returns (jdsp, grad, hdiag,
    hoff) as passed."""
    _dev_check(I_plus, I_minus, b)
    shape = tuple(I_plus.shape)
    if tuple(b.shape) != field_shape(shape, pe):
        raise ValueError(f"field shape {tuple(b.shape)} != {field_shape(shape, pe)}")
    g = make_grid(shape, pe, h)
    _check("rgp_loss_grad_noalloc", load().rgp_loss_grad_noalloc(
        ctypes.byref(g), dtype_code(I_plus.dtype), _ptr(I_plus), _ptr(I_minus),
        dtype_code(b.dtype), _ptr(b), float(alpha), float(beta), _ptr(jdsp), _ptr(grad),
        _ptr(hdiag), _ptr(hoff), _stream_ptr(stream)))
    return jdsp, grad, hdiag, hoff


def gn_hvp(hdiag, hoff, v, shape, pe, h=(1.0, 1.0, 1.0), alpha=300.0, *, ws=None, stream=None):
    """H_J v and v^T H_J v (device FP64 scalar tensor)."""
    _dev_check(hdiag, hoff, v)
    Hv = torch.empty_like(v)
    vhv = torch.empty(1, dtype=torch.float64, device=v.device)
    wsb, _ = _ws(OP_GN_HVP, shape, pe, h, v.dtype, v.device, ws=ws, stream=stream)
    g = make_grid(shape, pe, h)
    _check("rgp_gn_hvp", load().rgp_gn_hvp(
        ctypes.byref(g), dtype_code(v.dtype), _ptr(hdiag), _ptr(hoff), float(alpha), _ptr(v),
        _ptr(Hv), _ptr(vhv), _ptr(wsb), wsb.numel(), _stream_ptr(stream)))
    return Hv, vhv


def loss_grad_images(I_plus, I_minus, b, pe, h=(1.0, 1.0, 1.0), *, stream=None):
    """(dJ/dI+, dJ/dI-) as cell arrays of b's dtype (rgp_loss_grad_images)."""
    _dev_check(I_plus, I_minus, b)
    gp = torch.empty(tuple(I_plus.shape), dtype=b.dtype, device=b.device)
    gm = torch.empty_like(gp)
    g = make_grid(tuple(I_plus.shape), pe, h)
    _check("rgp_loss_grad_images", load().rgp_loss_grad_images(
        ctypes.byref(g), dtype_code(I_plus.dtype), _ptr(I_plus), _ptr(I_minus),
        dtype_code(b.dtype), _ptr(b), _ptr(gp), _ptr(gm), _stream_ptr(stream)))
    return gp, gm


def coarse_shape(shape: Sequence[int]) -> Tuple[int, int, int]:
    """Cell shape of the next coarser pyramid level: ceil(m / 2) per axis."""
    return tuple((int(m) + 1) // 2 for m in shape)


def restrict_image(I, real_dtype=None, *, stream=None):
    """The image on the next coarser pyramid level (rgp_restrict_image): means of 2x2x2 blocks,
    in real_dtype (default: the image's dtype, FP32 for BF16 images)."""
    _dev_check(I)
    if real_dtype is None:
        real_dtype = torch.float32 if I.dtype == torch.bfloat16 else I.dtype
    out = torch.empty(coarse_shape(I.shape), dtype=real_dtype, device=I.device)
    g = make_grid(tuple(I.shape), 0)
    _check("rgp_restrict_image", load().rgp_restrict_image(
        ctypes.byref(g), dtype_code(I.dtype), _ptr(I), dtype_code(real_dtype), _ptr(out),
        _stream_ptr(stream)))
    return out


def restrict_image_adjoint(g_coarse, fine_shape, *, out=None, accumulate=False, stream=None):
    """R^T g_coarse in the fine shape (rgp_restrict_image_adjoint); with `accumulate` it is added
    to `out`, which then must be given."""
    if accumulate and out is None:
        raise ValueError("accumulate needs out")
    fine_shape = tuple(int(m) for m in fine_shape)
    if tuple(g_coarse.shape) != coarse_shape(fine_shape):
        raise ValueError("g_coarse does not have the coarse shape of fine_shape")
    if out is None:
        out = torch.empty(fine_shape, dtype=g_coarse.dtype, device=g_coarse.device)
    elif tuple(out.shape) != fine_shape or out.dtype != g_coarse.dtype:
        raise ValueError("out must have the fine shape and g_coarse's dtype")
    _dev_check(g_coarse, out)
    g = make_grid(fine_shape, 0)
    _check("rgp_restrict_image_adjoint", load().rgp_restrict_image_adjoint(
        ctypes.byref(g), dtype_code(g_coarse.dtype), _ptr(g_coarse), _ptr(out),
        1 if accumulate else 0, _stream_ptr(stream)))
    return out


def pcg_solve(hdiag, hoff, rhs, shape, pe, h=(1.0, 1.0, 1.0), alpha=300.0, *, maxit=10,
              rtol=0.1, ws=None, stream=None):
    """Jacobi-PCG on H_J x = rhs.  Returns (x, iters int32 device, relres FP64 device)."""
    _dev_check(hdiag, hoff, rhs)
    x = torch.empty_like(rhs)
    it = torch.zeros(1, dtype=torch.int32, device=rhs.device)
    rr = torch.zeros(1, dtype=torch.float64, device=rhs.device)
    wsb, _ = _ws(OP_PCG_SOLVE, shape, pe, h, rhs.dtype, rhs.device, ws=ws, stream=stream)
    g = make_grid(shape, pe, h)
    _check("rgp_pcg_solve", load().rgp_pcg_solve(
        ctypes.byref(g), dtype_code(rhs.dtype), _ptr(hdiag), _ptr(hoff), float(alpha), _ptr(rhs),
        _ptr(x), int(maxit), float(rtol), _ptr(it), _ptr(rr), _ptr(wsb), wsb.numel(),
        _stream_ptr(stream)))
    return x, it, rr


def correct_lsq(I_plus, I_minus, b, pe, h=(1.0, 1.0, 1.0), *, maxit=30, rtol=1e-6,
                want_iters=True, stream=None):
    """Least-squares corrected image (rgp_correct_lsq) in the images' dtype, and the CGLS
    iterations per column (int32 device tensor of the two cross-axis extents) or None."""
    _dev_check(I_plus, I_minus, b)
    shape = tuple(I_plus.shape)
    out = torch.empty_like(I_plus)
    cross = tuple(n for d, n in enumerate(shape) if d != pe)
    it = torch.empty(cross, dtype=torch.int32, device=b.device) if want_iters else None
    g = make_grid(shape, pe, h)
    _check("rgp_correct_lsq", load().rgp_correct_lsq(
        ctypes.byref(g), dtype_code(I_plus.dtype), _ptr(I_plus), _ptr(I_minus),
        dtype_code(b.dtype), _ptr(b), int(maxit), float(rtol), _ptr(out), _ptr(it),
        _stream_ptr(stream)))
    return out, it


def apply_correction(I_plus, I_minus, b, pe, h=(1.0, 1.0, 1.0), *, stream=None):
    """Jacobian-modulation corrected pair (T+, T-) in the image dtype."""
    _dev_check(I_plus, I_minus, b)
    Tp = torch.empty_like(I_plus)
    Tm = torch.empty_like(I_minus)
    g = make_grid(tuple(I_plus.shape), pe, h)
    _check("rgp_apply_correction", load().rgp_apply_correction(
        ctypes.byref(g), dtype_code(I_plus.dtype), _ptr(I_plus), _ptr(I_minus),
        dtype_code(b.dtype), _ptr(b), _ptr(Tp), _ptr(Tm), _stream_ptr(stream)))
    return Tp, Tm


@dataclasses.dataclass
class Options:
    """Solver options (defaults: the paper's alpha, beta, PCG 10 iterations / rtol 0.1)."""

    alpha: float = 300.0
    beta: float = 1e-4
    levels: int = 1
    gn_iters: int = 5
    pcg_iters: int = 10
    ls_max_trials: int = 10
    pcg_rtol: float = 0.1
    armijo_c: float = 1e-4
    ot_eps: float = 1e-3
    ot_guard: bool = True
    ot_blur: bool = False
    solver: str = "gn"          # "gn" (Gauss-Newton-PCG), "lbfgs" or "admm"
    lbfgs_memory: int = 10
    admm_rho0: float = 0.0      # <= 0: alpha
    batch_march: int = 0        # batched plans: minimum PCG march length (0: the solo plans')

    def to_c(self, use_b_init: bool = False) -> SolverOpts:
        o = SolverOpts()
        o.alpha, o.beta = float(self.alpha), float(self.beta)
        o.levels, o.gn_iters, o.pcg_iters = int(self.levels), int(self.gn_iters), int(self.pcg_iters)
        o.ls_max_trials = int(self.ls_max_trials)
        o.pcg_rtol, o.armijo_c, o.ot_eps = float(self.pcg_rtol), float(self.armijo_c), float(self.ot_eps)
        o.ot_guard = int(bool(self.ot_guard))
        o.use_b_init = int(bool(use_b_init))
        o.ot_blur = int(bool(self.ot_blur))
        o.solver = SOLVERS[self.solver]
        o.lbfgs_memory = int(self.lbfgs_memory)
        o.admm_rho0 = float(self.admm_rho0)
        o.batch_march = int(self.batch_march)
        return o


def coarsest_shape(shape, levels):
    s = tuple(int(x) for x in shape)
    for _ in range(levels - 1):
        s = tuple((x + 1) // 2 for x in s)
    return s


def correct(I_plus, I_minus, pe, h=(1.0, 1.0, 1.0), opts: Optional[Options] = None, *,
            real_dtype=None, b_init=None, want_images=True, want_stats=True, out=None, ws=None,
            stream=None):
    """The whole hot path (rgp_correct).  Returns dict(b, T_plus, T_minus, stats)."""
    _dev_check(I_plus, I_minus, b_init)
    opts = opts or Options()
    real_dtype = real_dtype or (torch.float64 if I_plus.dtype == torch.float64 else torch.float32)
    shape = tuple(I_plus.shape)
    dev = I_plus.device
    copts = opts.to_c(use_b_init=b_init is not None)
    b = out if out is not None else torch.empty(field_shape(shape, pe), dtype=real_dtype, device=dev)
    Tp = torch.empty_like(I_plus) if want_images else None
    Tm = torch.empty_like(I_minus) if want_images else None
    stats = (torch.empty(STAT_HEADER + opts.levels * opts.gn_iters * STAT_FIELDS,
                         dtype=torch.float64, device=dev) if want_stats else None)
    wsb, _ = _ws(OP_CORRECT, shape, pe, h, real_dtype, dev, opts=copts, ws=ws, stream=stream)
    g = make_grid(shape, pe, h)
    _check("rgp_correct", load().rgp_correct(
        ctypes.byref(g), dtype_code(I_plus.dtype), _ptr(I_plus), _ptr(I_minus),
        dtype_code(real_dtype), ctypes.byref(copts), _ptr(b_init), _ptr(b), _ptr(Tp), _ptr(Tm),
        _ptr(stats), _ptr(wsb), wsb.numel(), _stream_ptr(stream)))
    return dict(b=b, T_plus=Tp, T_minus=Tm, stats=stats)


def parse_stats(stats: torch.Tensor, levels: int, gn_iters: int):
    """Host view of a stats buffer: (header dict, list of per-level lists of record dicts)."""
    s = stats.detach().double().cpu().numpy()
    head = dict(ot_guarded=int(s[0]) if math.isfinite(s[0]) else -1, ot_shift=float(s[1]),
                status=int(s[2]) if math.isfinite(s[2]) else 0)
    recs = s[STAT_HEADER:].reshape(levels, gn_iters, STAT_FIELDS)
    out = []
    for lv in range(levels):
        out.append([dict(zip(STAT_NAMES, map(float, recs[lv, it]))) for it in range(gn_iters)])
    return head, out


# ---------------------------------------------------------------------------------------------
# Allocation-free variants for timed loops: every output and the (zero-filled) workspace are
# passed in; nothing is checked beyond what the library itself validates.
# ---------------------------------------------------------------------------------------------

def correct_into(I_plus, I_minus, pe, opts: Options, b_out, T_plus, T_minus, ws, *, h=(1.0, 1.0, 1.0),
                 stats=None, b_init=None, stream=None):
    g = make_grid(tuple(I_plus.shape), pe, h)
    copts = opts.to_c(use_b_init=b_init is not None)
    _check("rgp_correct", load().rgp_correct(
        ctypes.byref(g), dtype_code(I_plus.dtype), _ptr(I_plus), _ptr(I_minus),
        dtype_code(b_out.dtype), ctypes.byref(copts), _ptr(b_init), _ptr(b_out), _ptr(T_plus),
        _ptr(T_minus), _ptr(stats), _ptr(ws), ws.numel(), _stream_ptr(stream)))


def loss_grad_into(I_plus, I_minus, b, pe, jdsp, grad, hdiag, hoff, ws, *, h=(1.0, 1.0, 1.0),
                   alpha=300.0, beta=1e-4, stream=None):
    g = make_grid(tuple(I_plus.shape), pe, h)
    _check("rgp_loss_grad", load().rgp_loss_grad(
        ctypes.byref(g), dtype_code(I_plus.dtype), _ptr(I_plus), _ptr(I_minus),
        dtype_code(b.dtype), _ptr(b), float(alpha), float(beta), _ptr(jdsp), _ptr(grad),
        _ptr(hdiag), _ptr(hoff), _ptr(ws), ws.numel(), _stream_ptr(stream)))


def gn_hvp_into(hdiag, hoff, v, Hv, vHv, shape, pe, ws, *, h=(1.0, 1.0, 1.0), alpha=300.0,
                stream=None):
    g = make_grid(shape, pe, h)
    _check("rgp_gn_hvp", load().rgp_gn_hvp(
        ctypes.byref(g), dtype_code(v.dtype), _ptr(hdiag), _ptr(hoff), float(alpha), _ptr(v),
        _ptr(Hv), _ptr(vHv), _ptr(ws), ws.numel(), _stream_ptr(stream)))


def pcg_solve_into(hdiag, hoff, rhs, x, shape, pe, maxit, ws, *, rtol=0.0, h=(1.0, 1.0, 1.0),
                   alpha=300.0, iters=None, relres=None, stream=None):
    g = make_grid(shape, pe, h)
    _check("rgp_pcg_solve", load().rgp_pcg_solve(
        ctypes.byref(g), dtype_code(rhs.dtype), _ptr(hdiag), _ptr(hoff), float(alpha), _ptr(rhs),
        _ptr(x), int(maxit), float(rtol), _ptr(iters), _ptr(relres), _ptr(ws), ws.numel(),
        _stream_ptr(stream)))


def ot_init_into(I_plus, I_minus, pe, b0, ws, *, h=(1.0, 1.0, 1.0), eps=1e-3, guard=True,
                 n_guarded=None, stream=None):
    g = make_grid(tuple(I_plus.shape), pe, h)
    _check("rgp_ot_init", load().rgp_ot_init(
        ctypes.byref(g), dtype_code(I_plus.dtype), _ptr(I_plus), _ptr(I_minus),
        dtype_code(b0.dtype), _ptr(b0), float(eps), int(bool(guard)), _ptr(n_guarded), _ptr(ws),
        ws.numel(), _stream_ptr(stream)))


class Plan:
    """A whole correction captured once into a HIP graph (rgp_correct_plan) and replayed with one
    launch per call.  Capture needs a non-default stream; the tensors passed here must stay alive
    for the plan's lifetime (the plan keeps references)."""

    def __init__(self, I_plus, I_minus, pe, opts: Options, b_out, T_plus, T_minus, ws, *,
                 h=(1.0, 1.0, 1.0), stats=None, b_init=None, stream):
        _dev_check(I_plus, I_minus, b_out, T_plus, T_minus, stats, b_init)
        self._keep = (I_plus, I_minus, b_out, T_plus, T_minus, ws, stats, b_init)
        self._grid = make_grid(tuple(I_plus.shape), pe, h)
        self._opts = opts.to_c(use_b_init=b_init is not None)
        self._handle = ctypes.c_void_p(None)
        self.stream = stream
        _check("rgp_correct_plan", load().rgp_correct_plan(
            ctypes.byref(self._grid), dtype_code(I_plus.dtype), _ptr(I_plus), _ptr(I_minus),
            dtype_code(b_out.dtype), ctypes.byref(self._opts), _ptr(b_init), _ptr(b_out),
            _ptr(T_plus), _ptr(T_minus), _ptr(stats), _ptr(ws), ws.numel(),
            _stream_ptr(stream), ctypes.byref(self._handle)))

    def launch(self, stream=None):
        _check("rgp_plan_launch", load().rgp_plan_launch(self._handle,
                                                         _stream_ptr(stream or self.stream)))

    def close(self):
        if self._handle:
            _check("rgp_plan_destroy", load().rgp_plan_destroy(self._handle))
            self._handle = ctypes.c_void_p(None)

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _ptr_array(ts):
    if ts is None:
        return None
    arr = (ctypes.c_void_p * len(ts))(*[t.data_ptr() for t in ts])
    return ctypes.cast(arr, ctypes.c_void_p), arr


def batch_workspace_size(shapes, pes, real_dtype, opts: "Options", hs=None) -> int:
    n = len(shapes)
    hs = hs or [(1.0, 1.0, 1.0)] * n
    grids = (Grid * n)(*[make_grid(tuple(sh), pe, h) for sh, pe, h in zip(shapes, pes, hs)])
    c = opts.to_c()
    out = ctypes.c_size_t(0)
    _check("rgp_batch_workspace_size", load().rgp_batch_workspace_size(
        n, grids, dtype_code(real_dtype), ctypes.byref(c), ctypes.byref(out)))
    return out.value


class BatchPlan:
    """n pairs of their own shapes and PE axes corrected by one captured graph in which every
    Gauss-Newton kernel is one launch over all pairs (rgp_correct_batch_plan).  Allocates the
    outputs (b, and the corrected images when want_images) and the workspace; `launch` replays."""

    def __init__(self, I_plus, I_minus, pes, opts: "Options", *, hs=None,
                 real_dtype=torch.float32, want_images=True, want_stats=False, stream):
        n = len(I_plus)
        assert len(I_minus) == n and len(pes) == n and n >= 1
        _dev_check(*I_plus, *I_minus)
        dev = I_plus[0].device
        hs = hs or [(1.0, 1.0, 1.0)] * n
        shapes = [tuple(t.shape) for t in I_plus]
        self.n = n
        self.pes = list(pes)
        self._grids = (Grid * n)(*[make_grid(sh, pe, h) for sh, pe, h in zip(shapes, pes, hs)])
        self._opts = opts.to_c()
        nbytes = batch_workspace_size(shapes, pes, real_dtype, opts, hs)
        self.ws = torch.zeros(nbytes, dtype=torch.uint8, device=dev)
        self.b = [torch.empty(field_shape(sh, pe), dtype=real_dtype, device=dev)
                  for sh, pe in zip(shapes, pes)]
        self.T_plus = [torch.empty_like(t) for t in I_plus] if want_images else None
        self.T_minus = [torch.empty_like(t) for t in I_minus] if want_images else None
        self.stats = ([torch.empty(STAT_HEADER + opts.levels * opts.gn_iters * STAT_FIELDS,
                                   dtype=torch.float64, device=dev) for _ in range(n)]
                      if want_stats else None)
        self._keep = (list(I_plus), list(I_minus))
        arrs = [_ptr_array(x) for x in (I_plus, I_minus, self.b, self.T_plus, self.T_minus,
                                        self.stats)]
        self._arrs = arrs
        vp = [a[0] if a is not None else None for a in arrs]
        self.stream = stream
        self._handle = ctypes.c_void_p(None)
        torch.cuda.synchronize()
        _check("rgp_correct_batch_plan", load().rgp_correct_batch_plan(
            n, self._grids, dtype_code(I_plus[0].dtype), vp[0], vp[1], dtype_code(real_dtype),
            ctypes.byref(self._opts), vp[2], vp[3], vp[4], vp[5], _ptr(self.ws), self.ws.numel(),
            _stream_ptr(stream), ctypes.byref(self._handle)))

    def run_eager(self, stream=None):
        """The same correction enqueued directly (rgp_correct_batch), without the graph."""
        vp = [a[0] if a is not None else None for a in self._arrs]
        _check("rgp_correct_batch", load().rgp_correct_batch(
            self.n, self._grids, dtype_code(self._keep[0][0].dtype), vp[0], vp[1],
            dtype_code(self.b[0].dtype), ctypes.byref(self._opts), vp[2], vp[3], vp[4], vp[5],
            _ptr(self.ws), self.ws.numel(), _stream_ptr(stream or self.stream)))

    def launch(self, stream=None):
        _check("rgp_plan_launch", load().rgp_plan_launch(self._handle,
                                                         _stream_ptr(stream or self.stream)))

    def close(self):
        if self._handle:
            _check("rgp_plan_destroy", load().rgp_plan_destroy(self._handle))
            self._handle = ctypes.c_void_p(None)

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def autotune(shape, pe, real_dtype, opts: "Options", *, h=(1.0, 1.0, 1.0), ws=None,
             stream=None):
    """Tune the PCG march of every pyramid level (rgp_autotune); returns the chosen XL per level."""
    g = make_grid(tuple(shape), pe, h)
    c = opts.to_c()
    dev = torch.device("cuda", torch.cuda.current_device())
    wsb, _ = _ws(OP_CORRECT, tuple(shape), pe, h, real_dtype, dev, opts=c, ws=ws, stream=stream)
    out = (ctypes.c_int32 * opts.levels)()
    _check("rgp_autotune", load().rgp_autotune(ctypes.byref(g), dtype_code(real_dtype),
                                               ctypes.byref(c), _ptr(wsb), wsb.numel(),
                                               _stream_ptr(stream), out))
    return list(out)


def timing_start(capacity: int = 65536):
    """Start recording the duration of every eager hot-kernel launch (rgp_timing_start)."""
    _check("rgp_timing_start", load().rgp_timing_start(int(capacity)))


def timing_stop(max_records: int = 65536):
    """Stop recording; returns one dict per timed launch (kernel, tag, grid, cells, nodes, ms)."""
    recs = (TimingRecord * max_records)()
    n = ctypes.c_int32(0)
    _check("rgp_timing_stop", load().rgp_timing_stop(recs, int(max_records), ctypes.byref(n)))
    return [dict(kernel=KERNEL_NAMES[r.kernel], tag=r.tag, grid=r.grid, cells=r.cells,
                 nodes=r.nodes, ms=r.ms) for r in recs[:n.value]]
