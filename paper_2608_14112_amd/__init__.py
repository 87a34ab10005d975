"""Python binding of libgve.so, the MI355X (gfx950) fixed-budget Gaussian volume encoder.

Argument marshalling only: every step of evaluation, binning, loss, gradient
and Adam runs in the HIP kernels of libgve.so (declared in include/gve.h).
torch tensors supply device memory and the HIP stream; they are passed to the
library as raw pointers.  Importing this module fails loudly if the library
has not been built (``python paper_2608_14112_amd/build.py``).

Names follow the C ABI without the ``gve_`` prefix:

    ctx = Context(k=3.0, brick=8, brick_z=32, lr=8e-3)
    p = Params(ctx, n)              # fixed budget n (paper Sec. III-A)
    p.upload(theta)                 # [11, n] float32 host array
    evaluate(ctx, p, grid, out)     # out: float32 cuda tensor [nz, ny, nx]
    L = loss_grad(ctx, p, field, grid, grad)
    losses = refine(ctx, p, field, grid, iters)
"""
from __future__ import annotations

import ctypes
import math
import os
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libgve.so")

if not os.path.exists(LIB_PATH):
    raise ImportError(
        f"{LIB_PATH} is missing: build it with `python paper_2608_14112_amd/build.py` "
        "(there is no fallback implementation)")

# torch first: its libraries load the HIP runtime it ships (soname
# libamdhip64.so.7), which libgve.so's dependency then resolves to.  Loaded the
# other way round, the system runtime comes first and torch still loads its own
# copy by path, leaving two HIP runtimes in the process (context creation then
# fails).
import torch  # noqa: E402,F401

_lib = ctypes.CDLL(LIB_PATH)

NPARAM = 11
PARAM_NAMES = ("mu_x", "mu_y", "mu_z", "q_w", "q_x", "q_y", "q_z", "l_x", "l_y", "l_z", "c")

STATUS = {0: "ok", 1: "invalid argument", 2: "budget infeasible", 3: "out of device memory",
          4: "device error", 5: "non-finite value", 6: "unsupported"}
OK, INVALID_ARGUMENT, BUDGET_INFEASIBLE, OUT_OF_MEMORY, DEVICE, NUMERIC, UNSUPPORTED = range(7)


class GveError(RuntimeError):
    def __init__(self, status, message):
        super().__init__(f"{STATUS.get(status, status)}: {message}")
        self.status = status
        self.message = message


class GridC(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int64), ("ny", ctypes.c_int64), ("nz", ctypes.c_int64),
                ("x0", ctypes.c_int64), ("y0", ctypes.c_int64), ("z0", ctypes.c_int64)]


class OptionsC(ctypes.Structure):
    _fields_ = [("k", ctypes.c_float), ("brick", ctypes.c_int32), ("lr", ctypes.c_float),
                ("beta1", ctypes.c_float), ("beta2", ctypes.c_float), ("eps", ctypes.c_float),
                ("ell_min", ctypes.c_float), ("ell_max", ctypes.c_float),
                ("brick_z", ctypes.c_int32), ("deterministic", ctypes.c_int32),
                ("schedule", ctypes.c_int32), ("brick_waves", ctypes.c_int32)]


class PaperOptionsC(ctypes.Structure):
    _fields_ = [(f, ctypes.c_float) for f in ("k", "rho0")] + [("samples", ctypes.c_int32)] + \
        [(f, ctypes.c_float) for f in ("frac_hi", "frac_mid", "v_hi", "v_occ", "lam_rho",
                                       "lam_sm_start", "lam_sm_end", "lam_anc", "lam_aniso",
                                       "lam_cap", "aniso_max", "ell_lo", "ell_hi", "lr", "beta1",
                                       "beta2", "eps", "cell")]


class TuneEntryC(ctypes.Structure):
    _fields_ = [("brick", ctypes.c_int32), ("brick_z", ctypes.c_int32),
                ("schedule", ctypes.c_int32), ("ms", ctypes.c_float), ("waves", ctypes.c_int32)]


SCHED_INDEX, SCHED_XCD, SCHED_QUEUE = 0, 1, 2


class StatsC(ctypes.Structure):
    _fields_ = [("n_primitives", ctypes.c_int64), ("n_bricks", ctypes.c_int64),
                ("n_overlaps", ctypes.c_int64), ("n_clamped", ctypes.c_int64),
                ("iterations", ctypes.c_int64), ("last_loss", ctypes.c_double),
                ("timed_iterations", ctypes.c_int64), ("ms_bin", ctypes.c_double),
                ("ms_fused", ctypes.c_double), ("ms_update", ctypes.c_double),
                ("workspace_bytes", ctypes.c_int64), ("n_in_support", ctypes.c_int64),
                ("n_candidates", ctypes.c_int64), ("n_atomics", ctypes.c_int64),
                ("n_nonfinite", ctypes.c_int64), ("n_resized", ctypes.c_int64),
                ("bin_brick", ctypes.c_int64), ("bin_brick_z", ctypes.c_int64),
                ("bin_schedule", ctypes.c_int64), ("n_degenerate_q", ctypes.c_int64),
                ("bin_waves", ctypes.c_int64)]


class ProbeC(ctypes.Structure):
    _fields_ = [("fma_flops_per_s", ctypes.c_double), ("exp_per_s", ctypes.c_double),
                ("copy_bytes_per_s", ctypes.c_double), ("atomic_instr_per_s", ctypes.c_double)]


class AllocInfoC(ctypes.Structure):
    _fields_ = [("n_detail", ctypes.c_int64), ("n_coverage", ctypes.c_int64),
                ("n_eligible", ctypes.c_int64), ("n_occupied", ctypes.c_int64),
                ("shortfall", ctypes.c_int64), ("s_base_detail", ctypes.c_double),
                ("s_base_coverage", ctypes.c_double), ("g99", ctypes.c_double),
                ("kappa", ctypes.c_double)]


_vp = ctypes.c_void_p
_i64 = ctypes.c_int64
_SIGS = {
    "gve_default_options": [ctypes.POINTER(OptionsC)],
    "gve_create": [ctypes.POINTER(_vp), ctypes.POINTER(OptionsC), _vp],
    "gve_destroy": [_vp],
    "gve_set_options": [_vp, ctypes.POINTER(OptionsC)],
    "gve_get_options": [_vp, ctypes.POINTER(OptionsC)],
    "gve_params_create": [_vp, _i64, ctypes.POINTER(_vp)],
    "gve_params_destroy": [_vp],
    "gve_params_size": [_vp, ctypes.POINTER(_i64)],
    "gve_params_upload": [_vp, _vp, _vp],
    "gve_params_download": [_vp, _vp, _vp],
    "gve_params_copy_from_device": [_vp, _vp, _vp],
    "gve_params_device": [_vp, ctypes.POINTER(_vp)],
    "gve_params_reset_adam": [_vp, _vp],
    "gve_params_adam_state": [_vp, ctypes.POINTER(_vp), ctypes.POINTER(_vp), ctypes.POINTER(_i64)],
    "gve_params_set_step": [_vp, _i64],
    "gve_evaluate": [_vp, _vp, GridC, _vp],
    "gve_loss_grad": [_vp, _vp, _vp, GridC, _vp, ctypes.POINTER(ctypes.c_double)],
    "gve_loss_grad_static": [_vp, _vp, _vp, GridC, _vp, ctypes.POINTER(ctypes.c_double)],
    "gve_dense_evaluate": [_vp, _vp, GridC, _vp],
    "gve_dense_loss_grad": [_vp, _vp, _vp, GridC, _vp, ctypes.POINTER(ctypes.c_double)],
    "gve_adam_step": [_vp, _vp, _vp],
    "gve_vjp": [_vp, _vp, _vp, GridC, _vp],
    "gve_export": [_vp, _vp, GridC, ctypes.c_float, ctypes.c_float, _vp, ctypes.c_size_t],
    "gve_import": [_vp, _vp, ctypes.c_size_t, ctypes.POINTER(_vp), ctypes.POINTER(GridC)],
    "gve_checkpoint_save": [_vp, _vp, ctypes.c_double, _vp, ctypes.c_size_t],
    "gve_checkpoint_load": [_vp, _vp, ctypes.c_size_t, ctypes.POINTER(_vp),
                            ctypes.POINTER(ctypes.c_double)],
    "gve_refine": [_vp, _vp, _vp, GridC, ctypes.c_int32, _vp],
    "gve_get_stats": [_vp, ctypes.POINTER(StatsC)],
    "gve_allocate": [_vp, _vp, GridC, _i64, ctypes.c_uint64, ctypes.POINTER(_vp),
                     ctypes.POINTER(AllocInfoC)],
    "gve_normalize": [_vp, _vp, _i64],
    "gve_set_timing": [_vp, ctypes.c_int32],
    "gve_mlp_create": [_vp, ctypes.c_uint64, ctypes.POINTER(_vp)],
    "gve_mlp_destroy": [_vp],
    "gve_mlp_export": [_vp, _vp, _vp],
    "gve_mlp_import": [_vp, _vp, _vp],
    "gve_mlp_forward": [_vp, _vp, _vp, _i64, _vp],
    "gve_mlp_loss_grad": [_vp, _vp, _vp, _vp, _i64, _vp, ctypes.POINTER(ctypes.c_double)],
    "gve_mlp_train": [_vp, _vp, _vp, _vp, _i64, ctypes.c_int32, ctypes.c_int32, ctypes.c_float,
                      ctypes.c_uint64, _vp],
    "gve_features": [_vp, _vp, _vp, GridC, _i64, ctypes.c_double, _vp],
    "gve_targets": [_vp, _vp, _vp, _vp],
    "gve_warmstart": [_vp, _vp, _vp, _vp, GridC, _i64, ctypes.c_double,
                      ctypes.POINTER(ctypes.c_int32), _vp],
    "gve_count_pairs": [_vp, _vp, GridC, ctypes.POINTER(_i64), ctypes.POINTER(_i64)],
    "gve_probe": [_vp, ctypes.POINTER(ProbeC)],
    "gve_bin_pairs": [_vp, _vp, GridC, _vp, _vp, _vp, _vp, _vp, _i64, ctypes.POINTER(_i64),
                      ctypes.POINTER(_i64)],
    "gve_batch_create": [_vp, ctypes.c_int32, _vp, _vp, ctypes.POINTER(_vp)],
    "gve_batch_params": [_vp, ctypes.POINTER(_vp)],
    "gve_batch_offsets": [_vp, _vp, _vp],
    "gve_batch_set_item": [_vp, _vp, ctypes.c_int32, _vp],
    "gve_batch_get_item": [_vp, _vp, ctypes.c_int32, _vp],
    "gve_batch_evaluate": [_vp, _vp, _vp],
    "gve_batch_loss_grad": [_vp, _vp, _vp, _vp, _vp],
    "gve_batch_refine": [_vp, _vp, _vp, ctypes.c_int32, _vp],
    "gve_batch_count_pairs": [_vp, _vp, ctypes.POINTER(_i64), ctypes.POINTER(_i64)],
    "gve_autotune": [_vp, _vp, _vp, GridC, _vp, ctypes.c_int32, _vp, ctypes.c_int32,
                     ctypes.POINTER(ctypes.c_int32)],
    "gve_paper_default_options": [ctypes.POINTER(PaperOptionsC)],
    "gve_paper_create": [_vp, _i64, ctypes.POINTER(_vp)],
    "gve_paper_upload": [_vp, _vp, _vp],
    "gve_paper_download": [_vp, _vp, _vp],
    "gve_paper_from_params": [_vp, _vp, _vp, ctypes.c_double, ctypes.c_float],
    "gve_paper_sample": [_vp, _vp, GridC, ctypes.POINTER(PaperOptionsC), ctypes.c_uint64, _i64,
                         _vp, _vp],
    "gve_paper_eval": [_vp, _vp, GridC, ctypes.POINTER(PaperOptionsC), _vp, _i64, _vp, _vp],
    "gve_paper_loss_grad": [_vp, _vp, _vp, GridC, ctypes.POINTER(PaperOptionsC), ctypes.c_float,
                            _vp, _vp, _i64, _vp, _vp, ctypes.POINTER(ctypes.c_double)],
    "gve_paper_refine": [_vp, _vp, _vp, GridC, ctypes.POINTER(PaperOptionsC), ctypes.c_uint64,
                         ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, _vp],
}
for _name, _args in _SIGS.items():
    _f = getattr(_lib, _name)
    _f.argtypes = _args
    _f.restype = ctypes.c_int
_lib.gve_status_string.argtypes = [ctypes.c_int]
_lib.gve_status_string.restype = ctypes.c_char_p
_lib.gve_last_error.argtypes = [_vp]
_lib.gve_last_error.restype = ctypes.c_char_p

for _name in ("gve_export_size", "gve_checkpoint_size"):
    getattr(_lib, _name).argtypes = [_i64]
    getattr(_lib, _name).restype = ctypes.c_size_t
_lib.gve_batch_destroy.argtypes = [_vp]
_lib.gve_batch_destroy.restype = None
_lib.gve_paper_destroy.argtypes = [_vp]
_lib.gve_paper_destroy.restype = None

EXPORTED = tuple(_SIGS) + ("gve_status_string", "gve_last_error", "gve_export_size",
                           "gve_checkpoint_size", "gve_batch_destroy", "gve_paper_destroy")
EXPORT_HEADER = 7000


def _check(status, ctx_handle=None):
    if status != OK:
        msg = _lib.gve_last_error(ctx_handle).decode() if ctx_handle else ""
        raise GveError(status, msg or _lib.gve_status_string(status).decode())


@dataclass(frozen=True)
class Grid:
    """Voxel grid: voxel (i, j, k) sits at (x0 + i, y0 + j, z0 + k); arrays [nz, ny, nx]."""

    nx: int
    ny: int
    nz: int
    x0: int = 0
    y0: int = 0
    z0: int = 0

    @property
    def shape(self):
        return (self.nz, self.ny, self.nx)

    def c(self):
        return GridC(self.nx, self.ny, self.nz, self.x0, self.y0, self.z0)


def _ptr(t, dtype=None, numel=None):
    """Device pointer of a contiguous cuda tensor (checked)."""
    import torch

    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError("expected a CUDA (HIP) torch tensor")
    if not t.is_contiguous():
        raise ValueError("tensor must be contiguous")
    if dtype is not None and t.dtype != dtype:
        raise TypeError(f"expected dtype {dtype}, got {t.dtype}")
    if numel is not None and t.numel() != numel:
        raise ValueError(f"expected {numel} elements, got {t.numel()}")
    return ctypes.c_void_p(t.data_ptr())


def default_options():
    o = OptionsC()
    _check(_lib.gve_default_options(ctypes.byref(o)))
    return o


class Context:
    """Owns a gve_ctx bound to a HIP stream (default: torch's current stream)."""

    def __init__(self, k=3.0, brick=8, lr=8e-3, beta1=0.9, beta2=0.999, eps=1e-8,
                 ell_min=-math.inf, ell_max=math.inf, brick_z=None, deterministic=False,
                 schedule=None, stream=None, brick_waves=1):
        import torch

        if brick_z is None:                       # library default shape 8 x 8 x 32
            brick_z = 32 if brick in (0, 8) else 0
        if schedule is None:
            schedule = default_options().schedule
        self._torch_stream = stream if stream is not None else torch.cuda.current_stream()
        o = OptionsC(k, brick, lr, beta1, beta2, eps, ell_min, ell_max, brick_z,
                     1 if deterministic else 0, schedule, brick_waves)
        h = _vp()
        st = _lib.gve_create(ctypes.byref(h), ctypes.byref(o),
                             _vp(self._torch_stream.cuda_stream))
        if st != OK:
            raise GveError(st, "gve_create failed")
        self.handle = h

    @property
    def options(self):
        o = OptionsC()
        _check(_lib.gve_get_options(self.handle, ctypes.byref(o)), self.handle)
        return o

    def set_options(self, **kw):
        o = self.options
        for key, val in kw.items():
            setattr(o, key, val)
        _check(_lib.gve_set_options(self.handle, ctypes.byref(o)), self.handle)

    def stats(self):
        s = StatsC()
        _check(_lib.gve_get_stats(self.handle, ctypes.byref(s)), self.handle)
        return {f: getattr(s, f) for f, _ in StatsC._fields_}

    def set_timing(self, enable=True):
        _check(_lib.gve_set_timing(self.handle, 1 if enable else 0), self.handle)

    def close(self):
        if getattr(self, "handle", None):
            _lib.gve_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Params:
    """A fixed-budget primitive set: device [11][n] parameters plus Adam state."""

    def __init__(self, ctx: Context, n: int, _handle=None, _owned=True):
        self.ctx = ctx
        self.n = int(n)
        self._owned = _owned
        if _handle is not None:
            self.handle = _handle
            return
        h = _vp()
        _check(_lib.gve_params_create(ctx.handle, _i64(self.n), ctypes.byref(h)), ctx.handle)
        self.handle = h

    def upload(self, theta):
        a = np.ascontiguousarray(np.asarray(theta, dtype=np.float32).reshape(NPARAM, self.n))
        _check(_lib.gve_params_upload(self.ctx.handle, self.handle, a.ctypes.data_as(_vp)),
               self.ctx.handle)
        return self

    def upload_device(self, theta):
        import torch

        _check(_lib.gve_params_copy_from_device(
            self.ctx.handle, self.handle, _ptr(theta, torch.float32, NPARAM * self.n)),
            self.ctx.handle)
        return self

    def download(self):
        a = np.empty((NPARAM, self.n), dtype=np.float32)
        _check(_lib.gve_params_download(self.ctx.handle, self.handle, a.ctypes.data_as(_vp)),
               self.ctx.handle)
        return a

    def device_ptr(self):
        d = _vp()
        _check(_lib.gve_params_device(self.handle, ctypes.byref(d)))
        return d.value

    def reset_adam(self):
        _check(_lib.gve_params_reset_adam(self.ctx.handle, self.handle), self.ctx.handle)

    @property
    def step(self):
        t = _i64()
        _check(_lib.gve_params_adam_state(self.handle, None, None, ctypes.byref(t)))
        return t.value

    @step.setter
    def step(self, t):
        _check(_lib.gve_params_set_step(self.handle, _i64(int(t))))

    def adam_state_ptrs(self):
        m, v, t = _vp(), _vp(), _i64()
        _check(_lib.gve_params_adam_state(self.handle, ctypes.byref(m), ctypes.byref(v),
                                          ctypes.byref(t)))
        return m.value, v.value, t.value

    def close(self):
        if getattr(self, "handle", None):
            if self._owned:
                _lib.gve_params_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def evaluate(ctx: Context, params: Params, grid: Grid, out=None):
    """gve_evaluate: truncated field on ``grid`` into ``out`` (float32 cuda [nz, ny, nx];
    allocated when not given)."""
    import torch

    if out is None:
        out = torch.empty(grid.shape, device="cuda", dtype=torch.float32)
    _check(_lib.gve_evaluate(ctx.handle, params.handle, grid.c(),
                             _ptr(out, torch.float32, grid.nx * grid.ny * grid.nz)), ctx.handle)
    return out


def loss_grad(ctx: Context, params: Params, field, grid: Grid, grad=None, want_loss=True):
    """gve_loss_grad: returns L (float) if want_loss; fills grad ([11, n] float32 cuda) if given."""
    import torch

    n = grid.nx * grid.ny * grid.nz
    gp = _ptr(grad, torch.float32, NPARAM * params.n) if grad is not None else None
    L = ctypes.c_double(0.0)
    _check(_lib.gve_loss_grad(ctx.handle, params.handle, _ptr(field, torch.float32, n), grid.c(),
                              gp, ctypes.byref(L) if want_loss else None), ctx.handle)
    return L.value if want_loss else None


def loss_grad_static(ctx: Context, params: Params, field, grid: Grid, grad=None, want_loss=True):
    """gve_loss_grad_static: gve_loss_grad with every work buffer taken from the
    library's fixed device array (no device allocation in the call)."""
    import torch

    n = grid.nx * grid.ny * grid.nz
    gp = _ptr(grad, torch.float32, NPARAM * params.n) if grad is not None else None
    L = ctypes.c_double(0.0)
    _check(_lib.gve_loss_grad_static(ctx.handle, params.handle, _ptr(field, torch.float32, n),
                                     grid.c(), gp, ctypes.byref(L) if want_loss else None),
           ctx.handle)
    return L.value if want_loss else None


def dense_evaluate(ctx: Context, params: Params, grid: Grid, out=None):
    """gve_dense_evaluate: the same truncated field with every (primitive, voxel) pair
    evaluated (no binning), into ``out`` (float32 cuda [nz, ny, nx]; allocated when not
    given)."""
    import torch

    if out is None:
        out = torch.empty(grid.shape, device="cuda", dtype=torch.float32)
    _check(_lib.gve_dense_evaluate(ctx.handle, params.handle, grid.c(),
                                   _ptr(out, torch.float32, grid.nx * grid.ny * grid.nz)),
           ctx.handle)
    return out


def dense_loss_grad(ctx: Context, params: Params, field, grid: Grid, grad=None, want_loss=True):
    """gve_dense_loss_grad: loss_grad with every (primitive, voxel) pair evaluated."""
    import torch

    n = grid.nx * grid.ny * grid.nz
    gp = _ptr(grad, torch.float32, NPARAM * params.n) if grad is not None else None
    L = ctypes.c_double(0.0)
    _check(_lib.gve_dense_loss_grad(ctx.handle, params.handle, _ptr(field, torch.float32, n),
                                    grid.c(), gp, ctypes.byref(L) if want_loss else None),
           ctx.handle)
    return L.value if want_loss else None


def vjp(ctx: Context, params: Params, upstream, grid: Grid, grad=None):
    """gve_vjp: sum_p upstream(p) dVhat(p)/dtheta as a [11, n] float32 cuda tensor."""
    import torch

    if grad is None:
        grad = torch.empty((NPARAM, params.n), device=upstream.device, dtype=torch.float32)
    _check(_lib.gve_vjp(ctx.handle, params.handle,
                        _ptr(upstream, torch.float32, grid.nx * grid.ny * grid.nz), grid.c(),
                        _ptr(grad, torch.float32, NPARAM * params.n)), ctx.handle)
    return grad


def adam_step(ctx: Context, params: Params, grad):
    """gve_adam_step: one Adam step from a caller gradient ([11, n] float32 cuda)."""
    import torch

    _check(_lib.gve_adam_step(ctx.handle, params.handle, _ptr(grad, torch.float32,
                                                               NPARAM * params.n)), ctx.handle)


def refine(ctx: Context, params: Params, field, grid: Grid, iters: int, want_losses=True):
    """gve_refine: ``iters`` fused iterations; returns the loss before each update."""
    import torch

    n = grid.nx * grid.ny * grid.nz
    hist = np.zeros(max(int(iters), 1), dtype=np.float64) if want_losses else None
    _check(_lib.gve_refine(ctx.handle, params.handle, _ptr(field, torch.float32, n), grid.c(),
                           ctypes.c_int32(int(iters)),
                           hist.ctypes.data_as(_vp) if want_losses else None), ctx.handle)
    return hist[:iters] if want_losses else None


class BudgetInfeasible(GveError):
    def __init__(self, info, message):
        super().__init__(BUDGET_INFEASIBLE, message)
        self.info = info
        self.shortfall = info["shortfall"]


def allocate(ctx: Context, field, grid: Grid, budget: int, seed: int):
    """gve_allocate: returns (Params, info dict); raises BudgetInfeasible (Sec. V-B)."""
    import torch

    n = grid.nx * grid.ny * grid.nz
    h = _vp()
    inf = AllocInfoC()
    st = _lib.gve_allocate(ctx.handle, _ptr(field, torch.float32, n), grid.c(), _i64(int(budget)),
                           ctypes.c_uint64(int(seed) & (2 ** 64 - 1)), ctypes.byref(h),
                           ctypes.byref(inf))
    info = {f: getattr(inf, f) for f, _ in AllocInfoC._fields_}
    if st == BUDGET_INFEASIBLE:
        raise BudgetInfeasible(info, _lib.gve_last_error(ctx.handle).decode())
    _check(st, ctx.handle)
    return Params(ctx, int(budget), _handle=h), info


def normalize(ctx: Context, field):
    """gve_normalize: min-max normalise a float32 cuda tensor to [0, 1] in place."""
    import torch

    _check(_lib.gve_normalize(ctx.handle, _ptr(field, torch.float32), _i64(field.numel())),
           ctx.handle)
    return field


def count_pairs(ctx: Context, params: Params, grid: Grid):
    """gve_count_pairs: (in-support pairs, candidate lane-voxel evaluations)."""
    a, b = _i64(), _i64()
    _check(_lib.gve_count_pairs(ctx.handle, params.handle, grid.c(), ctypes.byref(a),
                                ctypes.byref(b)), ctx.handle)
    return a.value, b.value


def probe(ctx: Context):
    """gve_probe: measured fp32 FMA, exponential, copy and atomic rates (dict)."""
    r = ProbeC()
    _check(_lib.gve_probe(ctx.handle, ctypes.byref(r)), ctx.handle)
    return {f: getattr(r, f) for f, _ in ProbeC._fields_}


MLP_NWEIGHT = 20107
MLP_NFLAT = MLP_NWEIGHT + 54
MLP_LAYOUT = (("W1", (128, 16)), ("b1", (128,)), ("W2", (128, 128)), ("b2", (128,)),
              ("W3", (11, 128)), ("b3", (11,)))


def bin_pairs(ctx: Context, params: Params, grid: Grid):
    """gve_bin_pairs: (emitted keys, emitted values, sorted keys, sorted values,
    brick starts) as uint32 numpy arrays."""
    import torch

    T = ctypes.c_int64()
    nb = ctypes.c_int64()
    _check(_lib.gve_bin_pairs(ctx.handle, params.handle, grid.c(), None, None, None, None, None,
                              _i64(0), ctypes.byref(T), ctypes.byref(nb)), ctx.handle)
    cap = max(int(T.value), 1)
    bufs = [torch.empty(cap, device="cuda", dtype=torch.int32) for _ in range(4)]
    start = torch.empty(int(nb.value) + 1, device="cuda", dtype=torch.int32)
    _check(_lib.gve_bin_pairs(ctx.handle, params.handle, grid.c(), *[_ptr(b) for b in bufs],
                              _ptr(start), _i64(cap), ctypes.byref(T), ctypes.byref(nb)),
           ctx.handle)
    n = int(T.value)
    out = [b[:n].cpu().numpy().view(np.uint32) for b in bufs]
    return (*out, start.cpu().numpy().view(np.uint32))


class MLP:
    """The warm-start network (gve_mlp): 16 -> 128 -> 128 -> 11, GELU."""

    def __init__(self, ctx: Context, seed: int = 0):
        self.ctx = ctx
        h = _vp()
        _check(_lib.gve_mlp_create(ctx.handle, ctypes.c_uint64(int(seed)), ctypes.byref(h)),
               ctx.handle)
        self.handle = h

    def export(self):
        """Flat float32 array: weights (MLP_LAYOUT order) then feature/target mean and std."""
        a = np.empty(MLP_NFLAT, dtype=np.float32)
        _check(_lib.gve_mlp_export(self.ctx.handle, self.handle, a.ctypes.data_as(_vp)),
               self.ctx.handle)
        return a

    def load(self, flat):
        a = np.ascontiguousarray(np.asarray(flat, dtype=np.float32).reshape(MLP_NFLAT))
        _check(_lib.gve_mlp_import(self.ctx.handle, self.handle, a.ctypes.data_as(_vp)),
               self.ctx.handle)

    def tensors(self):
        """Weights as a dict of float64 arrays plus the standardisation statistics."""
        a = self.export().astype(np.float64)
        out, off = {}, 0
        for name, shape in MLP_LAYOUT:
            size = int(np.prod(shape))
            out[name] = a[off:off + size].reshape(shape)
            off += size
        st = a[MLP_NWEIGHT:]
        out["fmean"], out["fstd"], out["tmean"], out["tstd"] = st[:16], st[16:32], st[32:43], st[43:]
        return out

    def close(self):
        if getattr(self, "handle", None):
            _lib.gve_mlp_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def mlp_forward(ctx: Context, mlp: MLP, X):
    """gve_mlp_forward on standardised X (float32 cuda [n, 16]) -> [n, 11]."""
    import torch

    n = X.shape[0]
    Y = torch.empty((n, 11), device=X.device, dtype=torch.float32)
    _check(_lib.gve_mlp_forward(ctx.handle, mlp.handle, _ptr(X, torch.float32, n * 16), _i64(n),
                                _ptr(Y)), ctx.handle)
    return Y


def mlp_loss_grad(ctx: Context, mlp: MLP, X, T):
    """gve_mlp_loss_grad: (loss, flat gradient [MLP_NWEIGHT] cuda tensor)."""
    import torch

    n = X.shape[0]
    g = torch.empty(MLP_NWEIGHT, device=X.device, dtype=torch.float32)
    L = ctypes.c_double()
    _check(_lib.gve_mlp_loss_grad(ctx.handle, mlp.handle, _ptr(X, torch.float32, n * 16),
                                  _ptr(T, torch.float32, n * 11), _i64(n), _ptr(g),
                                  ctypes.byref(L)), ctx.handle)
    return L.value, g


def mlp_train(ctx: Context, mlp: MLP, X, T, epochs, batch=4096, lr=1e-3, seed=0):
    """gve_mlp_train on raw features / targets; returns the per-epoch mean loss."""
    import torch

    n = X.shape[0]
    hist = np.zeros(max(int(epochs), 1))
    _check(_lib.gve_mlp_train(ctx.handle, mlp.handle, _ptr(X, torch.float32, n * 16),
                              _ptr(T, torch.float32, n * 11), _i64(n), ctypes.c_int32(int(epochs)),
                              ctypes.c_int32(int(batch)), ctypes.c_float(lr),
                              ctypes.c_uint64(int(seed)), hist.ctypes.data_as(_vp)), ctx.handle)
    return hist[:epochs]


def features(ctx: Context, params: Params, field, grid: Grid, n_detail: int, g99: float):
    """gve_features -> float32 cuda [n, 16]."""
    import torch

    X = torch.empty((params.n, 16), device=field.device, dtype=torch.float32)
    _check(_lib.gve_features(ctx.handle, params.handle,
                             _ptr(field, torch.float32, grid.nx * grid.ny * grid.nz), grid.c(),
                             _i64(int(n_detail)), ctypes.c_double(float(g99)), _ptr(X)), ctx.handle)
    return X


def targets(ctx: Context, alloc: Params, refined: Params, device="cuda"):
    """gve_targets -> float32 cuda [n, 11]."""
    import torch

    T = torch.empty((alloc.n, 11), device=device, dtype=torch.float32)
    _check(_lib.gve_targets(ctx.handle, alloc.handle, refined.handle, _ptr(T)), ctx.handle)
    return T


def warmstart(ctx: Context, mlp: MLP, params: Params, field, grid: Grid, n_detail: int,
              g99: float):
    """gve_warmstart: returns (applied, losses[4])."""
    import torch

    applied = ctypes.c_int32()
    L = np.zeros(4)
    _check(_lib.gve_warmstart(ctx.handle, mlp.handle, params.handle,
                              _ptr(field, torch.float32, grid.nx * grid.ny * grid.nz), grid.c(),
                              _i64(int(n_detail)), ctypes.c_double(float(g99)),
                              ctypes.byref(applied), L.ctypes.data_as(_vp)), ctx.handle)
    return applied.value, L


def export_bytes(ctx: Context, params: Params, grid: Grid, vmin=0.0, vmax=1.0) -> bytes:
    """gve_export: the 48-byte-per-primitive encoding with its fixed header."""
    size = _lib.gve_export_size(_i64(params.n))
    buf = ctypes.create_string_buffer(size)
    _check(_lib.gve_export(ctx.handle, params.handle, grid.c(), ctypes.c_float(vmin),
                           ctypes.c_float(vmax), ctypes.cast(buf, _vp), ctypes.c_size_t(size)),
           ctx.handle)
    return buf.raw


def import_bytes(ctx: Context, data: bytes):
    """gve_import: (Params, Grid) from an export."""
    h = _vp()
    gc = GridC()
    buf = ctypes.create_string_buffer(data, len(data))
    _check(_lib.gve_import(ctx.handle, ctypes.cast(buf, _vp), ctypes.c_size_t(len(data)),
                           ctypes.byref(h), ctypes.byref(gc)), ctx.handle)
    n = ctypes.c_int64()
    _check(_lib.gve_params_size(h, ctypes.byref(n)))
    return Params(ctx, n.value, _handle=h), Grid(gc.nx, gc.ny, gc.nz, gc.x0, gc.y0, gc.z0)


def checkpoint_bytes(ctx: Context, params: Params, elapsed_s=0.0) -> bytes:
    size = _lib.gve_checkpoint_size(_i64(params.n))
    buf = ctypes.create_string_buffer(size)
    _check(_lib.gve_checkpoint_save(ctx.handle, params.handle, ctypes.c_double(elapsed_s),
                                    ctypes.cast(buf, _vp), ctypes.c_size_t(size)), ctx.handle)
    return buf.raw


def checkpoint_load(ctx: Context, data: bytes):
    """(Params with Adam state and step, elapsed seconds) from a checkpoint."""
    h = _vp()
    el = ctypes.c_double()
    buf = ctypes.create_string_buffer(data, len(data))
    _check(_lib.gve_checkpoint_load(ctx.handle, ctypes.cast(buf, _vp), ctypes.c_size_t(len(data)),
                                    ctypes.byref(h), ctypes.byref(el)), ctx.handle)
    n = ctypes.c_int64()
    _check(_lib.gve_params_size(h, ctypes.byref(n)))
    return Params(ctx, n.value, _handle=h), el.value


class Batch:
    """gve_batch: many volumes binned and refined together.

    ``grids`` is a list of Grid, ``counts`` the primitives of each.  Fields and
    outputs are one concatenated float32 cuda buffer (``voxel_offsets``);
    parameters are one [11, sum(counts)] set (``prim_offsets``).
    """

    def __init__(self, ctx: Context, grids, counts):
        self.ctx = ctx
        self.grids = list(grids)
        n = len(self.grids)
        g = (GridC * n)(*[gr.c() for gr in self.grids])
        c = (ctypes.c_int64 * n)(*[int(x) for x in counts])
        h = _vp()
        _check(_lib.gve_batch_create(ctx.handle, ctypes.c_int32(n), ctypes.cast(g, _vp),
                                     ctypes.cast(c, _vp), ctypes.byref(h)), ctx.handle)
        self.handle = h
        po = np.zeros(n + 1, dtype=np.int64)
        vo = np.zeros(n + 1, dtype=np.int64)
        _check(_lib.gve_batch_offsets(h, po.ctypes.data_as(_vp), vo.ctypes.data_as(_vp)))
        self.prim_offsets, self.voxel_offsets = po, vo
        ph = _vp()
        _check(_lib.gve_batch_params(h, ctypes.byref(ph)))
        self.params = Params(ctx, int(po[-1]), _handle=ph, _owned=False)

    @property
    def n_items(self):
        return len(self.grids)

    def set_item(self, i, params: Params):
        _check(_lib.gve_batch_set_item(self.ctx.handle, self.handle, ctypes.c_int32(i),
                                       params.handle), self.ctx.handle)

    def get_item(self, i, params: Params):
        _check(_lib.gve_batch_get_item(self.ctx.handle, self.handle, ctypes.c_int32(i),
                                       params.handle), self.ctx.handle)
        return params

    def close(self):
        if getattr(self, "handle", None):
            self.params.handle = None
            _lib.gve_batch_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def batch_evaluate(ctx: Context, batch: Batch, out=None):
    import torch

    m = int(batch.voxel_offsets[-1])
    if out is None:
        out = torch.empty(m, device="cuda", dtype=torch.float32)
    _check(_lib.gve_batch_evaluate(ctx.handle, batch.handle, _ptr(out, torch.float32, m)),
           ctx.handle)
    return out


def batch_loss_grad(ctx: Context, batch: Batch, fields, grad=None):
    """Per-volume losses (numpy [n_items]); fills grad ([11, N] float32 cuda) if given."""
    import torch

    m = int(batch.voxel_offsets[-1])
    losses = np.zeros(batch.n_items, dtype=np.float64)
    gp = _ptr(grad, torch.float32, NPARAM * batch.params.n) if grad is not None else None
    _check(_lib.gve_batch_loss_grad(ctx.handle, batch.handle, _ptr(fields, torch.float32, m), gp,
                                    losses.ctypes.data_as(_vp)), ctx.handle)
    return losses


def batch_refine(ctx: Context, batch: Batch, fields, iters: int, want_losses=True):
    """Returns the per-volume loss before each update, [iters, n_items]."""
    import torch

    m = int(batch.voxel_offsets[-1])
    hist = np.zeros((max(int(iters), 1), batch.n_items), dtype=np.float64) if want_losses else None
    _check(_lib.gve_batch_refine(ctx.handle, batch.handle, _ptr(fields, torch.float32, m),
                                 ctypes.c_int32(int(iters)),
                                 hist.ctypes.data_as(_vp) if want_losses else None), ctx.handle)
    return hist[:iters] if want_losses else None


def batch_count_pairs(ctx: Context, batch: Batch):
    a, b = _i64(), _i64()
    _check(_lib.gve_batch_count_pairs(ctx.handle, batch.handle, ctypes.byref(a), ctypes.byref(b)),
           ctx.handle)
    return a.value, b.value


def autotune(ctx: Context, field, params: Params = None, grid: Grid = None, batch: Batch = None,
             reps=3):
    """gve_autotune: pick the fastest brick shape, waves per brick and schedule for
    this workload.

    Returns a list of (brick, brick_z, schedule, ms, waves) per candidate timed
    (empty when the context's cache already held the answer); the context keeps
    the choice.
    """
    import torch

    cap = 64
    table = (TuneEntryC * cap)()
    nw = ctypes.c_int32()
    if batch is not None:
        fp = _ptr(field, torch.float32, int(batch.voxel_offsets[-1]))
        st = _lib.gve_autotune(ctx.handle, None, fp, GridC(), batch.handle, ctypes.c_int32(reps),
                               ctypes.cast(table, _vp), cap, ctypes.byref(nw))
    else:
        fp = _ptr(field, torch.float32, grid.nx * grid.ny * grid.nz)
        st = _lib.gve_autotune(ctx.handle, params.handle, fp, grid.c(), None,
                               ctypes.c_int32(reps), ctypes.cast(table, _vp), cap,
                               ctypes.byref(nw))
    _check(st, ctx.handle)
    return [(e.brick, e.brick_z, e.schedule, e.ms, e.waves) for e in table[:nw.value]]


# ---- the paper's own training loop ------------------------------------------------------

PAPER_NPARAM = 12


def paper_options(**kw):
    """gve_paper_default_options with fields overridden by keyword."""
    o = PaperOptionsC()
    _check(_lib.gve_paper_default_options(ctypes.byref(o)))
    for key, val in kw.items():
        if not hasattr(o, key):
            raise AttributeError(key)
        setattr(o, key, val)
    return o


class PaperParams:
    """gve_paper: 12-row primitives (mu, q, ell, a, weight logit) plus Adam state."""

    def __init__(self, ctx: Context, n: int):
        self.ctx = ctx
        self.n = int(n)
        h = _vp()
        _check(_lib.gve_paper_create(ctx.handle, _i64(self.n), ctypes.byref(h)), ctx.handle)
        self.handle = h

    def upload(self, theta):
        a = np.ascontiguousarray(np.asarray(theta, dtype=np.float32).reshape(PAPER_NPARAM, self.n))
        _check(_lib.gve_paper_upload(self.ctx.handle, self.handle, a.ctypes.data_as(_vp)),
               self.ctx.handle)
        return self

    def download(self):
        a = np.empty((PAPER_NPARAM, self.n), dtype=np.float32)
        _check(_lib.gve_paper_download(self.ctx.handle, self.handle, a.ctypes.data_as(_vp)),
               self.ctx.handle)
        return a

    def from_params(self, params: Params, kappa, w0=0.1):
        _check(_lib.gve_paper_from_params(self.ctx.handle, self.handle, params.handle,
                                          ctypes.c_double(kappa), ctypes.c_float(w0)),
               self.ctx.handle)
        return self

    def close(self):
        if getattr(self, "handle", None):
            _lib.gve_paper_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def paper_sample(ctx: Context, field, grid: Grid, opts, seed, it):
    """(points [2S, 3] float32 cuda: samples then partners, values [S])."""
    import torch

    S = opts.samples
    pts = torch.empty((2 * S, 3), device="cuda", dtype=torch.float32)
    vals = torch.empty(S, device="cuda", dtype=torch.float32)
    _check(_lib.gve_paper_sample(ctx.handle, _ptr(field, torch.float32, grid.nx * grid.ny * grid.nz),
                                 grid.c(), ctypes.byref(opts), ctypes.c_uint64(int(seed)),
                                 _i64(int(it)), _ptr(pts), _ptr(vals)), ctx.handle)
    return pts, vals


def paper_eval(ctx: Context, params: PaperParams, grid: Grid, opts, pts):
    """(Vt, density) at points [npts, 3] (float32 cuda)."""
    import torch

    npts = pts.shape[0]
    vt = torch.empty(npts, device="cuda", dtype=torch.float32)
    den = torch.empty(npts, device="cuda", dtype=torch.float32)
    _check(_lib.gve_paper_eval(ctx.handle, params.handle, grid.c(), ctypes.byref(opts),
                               _ptr(pts, torch.float32, 3 * npts), _i64(npts), _ptr(vt),
                               _ptr(den)), ctx.handle)
    return vt, den


def paper_loss_grad(ctx: Context, params: PaperParams, field, grid: Grid, opts, lam_sm, pts, vals):
    """(objective, six terms, gradient [12, n] float32 cuda) at the given points."""
    import torch

    S = vals.shape[0]
    grad = torch.empty((PAPER_NPARAM, params.n), device="cuda", dtype=torch.float32)
    parts = np.zeros(6, dtype=np.float64)
    L = ctypes.c_double()
    _check(_lib.gve_paper_loss_grad(ctx.handle, params.handle,
                                    _ptr(field, torch.float32, grid.nx * grid.ny * grid.nz),
                                    grid.c(), ctypes.byref(opts), ctypes.c_float(lam_sm),
                                    _ptr(pts, torch.float32, 6 * S), _ptr(vals, torch.float32, S),
                                    _i64(S), _ptr(grad), parts.ctypes.data_as(_vp),
                                    ctypes.byref(L)), ctx.handle)
    return L.value, parts, grad


def paper_refine(ctx: Context, params: PaperParams, field, grid: Grid, opts, seed, iters,
                 first_iter=0, schedule_len=None):
    """Objective before each of ``iters`` iterations (numpy)."""
    import torch

    hist = np.zeros(max(int(iters), 1), dtype=np.float64)
    sched = int(schedule_len) if schedule_len else int(first_iter) + int(iters)
    _check(_lib.gve_paper_refine(ctx.handle, params.handle,
                                 _ptr(field, torch.float32, grid.nx * grid.ny * grid.nz),
                                 grid.c(), ctypes.byref(opts), ctypes.c_uint64(int(seed)),
                                 ctypes.c_int32(int(iters)), ctypes.c_int32(int(first_iter)),
                                 ctypes.c_int32(sched), hist.ctypes.data_as(_vp)), ctx.handle)
    return hist[:iters]
