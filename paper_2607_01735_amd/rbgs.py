"""Thin ctypes binding of librbgs.so (include/rbgs.h).

Argument marshalling only: every step of the method runs in the library's
HIP kernels.  Tensors are torch CUDA (HIP) tensors in the natural layout, a
2-D view of shape (n+2, m) with m >= n+2, unit column stride and row stride
ld >= n+2; the ring holds the Dirichlet data.  Streams default to torch's
current stream; workspaces are allocated through torch unless given.

If the shared library is missing this module raises ImportError: there is
no CPU or PyTorch fallback.
"""
import ctypes
import os

# torch first: its bundled HIP runtime and librbgs.so's must be one and the
# same library in the process (same SONAME; the first one loaded is shared).
import torch  # noqa: F401

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "librbgs.so")

if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is missing: build it with "
                      "`python -c 'import __graft_entry__ as g; g.build()'`")

_lib = ctypes.CDLL(LIB_PATH)

OK, EINVAL, EHIP, ENOCONV, ETIMEOUT, ENONFINITE, EUNSUPPORTED, EWORKSPACE, EORDER = \
    0, -1, -2, -3, -4, -5, -6, -8, -9
F64, F32 = 0, 1
KERNEL_AUTO, KERNEL_PLAIN, KERNEL_BLOCKED, KERNEL_RESIDENT = 0, 1, 2, 3
PREC_F64, PREC_F32_IR, PREC_BF16RHS_IR = 0, 1, 2

_KERNELS = {"auto": KERNEL_AUTO, "plain": KERNEL_PLAIN, "blocked": KERNEL_BLOCKED,
            "resident": KERNEL_RESIDENT}
_PRECISIONS = {"f64": PREC_F64, "f32_ir": PREC_F32_IR, "bf16rhs_ir": PREC_BF16RHS_IR}


class rbgs_grid(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32), ("ld", ctypes.c_int64), ("h", ctypes.c_double)]


class rbgs_timing(ctypes.Structure):
    _fields_ = [("pack_ms", ctypes.c_float), ("sweep_ms", ctypes.c_float),
                ("unpack_ms", ctypes.c_float), ("sweep_launches", ctypes.c_int32),
                ("persistent_ms", ctypes.c_float), ("persistent_launches", ctypes.c_int32),
                ("passes", ctypes.c_int32), ("fuse", ctypes.c_int32)]


def _timing_dict(t):
    return {name: getattr(t, name) for name, _ in rbgs_timing._fields_}


class rbgs_sweep_opts(ctypes.Structure):
    _fields_ = [("kernel", ctypes.c_int32), ("fuse", ctypes.c_int32),
                ("tile_rows", ctypes.c_int32), ("tile_cols", ctypes.c_int32),
                ("rows_per_block", ctypes.c_int32), ("debug_delay", ctypes.c_int32),
                ("debug_spin_limit", ctypes.c_int32), ("debug_stall_tile", ctypes.c_int32),
                ("timing", ctypes.POINTER(rbgs_timing)), ("lds_max_n", ctypes.c_int32),
                ("debug_tile_order", ctypes.c_int32), ("debug_seed", ctypes.c_uint32),
                ("debug_stamp_check", ctypes.c_int32), ("debug_trace_items", ctypes.c_int32),
                ("debug_trace", ctypes.c_void_p)]


class rbgs_solve_opts(ctypes.Structure):
    _fields_ = [("max_sweeps", ctypes.c_int32), ("rel_tol", ctypes.c_double),
                ("check_every", ctypes.c_int32), ("precision", ctypes.c_int32),
                ("inner_sweeps", ctypes.c_int32), ("omega", ctypes.c_double),
                ("sweep", rbgs_sweep_opts), ("fallback", ctypes.c_int32)]


class rbgs_solve_info(ctypes.Structure):
    _fields_ = [("sweeps", ctypes.c_int32), ("outer_iters", ctypes.c_int32),
                ("rel_residual", ctypes.c_double), ("abs_residual", ctypes.c_double),
                ("status", ctypes.c_int32), ("precision", ctypes.c_int32)]


class rbgs_mg_opts(ctypes.Structure):
    _fields_ = [("max_cycles", ctypes.c_int32), ("rel_tol", ctypes.c_double),
                ("pre_sweeps", ctypes.c_int32), ("post_sweeps", ctypes.c_int32),
                ("max_levels", ctypes.c_int32), ("coarse_sweeps", ctypes.c_int32),
                ("sweep", rbgs_sweep_opts)]


class rbgs_mg_info(ctypes.Structure):
    _fields_ = [("cycles", ctypes.c_int32), ("levels", ctypes.c_int32),
                ("coarsest_n", ctypes.c_int32), ("coarse_sweeps", ctypes.c_int32),
                ("rel_residual", ctypes.c_double), ("abs_residual", ctypes.c_double),
                ("graph", ctypes.c_int32), ("status", ctypes.c_int32)]


_P = ctypes.POINTER
_vp = ctypes.c_void_p
_lib.rbgs_mg_workspace_size.argtypes = [_P(rbgs_grid), ctypes.c_int, _P(rbgs_mg_opts)]
_lib.rbgs_mg_workspace_size.restype = ctypes.c_size_t
_lib.rbgs_mg_solve.argtypes = [_P(rbgs_grid), ctypes.c_int, _vp, _vp, _P(rbgs_mg_opts),
                               _P(rbgs_mg_info), _vp, ctypes.c_size_t, _vp]
_lib.rbgs_mg_solve.restype = ctypes.c_int
_lib.rbgs_mc9_workspace_size.argtypes = [_P(rbgs_grid)]
_lib.rbgs_mc9_workspace_size.restype = ctypes.c_size_t
_lib.rbgs_mc9_sweep.argtypes = [_P(rbgs_grid), _vp, _vp, ctypes.c_int32, ctypes.c_int32, _vp,
                                ctypes.c_size_t, _vp]
_lib.rbgs_mc9_sweep.restype = ctypes.c_int
_lib.rbgs_mc9_residual.argtypes = [_P(rbgs_grid), _vp, _vp, _P(ctypes.c_double),
                                   _P(ctypes.c_double), _vp, ctypes.c_size_t, _vp]
_lib.rbgs_mc9_residual.restype = ctypes.c_int
_lib.rbgs_mc9_solve.argtypes = [_P(rbgs_grid), _vp, _vp, ctypes.c_int32, ctypes.c_double,
                                ctypes.c_int32, ctypes.c_int32, _P(rbgs_solve_info), _vp,
                                ctypes.c_size_t, _vp]
_lib.rbgs_mc9_solve.restype = ctypes.c_int
_lib.rbgs_split_pitch.argtypes = [_P(rbgs_grid), ctypes.c_int]
_lib.rbgs_split_pitch.restype = ctypes.c_int64
_lib.rbgs_pack.argtypes = [_P(rbgs_grid), ctypes.c_int, _vp, _vp, _vp, _vp]
_lib.rbgs_pack.restype = ctypes.c_int
_lib.rbgs_unpack.argtypes = [_P(rbgs_grid), ctypes.c_int, _vp, _vp, _vp, _vp]
_lib.rbgs_unpack.restype = ctypes.c_int
_lib.rbgs_sweep_split.argtypes = [_P(rbgs_grid), ctypes.c_int, _vp, _vp, _vp, _vp, ctypes.c_int32,
                                  _P(rbgs_sweep_opts), _vp, ctypes.c_size_t, _vp]
_lib.rbgs_sweep_split.restype = ctypes.c_int
_lib.rbgs_rb3_workspace_size.argtypes = [_P(rbgs_grid)]
_lib.rbgs_rb3_workspace_size.restype = ctypes.c_size_t
_lib.rbgs_rb3_sweep.argtypes = [_P(rbgs_grid), _vp, _vp, ctypes.c_int32, _vp, ctypes.c_size_t, _vp]
_lib.rbgs_rb3_sweep.restype = ctypes.c_int
_lib.rbgs_rb3_residual.argtypes = [_P(rbgs_grid), _vp, _vp, _P(ctypes.c_double),
                                   _P(ctypes.c_double), _vp, ctypes.c_size_t, _vp]
_lib.rbgs_rb3_residual.restype = ctypes.c_int
_lib.rbgs_rb3_solve.argtypes = [_P(rbgs_grid), _vp, _vp, ctypes.c_int32, ctypes.c_double,
                                ctypes.c_int32, _P(rbgs_solve_info), _vp, ctypes.c_size_t, _vp]
_lib.rbgs_rb3_solve.restype = ctypes.c_int


class rbgs_rb3_opts(ctypes.Structure):
    _fields_ = [("kernel", ctypes.c_int32), ("debug_delay", ctypes.c_int32),
                ("debug_spin_limit", ctypes.c_int32), ("debug_stall_block", ctypes.c_int32)]


_lib.rbgs_rb3_sweep_ex.argtypes = [_P(rbgs_grid), _vp, _vp, ctypes.c_int32, _P(rbgs_rb3_opts), _vp,
                                   ctypes.c_size_t, _vp]
_lib.rbgs_rb3_sweep_ex.restype = ctypes.c_int
_lib.rbgs_rb3_solve_ex.argtypes = [_P(rbgs_grid), _vp, _vp, ctypes.c_int32, ctypes.c_double,
                                   ctypes.c_int32, _P(rbgs_rb3_opts), _P(rbgs_solve_info), _vp,
                                   ctypes.c_size_t, _vp]
_lib.rbgs_rb3_solve_ex.restype = ctypes.c_int
_lib.rbgs_workspace_size.argtypes = [_P(rbgs_grid), ctypes.c_int, _P(rbgs_solve_opts)]
_lib.rbgs_workspace_size.restype = ctypes.c_size_t
_lib.rbgs_sweep.argtypes = [_P(rbgs_grid), ctypes.c_int, _vp, _vp, ctypes.c_int32,
                            _P(rbgs_sweep_opts), _vp, ctypes.c_size_t, _vp]
_lib.rbgs_sweep.restype = ctypes.c_int
_lib.rbgs_residual.argtypes = [_P(rbgs_grid), ctypes.c_int, _vp, _vp, _P(ctypes.c_double),
                               _P(ctypes.c_double), _vp, ctypes.c_size_t, _vp]
_lib.rbgs_residual.restype = ctypes.c_int
_lib.rbgs_residual_noalloc.argtypes = [_P(rbgs_grid), ctypes.c_int, _vp, _vp,
                                       _P(ctypes.c_double), _P(ctypes.c_double), _vp]
_lib.rbgs_residual_noalloc.restype = ctypes.c_int
_lib.rbgs_solve.argtypes = [_P(rbgs_grid), ctypes.c_int, _vp, _vp, _P(rbgs_solve_opts),
                            _P(rbgs_solve_info), _vp, ctypes.c_size_t, _vp]
_lib.rbgs_solve.restype = ctypes.c_int
_lib.rbgs_stream_probe.argtypes = [ctypes.c_int32, _vp, _vp, _vp, ctypes.c_int64,
                                   ctypes.c_double, _vp]
_lib.rbgs_stream_probe.restype = ctypes.c_int
_lib.rbgs_strerror.argtypes = [ctypes.c_int]
_lib.rbgs_strerror.restype = ctypes.c_char_p
_lib.rbgs_last_error.argtypes = []
_lib.rbgs_last_error.restype = ctypes.c_char_p

_lib.rbgs_batch_workspace_size.argtypes = [ctypes.c_int32, _P(rbgs_grid), ctypes.c_int]
_lib.rbgs_batch_workspace_size.restype = ctypes.c_size_t
_lib.rbgs_sweep_batched.argtypes = [ctypes.c_int32, _P(rbgs_grid), ctypes.c_int, _P(_vp), _P(_vp),
                                    ctypes.c_int32, _P(rbgs_sweep_opts), _vp, ctypes.c_size_t, _vp]
_lib.rbgs_sweep_batched.restype = ctypes.c_int
_lib.rbgs_batch_plan_create.argtypes = [_P(_vp), ctypes.c_int32, _P(rbgs_grid), ctypes.c_int,
                                        _P(_vp), _P(_vp), ctypes.c_int32, _P(rbgs_sweep_opts), _vp,
                                        ctypes.c_size_t]
_lib.rbgs_batch_plan_create.restype = ctypes.c_int
_lib.rbgs_batch_plan_launch.argtypes = [_vp, _vp]
_lib.rbgs_batch_plan_launch.restype = ctypes.c_int
_lib.rbgs_batch_plan_check.argtypes = [_vp, _vp]
_lib.rbgs_batch_plan_check.restype = ctypes.c_int
_lib.rbgs_batch_plan_destroy.argtypes = [_vp]
_lib.rbgs_batch_plan_destroy.restype = ctypes.c_int
_lib.rbgs_autotune_batched.argtypes = [ctypes.c_int32, _P(rbgs_grid), ctypes.c_int, _P(_vp),
                                       _P(_vp), _vp, ctypes.c_size_t, _vp, _P(rbgs_sweep_opts),
                                       _P(ctypes.c_float)]
_lib.rbgs_autotune_batched.restype = ctypes.c_int
_lib.rbgs_batch_last_error.argtypes = []
_lib.rbgs_batch_last_error.restype = ctypes.c_char_p

EXPORTED = ("rbgs_workspace_size", "rbgs_sweep", "rbgs_residual", "rbgs_residual_noalloc",
            "rbgs_solve",
            "rbgs_stream_probe", "rbgs_strerror", "rbgs_last_error", "rbgs_batch_workspace_size",
            "rbgs_sweep_batched", "rbgs_batch_plan_create", "rbgs_batch_plan_launch",
            "rbgs_batch_plan_check", "rbgs_batch_plan_destroy", "rbgs_autotune_batched",
            "rbgs_batch_last_error", "rbgs_unet_param_count", "rbgs_unet_workspace_size",
            "rbgs_unet_create", "rbgs_unet_destroy", "rbgs_unet_set_params",
            "rbgs_unet_get_params", "rbgs_unet_get_grads", "rbgs_unet_get_adam",
            "rbgs_unet_set_adam", "rbgs_unet_forward",
            "rbgs_unet_train_step", "rbgs_solve_learned", "rbgs_unet_last_error",
            "rbgs_restrict", "rbgs_prolong", "rbgs_batch_solve_workspace_size",
            "rbgs_solve_batched", "rbgs_mg_workspace_size", "rbgs_mg_solve",
            "rbgs_mc9_workspace_size", "rbgs_mc9_sweep", "rbgs_mc9_residual", "rbgs_mc9_solve",
            "rbgs_rb3_workspace_size", "rbgs_rb3_sweep", "rbgs_rb3_residual", "rbgs_rb3_solve",
            "rbgs_rb3_sweep_ex", "rbgs_rb3_solve_ex",
            "rbgs_split_pitch", "rbgs_pack", "rbgs_unpack", "rbgs_sweep_split")


class RbgsError(RuntimeError):
    def __init__(self, status, message):
        super().__init__(f"{rbgs_strerror(status)}: {message}")
        self.status = status


def rbgs_strerror(status):
    return _lib.rbgs_strerror(int(status)).decode()


def rbgs_last_error():
    return _lib.rbgs_last_error().decode()


def _check(rc, allow=(OK,)):
    if rc not in allow:
        raise RbgsError(rc, rbgs_last_error())
    return rc


def rbgs_batch_last_error():
    return _lib.rbgs_batch_last_error().decode()


_lib.rbgs_batch_solve_workspace_size.argtypes = [ctypes.c_int32, _P(rbgs_grid)]
_lib.rbgs_batch_solve_workspace_size.restype = ctypes.c_size_t
_lib.rbgs_solve_batched.argtypes = [ctypes.c_int32, _P(rbgs_grid), _P(_vp), _P(_vp),
                                    _P(rbgs_solve_opts), _P(rbgs_solve_info), _vp, ctypes.c_size_t,
                                    _vp]
_lib.rbgs_solve_batched.restype = ctypes.c_int


def _bcheck(rc):
    if rc != OK:
        raise RbgsError(rc, rbgs_batch_last_error())
    return rc


def _dtype_code(t):
    import torch
    if t.dtype == torch.float64:
        return F64
    if t.dtype == torch.float32:
        return F32
    raise TypeError(f"unsupported dtype {t.dtype}")


def make_grid(u, h=None):
    """rbgs_grid for a natural-layout tensor of shape (n+2, m >= n+2)."""
    if u.dim() != 2 or u.shape[0] < 3 or u.shape[1] < u.shape[0] or u.stride(1) != 1:
        raise ValueError("expected a 2-D (n+2, m>=n+2) tensor with unit column stride")
    n = u.shape[0] - 2
    h = 1.0 / (n + 1) if h is None else float(h)
    return rbgs_grid(n, u.stride(0), h)


def _stream_ptr(stream, device):
    import torch
    if stream is None:
        stream = torch.cuda.current_stream(device if device.type == "cuda" else None)
    return _vp(stream.cuda_stream)


def _same_layout(u, f):
    if f.shape != u.shape or f.stride() != u.stride() or f.dtype != u.dtype or f.device != u.device:
        raise ValueError("u and f must share shape, strides, dtype and device")


def rbgs_workspace_size(grid, dtype_code, precision=PREC_F64):
    opts = rbgs_solve_opts()
    opts.precision = precision
    return int(_lib.rbgs_workspace_size(ctypes.byref(grid), dtype_code, ctypes.byref(opts)))


def _workspace(grid, code, device, precision=PREC_F64, workspace=None):
    import torch
    need = rbgs_workspace_size(grid, code, precision)
    if need == 0:
        raise RbgsError(EINVAL, "invalid grid")
    if workspace is None:
        workspace = torch.empty(need, dtype=torch.uint8, device=device)
    return workspace


def _sweep_opts(kernel="auto", fuse=0, tile_rows=0, tile_cols=0, rows_per_block=0,
                debug_delay=0, debug_spin_limit=0, debug_stall_tile=0, timing=None, lds_max_n=0,
                debug_tile_order=0, debug_seed=0, debug_stamp_check=0, debug_trace=None):
    """debug_trace: a device tensor of int64 (any shape; its element count / 4
    records) that receives the persistent kernel's per-item trace."""
    o = rbgs_sweep_opts()
    o.lds_max_n = lds_max_n
    o.debug_tile_order, o.debug_seed, o.debug_stamp_check = debug_tile_order, debug_seed, debug_stamp_check
    if debug_trace is not None:
        if debug_trace.dtype.itemsize != 8 or not debug_trace.is_contiguous():
            raise ValueError("debug_trace must be a contiguous 8-byte integer tensor")
        o.debug_trace = debug_trace.data_ptr()
        o.debug_trace_items = debug_trace.numel() // 4
    o.kernel = _KERNELS[kernel] if isinstance(kernel, str) else int(kernel)
    o.fuse, o.tile_rows, o.tile_cols = fuse, tile_rows, tile_cols
    o.rows_per_block, o.debug_delay, o.debug_spin_limit = rows_per_block, debug_delay, debug_spin_limit
    o.debug_stall_tile = debug_stall_tile
    if timing is not None:
        o.timing = ctypes.pointer(timing)
    return o


def rbgs_sweep(u, f, nsweeps, h=None, kernel="auto", workspace=None, stream=None, timing=False,
               **tuning):
    """nsweeps red-black sweeps of u in place on the GPU (asynchronous unless
    timing=True, which returns a dict of per-phase milliseconds)."""
    _same_layout(u, f)
    grid = make_grid(u, h)
    code = _dtype_code(u)
    ws = _workspace(grid, code, u.device, workspace=workspace)
    t = rbgs_timing() if timing else None
    opts = _sweep_opts(kernel=kernel, timing=t, **tuning)
    _check(_lib.rbgs_sweep(ctypes.byref(grid), code, _vp(u.data_ptr()), _vp(f.data_ptr()),
                           int(nsweeps), ctypes.byref(opts), _vp(ws.data_ptr()), ws.numel(),
                           _stream_ptr(stream, u.device)))
    if timing:
        return _timing_dict(t)
    return None


def rbgs_residual(u, f, h=None, workspace=None, stream=None):
    """(||r||_2, ||r||_2/||b||_2) computed on the GPU in FP64."""
    _same_layout(u, f)
    grid = make_grid(u, h)
    code = _dtype_code(u)
    ws = _workspace(grid, code, u.device, workspace=workspace)
    a = ctypes.c_double()
    r = ctypes.c_double()
    _check(_lib.rbgs_residual(ctypes.byref(grid), code, _vp(u.data_ptr()), _vp(f.data_ptr()),
                              ctypes.byref(a), ctypes.byref(r), _vp(ws.data_ptr()), ws.numel(),
                              _stream_ptr(stream, u.device)))
    return a.value, r.value


def rbgs_residual_noalloc(u, f, h=None, stream=None):
    """(||r||_2, ||r||_2/||b||_2) in FP64 without a workspace: the library's
    static per-GPU scratch holds the partial sums (no device allocation, not
    even by this binding).  Calls overlapping on one GPU race."""
    _same_layout(u, f)
    grid = make_grid(u, h)
    a = ctypes.c_double()
    r = ctypes.c_double()
    rc = _lib.rbgs_residual_noalloc(ctypes.byref(grid), _dtype_code(u), _vp(u.data_ptr()),
                                    _vp(f.data_ptr()), ctypes.byref(a), ctypes.byref(r),
                                    _stream_ptr(stream, u.device))
    _check(rc)
    return a.value, r.value


def rbgs_solve(u, f, max_sweeps, rel_tol, check_every=100, h=None, precision="f64",
               inner_sweeps=0, omega=1.0, kernel="auto", workspace=None, stream=None,
               raise_on_noconv=False, timing=False, fallback=False, **tuning):
    """Solve to rel_tol on the GPU; returns a dict with sweeps, outer_iters,
    rel_residual, abs_residual and status."""
    _same_layout(u, f)
    grid = make_grid(u, h)
    code = _dtype_code(u)
    prec = _PRECISIONS[precision] if isinstance(precision, str) else int(precision)
    ws = _workspace(grid, code, u.device, precision=prec, workspace=workspace)
    opts = rbgs_solve_opts()
    opts.max_sweeps, opts.rel_tol, opts.check_every = int(max_sweeps), float(rel_tol), int(check_every)
    opts.precision, opts.inner_sweeps, opts.omega = prec, int(inner_sweeps), float(omega)
    opts.fallback = 1 if fallback else 0
    t = rbgs_timing() if timing else None
    opts.sweep = _sweep_opts(kernel=kernel, timing=t, **tuning)
    info = rbgs_solve_info()
    rc = _lib.rbgs_solve(ctypes.byref(grid), code, _vp(u.data_ptr()), _vp(f.data_ptr()),
                         ctypes.byref(opts), ctypes.byref(info), _vp(ws.data_ptr()), ws.numel(),
                         _stream_ptr(stream, u.device))
    _check(rc, allow=(OK,) if raise_on_noconv else (OK, ENOCONV, ENONFINITE))
    out = {"sweeps": info.sweeps, "outer_iters": info.outer_iters,
           "rel_residual": info.rel_residual, "abs_residual": info.abs_residual,
           "status": info.status, "precision": info.precision}
    if timing:
        out["timing"] = _timing_dict(t)
    return out


def _mg_opts(max_cycles, rel_tol, pre_sweeps, post_sweeps, max_levels, coarse_sweeps, kernel,
             **tuning):
    o = rbgs_mg_opts()
    o.max_cycles, o.rel_tol = int(max_cycles), float(rel_tol)
    o.pre_sweeps, o.post_sweeps = int(pre_sweeps), int(post_sweeps)
    o.max_levels, o.coarse_sweeps = int(max_levels), int(coarse_sweeps)
    o.sweep = _sweep_opts(kernel=kernel, **tuning)
    return o


def rbgs_mg_workspace_size(grid, dtype_code, max_levels=0):
    opts = rbgs_mg_opts()
    opts.max_levels = max_levels
    return int(_lib.rbgs_mg_workspace_size(ctypes.byref(grid), dtype_code, ctypes.byref(opts)))


def rbgs_mg_solve(u, f, max_cycles, rel_tol, pre_sweeps=2, post_sweeps=2, max_levels=0,
                  coarse_sweeps=0, h=None, kernel="auto", workspace=None, stream=None,
                  raise_on_noconv=False, **tuning):
    """V-cycles with red-black Gauss-Seidel smoothing on the GPU (FP64);
    returns a dict with cycles, levels, coarsest_n, coarse_sweeps,
    rel_residual, abs_residual, graph and status."""
    _same_layout(u, f)
    grid = make_grid(u, h)
    code = _dtype_code(u)
    opts = _mg_opts(max_cycles, rel_tol, pre_sweeps, post_sweeps, max_levels, coarse_sweeps,
                    kernel, **tuning)
    if workspace is None:
        import torch
        need = int(_lib.rbgs_mg_workspace_size(ctypes.byref(grid), code, ctypes.byref(opts)))
        # need == 0 (an invalid request): the library names the problem below
        workspace = torch.empty(need, dtype=torch.uint8, device=u.device) if need else None
    info = rbgs_mg_info()
    wsp = _vp(workspace.data_ptr()) if workspace is not None else None
    rc = _lib.rbgs_mg_solve(ctypes.byref(grid), code, _vp(u.data_ptr()), _vp(f.data_ptr()),
                            ctypes.byref(opts), ctypes.byref(info), wsp,
                            workspace.numel() if workspace is not None else 0,
                            _stream_ptr(stream, u.device))
    _check(rc, allow=(OK,) if raise_on_noconv else (OK, ENOCONV, ENONFINITE))
    return {k: getattr(info, k) for k, _ in rbgs_mg_info._fields_}


def _mc9_args(u, f, h, workspace):
    import torch
    _same_layout(u, f)
    if u.dtype != torch.float64:
        raise RbgsError(EUNSUPPORTED, "the 9-point sweep runs in FP64")
    grid = make_grid(u, h)
    if workspace is None:
        need = int(_lib.rbgs_mc9_workspace_size(ctypes.byref(grid)))
        if need == 0:
            raise RbgsError(EINVAL, "invalid grid")
        workspace = torch.empty(need, dtype=torch.uint8, device=u.device)
    return grid, workspace


def rbgs_mc9_workspace_size(grid):
    return int(_lib.rbgs_mc9_workspace_size(ctypes.byref(grid)))


def _kernel_code(kernel):
    return _KERNELS[kernel] if isinstance(kernel, str) else int(kernel)


def rbgs_mc9_sweep(u, f, nsweeps, h=None, kernel="auto", workspace=None, stream=None):
    """nsweeps four-colour sweeps of the 9-point system, in place (FP64);
    kernel "auto" or "plain" (a launch per colour), or "resident" (the
    flag-driven form: one launch, a counter per block; synchronises)."""
    grid, ws = _mc9_args(u, f, h, workspace)
    _check(_lib.rbgs_mc9_sweep(ctypes.byref(grid), _vp(u.data_ptr()), _vp(f.data_ptr()),
                               int(nsweeps), _kernel_code(kernel), _vp(ws.data_ptr()), ws.numel(),
                               _stream_ptr(stream, u.device)))


def rbgs_mc9_residual(u, f, h=None, workspace=None, stream=None):
    """(||r||_2, ||r||_2/||b||_2) of the 9-point system, on the GPU."""
    grid, ws = _mc9_args(u, f, h, workspace)
    a, r = ctypes.c_double(), ctypes.c_double()
    _check(_lib.rbgs_mc9_residual(ctypes.byref(grid), _vp(u.data_ptr()), _vp(f.data_ptr()),
                                  ctypes.byref(a), ctypes.byref(r), _vp(ws.data_ptr()), ws.numel(),
                                  _stream_ptr(stream, u.device)))
    return a.value, r.value


def rbgs_mc9_solve(u, f, max_sweeps, rel_tol, check_every=100, h=None, kernel="auto",
                   workspace=None, stream=None, raise_on_noconv=False):
    """Four-colour 9-point sweeps until rel <= rel_tol; returns a dict with
    sweeps, rel_residual, abs_residual and status."""
    grid, ws = _mc9_args(u, f, h, workspace)
    info = rbgs_solve_info()
    rc = _lib.rbgs_mc9_solve(ctypes.byref(grid), _vp(u.data_ptr()), _vp(f.data_ptr()),
                             int(max_sweeps), float(rel_tol), int(check_every),
                             _kernel_code(kernel), ctypes.byref(info),
                             _vp(ws.data_ptr()), ws.numel(), _stream_ptr(stream, u.device))
    _check(rc, allow=(OK,) if raise_on_noconv else (OK, ENOCONV, ENONFINITE))
    return {"sweeps": info.sweeps, "rel_residual": info.rel_residual,
            "abs_residual": info.abs_residual, "status": info.status}


def make_grid3(u, h=None):
    """rbgs_grid for a 3-D tensor of shape (n+2, n+2, m >= n+2), contiguous
    planes and rows (the row pitch is the last dimension's length)."""
    if (u.dim() != 3 or u.shape[0] < 3 or u.shape[1] != u.shape[0] or u.shape[2] < u.shape[0]
            or not u.is_contiguous()):
        raise ValueError("expected a contiguous (n+2, n+2, m>=n+2) tensor")
    n = u.shape[0] - 2
    return rbgs_grid(n, u.shape[2], 1.0 / (n + 1) if h is None else float(h))


def _rb3_args(u, f, h, workspace):
    import torch
    _same_layout(u, f)
    if u.dtype != torch.float64:
        raise RbgsError(EUNSUPPORTED, "the 3D sweep runs in FP64")
    grid = make_grid3(u, h)
    if workspace is None:
        need = int(_lib.rbgs_rb3_workspace_size(ctypes.byref(grid)))
        if need == 0:
            raise RbgsError(EINVAL, "invalid grid")
        workspace = torch.empty(need, dtype=torch.uint8, device=u.device)
    return grid, workspace


def rbgs_rb3_workspace_size(grid):
    return int(_lib.rbgs_rb3_workspace_size(ctypes.byref(grid)))


def _rb3_opts(kernel="plain", debug_delay=0, debug_spin_limit=0, debug_stall_block=0):
    o = rbgs_rb3_opts()
    o.kernel = _KERNELS[kernel] if isinstance(kernel, str) else int(kernel)
    o.debug_delay, o.debug_spin_limit = int(debug_delay), int(debug_spin_limit)
    o.debug_stall_block = int(debug_stall_block)
    return o


def rbgs_rb3_sweep(u, f, nsweeps, h=None, workspace=None, stream=None, kernel="plain", **debug):
    """nsweeps 3D red-black sweeps (7-point Laplacian), in place (FP64).
    kernel "plain": one launch per half-sweep; "resident": the flag-driven
    form (one launch, per-block progress counters; synchronises)."""
    grid, ws = _rb3_args(u, f, h, workspace)
    o = _rb3_opts(kernel, **debug)
    _check(_lib.rbgs_rb3_sweep_ex(ctypes.byref(grid), _vp(u.data_ptr()), _vp(f.data_ptr()),
                                  int(nsweeps), ctypes.byref(o), _vp(ws.data_ptr()), ws.numel(),
                                  _stream_ptr(stream, u.device)))


def rbgs_rb3_residual(u, f, h=None, workspace=None, stream=None):
    """(||r||_2, ||r||_2/||b||_2) of the 3D 7-point system, on the GPU."""
    grid, ws = _rb3_args(u, f, h, workspace)
    a, r = ctypes.c_double(), ctypes.c_double()
    _check(_lib.rbgs_rb3_residual(ctypes.byref(grid), _vp(u.data_ptr()), _vp(f.data_ptr()),
                                  ctypes.byref(a), ctypes.byref(r), _vp(ws.data_ptr()), ws.numel(),
                                  _stream_ptr(stream, u.device)))
    return a.value, r.value


def rbgs_rb3_solve(u, f, max_sweeps, rel_tol, check_every=100, h=None, workspace=None,
                   stream=None, raise_on_noconv=False, kernel="plain", **debug):
    """3D red-black sweeps until rel <= rel_tol; returns a dict with sweeps,
    rel_residual, abs_residual and status.  kernel as in rbgs_rb3_sweep."""
    grid, ws = _rb3_args(u, f, h, workspace)
    info = rbgs_solve_info()
    o = _rb3_opts(kernel, **debug)
    rc = _lib.rbgs_rb3_solve_ex(ctypes.byref(grid), _vp(u.data_ptr()), _vp(f.data_ptr()),
                                int(max_sweeps), float(rel_tol), int(check_every), ctypes.byref(o),
                                ctypes.byref(info), _vp(ws.data_ptr()), ws.numel(),
                                _stream_ptr(stream, u.device))
    _check(rc, allow=(OK,) if raise_on_noconv else (OK, ENOCONV, ENONFINITE))
    return {"sweeps": info.sweeps, "rel_residual": info.rel_residual,
            "abs_residual": info.abs_residual, "status": info.status}


def rbgs_split_pitch(grid, dtype_code):
    return int(_lib.rbgs_split_pitch(ctypes.byref(grid), dtype_code))


def rbgs_pack(u, h=None, stream=None):
    """Natural (n+2, ld) tensor -> (red, black) tensors of shape (n+2, pitch)."""
    import torch
    grid = make_grid(u, h)
    code = _dtype_code(u)
    pitch = rbgs_split_pitch(grid, code)
    red = torch.empty((grid.n + 2, pitch), dtype=u.dtype, device=u.device)
    black = torch.empty_like(red)
    _check(_lib.rbgs_pack(ctypes.byref(grid), code, _vp(u.data_ptr()), _vp(red.data_ptr()),
                          _vp(black.data_ptr()), _stream_ptr(stream, u.device)))
    return red, black


def rbgs_unpack(u, red, black, h=None, stream=None):
    """(red, black) -> the interior of the natural tensor u, in place."""
    grid = make_grid(u, h)
    code = _dtype_code(u)
    _check(_lib.rbgs_unpack(ctypes.byref(grid), code, _vp(u.data_ptr()), _vp(red.data_ptr()),
                            _vp(black.data_ptr()), _stream_ptr(stream, u.device)))
    return u


def rbgs_sweep_split(n, u_red, u_black, f_red, f_black, nsweeps, h=None, kernel="auto",
                     workspace=None, stream=None, **tuning):
    """nsweeps sweeps of split arrays (as rbgs_pack makes them) in place."""
    code = _dtype_code(u_red)
    grid = rbgs_grid(int(n), int(n) + 2, 1.0 / (n + 1) if h is None else float(h))
    ws = _workspace(grid, code, u_red.device, workspace=workspace)
    opts = _sweep_opts(kernel=kernel, **tuning)
    _check(_lib.rbgs_sweep_split(ctypes.byref(grid), code, _vp(u_red.data_ptr()),
                                 _vp(u_black.data_ptr()), _vp(f_red.data_ptr()),
                                 _vp(f_black.data_ptr()), int(nsweeps), ctypes.byref(opts),
                                 _vp(ws.data_ptr()), ws.numel(), _stream_ptr(stream, u_red.device)))


def rbgs_stream_probe(kind, a, b, c=None, s=3.0, stream=None):
    """STREAM copy (kind 0: b = a) or triad (kind 1: a = b + s*c) on FP64
    device tensors of equal, even length."""
    n = a.numel()
    cp = _vp(c.data_ptr()) if c is not None else None
    _check(_lib.rbgs_stream_probe(int(kind), _vp(a.data_ptr()), _vp(b.data_ptr()), cp, n,
                                  float(s), _stream_ptr(stream, a.device)))


_lib.rbgs_restrict.argtypes = [ctypes.c_int32, ctypes.c_int, _P(rbgs_grid), _vp, ctypes.c_int64,
                               _P(rbgs_grid), _vp, ctypes.c_int64, _vp]
_lib.rbgs_restrict.restype = ctypes.c_int
_lib.rbgs_prolong.argtypes = [ctypes.c_int32, ctypes.c_int, _P(rbgs_grid), _vp, ctypes.c_int64,
                              _P(rbgs_grid), _vp, ctypes.c_int64, _vp]
_lib.rbgs_prolong.restype = ctypes.c_int


def _level(x):
    """(batch, grid, stride) of a (B, n+2, m) or (n+2, m) natural-layout tensor."""
    if x.dim() == 2:
        return 1, make_grid(x), x.shape[0] * x.stride(0)
    if x.dim() != 3:
        raise ValueError("expected a (n+2, m) or (B, n+2, m) tensor")
    return x.shape[0], make_grid(x[0]), x.stride(0)


def _transfer(src, dst, stream):
    bs, gs, ss = _level(src)
    bd, gd, sd = _level(dst)
    if bs != bd or src.dtype != dst.dtype or src.device != dst.device:
        raise ValueError("src and dst must share batch size, dtype and device")
    return bs, gs, ss, gd, sd, _stream_ptr(stream, src.device)


def rbgs_restrict(fine, coarse, stream=None):
    """coarse interior <- full weighting of fine's interior (n_f = 2 n_c + 1)."""
    b, gf, sf, gc, sc, st = _transfer(fine, coarse, stream)
    _check(_lib.rbgs_restrict(b, _dtype_code(fine), ctypes.byref(gf), _vp(fine.data_ptr()), sf,
                              ctypes.byref(gc), _vp(coarse.data_ptr()), sc, st))


def rbgs_prolong(coarse, fine, stream=None):
    """fine interior <- bilinear interpolation of coarse (ring included)."""
    b, gc, sc, gf, sf, st = _transfer(coarse, fine, stream)
    _check(_lib.rbgs_prolong(b, _dtype_code(coarse), ctypes.byref(gc), _vp(coarse.data_ptr()), sc,
                             ctypes.byref(gf), _vp(fine.data_ptr()), sf, st))


# ---------------------------------------------------------------------------
# Batches of grids
# ---------------------------------------------------------------------------
class _Batch:
    """Host arrays of one batch: grid descriptors and device pointers."""

    def __init__(self, us, fs, hs=None):
        if len(us) != len(fs) or not us:
            raise ValueError("need equal, non-empty lists of u and f tensors")
        self.count = len(us)
        self.code = _dtype_code(us[0])
        self.grids = (rbgs_grid * self.count)()
        self.u = (_vp * self.count)()
        self.f = (_vp * self.count)()
        for g, (u, f) in enumerate(zip(us, fs)):
            _same_layout(u, f)
            if _dtype_code(u) != self.code or u.device != us[0].device:
                raise ValueError("all grids of a batch share dtype and device")
            self.grids[g] = make_grid(u, None if hs is None else hs[g])
            self.u[g] = u.data_ptr()
            self.f[g] = f.data_ptr()
        self.device = us[0].device
        self.tensors = (list(us), list(fs))  # keep the arrays alive

    def workspace(self, workspace=None):
        import torch
        need = int(_lib.rbgs_batch_workspace_size(self.count, self.grids, self.code))
        if need == 0:
            raise RbgsError(EINVAL, "invalid batch")
        if workspace is None:
            workspace = torch.empty(need, dtype=torch.uint8, device=self.device)
        return workspace


def rbgs_batch_workspace_size(us, fs, hs=None):
    b = _Batch(us, fs, hs)
    return int(_lib.rbgs_batch_workspace_size(b.count, b.grids, b.code))


def rbgs_sweep_batched(us, fs, nsweeps, hs=None, workspace=None, stream=None, timing=False,
                       **tuning):
    """nsweeps sweeps of every grid in one persistent launch (synchronises)."""
    b = _Batch(us, fs, hs)
    ws = b.workspace(workspace)
    t = rbgs_timing() if timing else None
    opts = _sweep_opts(kernel=tuning.pop("kernel", "auto"), timing=t, **tuning)
    _bcheck(_lib.rbgs_sweep_batched(b.count, b.grids, b.code, b.u, b.f, int(nsweeps),
                                    ctypes.byref(opts), _vp(ws.data_ptr()), ws.numel(),
                                    _stream_ptr(stream, b.device)))
    if timing:
        return {"sweep_ms": t.sweep_ms, "sweep_launches": t.sweep_launches}
    return None


class BatchPlan:
    """A batched sweep captured into a HIP graph; launch() replays it."""

    def __init__(self, us, fs, nsweeps, hs=None, workspace=None, **tuning):
        self._batch = _Batch(us, fs, hs)
        self.workspace = self._batch.workspace(workspace)
        opts = _sweep_opts(kernel=tuning.pop("kernel", "auto"), **tuning)
        handle = _vp()
        b = self._batch
        _bcheck(_lib.rbgs_batch_plan_create(ctypes.byref(handle), b.count, b.grids, b.code, b.u,
                                            b.f, int(nsweeps), ctypes.byref(opts),
                                            _vp(self.workspace.data_ptr()), self.workspace.numel()))
        self._handle = handle
        self.nsweeps = int(nsweeps)

    def launch(self, stream=None):
        _bcheck(_lib.rbgs_batch_plan_launch(self._handle, _stream_ptr(stream, self._batch.device)))

    def check(self, stream=None):
        _bcheck(_lib.rbgs_batch_plan_check(self._handle, _stream_ptr(stream, self._batch.device)))

    def close(self):
        if getattr(self, "_handle", None) is not None and self._handle.value:
            _lib.rbgs_batch_plan_destroy(self._handle)
            self._handle = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()
        return False

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def rbgs_solve_batched(us, fs, max_sweeps, rel_tol, inner_sweeps, precision="f32_ir", hs=None,
                       workspace=None, stream=None, omega=1.0, **tuning):
    """Solve every FP64 grid of the batch to rel_tol: precision "f64" sweeps
    in FP64 and checks the residual every inner_sweeps sweeps; "f32_ir" and
    "bf16rhs_ir" refine in FP64 around inner_sweeps FP32 sweeps.  The sweeps
    of all unconverged grids run in one batched launch per round; returns
    one dict per grid like rbgs_solve's.  omega != 1 ("f64" only): red-black
    SOR, 0 = each grid's optimum.  Synchronises."""
    b = _Batch(us, fs, hs)
    if b.code != F64:
        raise RbgsError(EINVAL, "batched solves take FP64 u and f")
    need = int(_lib.rbgs_batch_solve_workspace_size(b.count, b.grids))
    if need == 0:
        raise RbgsError(EINVAL, "invalid batch")
    if workspace is None:
        import torch
        workspace = torch.empty(need, dtype=torch.uint8, device=b.device)
    opts = rbgs_solve_opts()
    opts.max_sweeps, opts.rel_tol, opts.check_every = int(max_sweeps), float(rel_tol), int(inner_sweeps)
    opts.precision = _PRECISIONS[precision] if isinstance(precision, str) else int(precision)
    opts.inner_sweeps, opts.omega = int(inner_sweeps), float(omega)
    opts.sweep = _sweep_opts(kernel=tuning.pop("kernel", "auto"), **tuning)
    infos = (rbgs_solve_info * b.count)()
    rc = _lib.rbgs_solve_batched(b.count, b.grids, b.u, b.f, ctypes.byref(opts), infos,
                                 _vp(workspace.data_ptr()), workspace.numel(),
                                 _stream_ptr(stream, b.device))
    if rc not in (OK, ENOCONV, ENONFINITE):
        _bcheck(rc)
    return [{"sweeps": i.sweeps, "outer_iters": i.outer_iters, "rel_residual": i.rel_residual,
             "abs_residual": i.abs_residual, "status": i.status, "precision": i.precision}
            for i in infos]


def rbgs_autotune_batched(us, fs, hs=None, workspace=None, stream=None):
    """Tune (fuse, tile_rows, lds_max_n) for this batch shape; returns the choice."""
    b = _Batch(us, fs, hs)
    ws = b.workspace(workspace)
    best = rbgs_sweep_opts()
    ms = ctypes.c_float()
    _bcheck(_lib.rbgs_autotune_batched(b.count, b.grids, b.code, b.u, b.f, _vp(ws.data_ptr()),
                                       ws.numel(), _stream_ptr(stream, b.device),
                                       ctypes.byref(best), ctypes.byref(ms)))
    return {"fuse": best.fuse, "tile_rows": best.tile_rows, "lds_max_n": best.lds_max_n,
            "ms_per_sweep": ms.value}


# ---------------------------------------------------------------------------
# Learned initial guess (U-Net run and trained by the library's kernels)
# ---------------------------------------------------------------------------
_lib.rbgs_unet_param_count.argtypes = []
_lib.rbgs_unet_param_count.restype = ctypes.c_size_t
_lib.rbgs_unet_workspace_size.argtypes = [ctypes.c_int32, ctypes.c_int32, ctypes.c_int32]
_lib.rbgs_unet_workspace_size.restype = ctypes.c_size_t
_lib.rbgs_unet_create.argtypes = [_P(_vp), ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, _vp,
                                  ctypes.c_size_t]
_lib.rbgs_unet_create.restype = ctypes.c_int
_lib.rbgs_unet_destroy.argtypes = [_vp]
_lib.rbgs_unet_destroy.restype = ctypes.c_int
for _name in ("rbgs_unet_set_params", "rbgs_unet_get_params", "rbgs_unet_get_grads"):
    getattr(_lib, _name).argtypes = [_vp, _vp, ctypes.c_size_t, _vp]
    getattr(_lib, _name).restype = ctypes.c_int
_lib.rbgs_unet_get_adam.argtypes = [_vp, _vp, _vp, ctypes.c_size_t, _P(ctypes.c_int32), _vp]
_lib.rbgs_unet_get_adam.restype = ctypes.c_int
_lib.rbgs_unet_set_adam.argtypes = [_vp, _vp, _vp, ctypes.c_size_t, ctypes.c_int32, _vp]
_lib.rbgs_unet_set_adam.restype = ctypes.c_int
_lib.rbgs_unet_forward.argtypes = [_vp, ctypes.c_int32, _vp, ctypes.c_int64, _vp, _vp]
_lib.rbgs_unet_forward.restype = ctypes.c_int
_lib.rbgs_unet_train_step.argtypes = [_vp, ctypes.c_int32, _vp, _vp, ctypes.c_int64, ctypes.c_float,
                                      ctypes.c_int32, _P(ctypes.c_float), _vp]
_lib.rbgs_unet_train_step.restype = ctypes.c_int
_lib.rbgs_solve_learned.argtypes = [_vp, _P(rbgs_grid), _vp, _vp, _P(rbgs_solve_opts),
                                    ctypes.c_int32, _P(rbgs_solve_info), _P(ctypes.c_int32),
                                    _P(ctypes.c_double), _vp, ctypes.c_size_t, _vp]
_lib.rbgs_solve_learned.restype = ctypes.c_int
_lib.rbgs_unet_last_error.argtypes = []
_lib.rbgs_unet_last_error.restype = ctypes.c_char_p


def rbgs_unet_param_count():
    return int(_lib.rbgs_unet_param_count())


def _ncheck(rc, allow=(OK,)):
    if rc not in allow:
        raise RbgsError(rc, _lib.rbgs_unet_last_error().decode())
    return rc


class UNet:
    """The learned-guess network for N x N grids and up to `batch` samples
    per call, levels coarsened by `factor` (2: N = 2^k - 1 >= 63; 4: N + 1 a
    multiple of 64, N >= 127); all state in one device workspace."""

    def __init__(self, n, batch, factor=4, device="cuda", workspace=None):
        import torch
        self.n, self.batch, self.factor = int(n), int(batch), int(factor)
        need = int(_lib.rbgs_unet_workspace_size(self.n, self.batch, self.factor))
        if need == 0:
            raise RbgsError(EINVAL, "unsupported n / batch / factor (factor 2: n = 2^k - 1 >= 63; "
                                    "factor 4: n + 1 a multiple of 64, n >= 127; batch 1..4096)")
        self.device = torch.device(device)
        self.workspace = workspace if workspace is not None else torch.empty(
            need, dtype=torch.uint8, device=self.device)
        h = _vp()
        _ncheck(_lib.rbgs_unet_create(ctypes.byref(h), self.n, self.batch, self.factor,
                                      _vp(self.workspace.data_ptr()), self.workspace.numel()))
        self._h = h
        self.count = rbgs_unet_param_count()

    def _stream(self, stream):
        return _stream_ptr(stream, self.device)

    def set_params(self, params, stream=None):
        import numpy as np
        p = np.ascontiguousarray(params, dtype=np.float32)
        if p.size != self.count:
            raise ValueError(f"expected {self.count} parameters")
        _ncheck(_lib.rbgs_unet_set_params(self._h, _vp(p.ctypes.data), p.size, self._stream(stream)))

    def _get(self, fn, stream):
        import numpy as np
        out = np.empty(self.count, np.float32)
        _ncheck(fn(self._h, _vp(out.ctypes.data), out.size, self._stream(stream)))
        return out

    def get_params(self, stream=None):
        return self._get(_lib.rbgs_unet_get_params, stream)

    def get_grads(self, stream=None):
        return self._get(_lib.rbgs_unet_get_grads, stream)

    def get_adam(self, stream=None):
        """Adam's state for resuming training: (m, v, step)."""
        import numpy as np
        m, v = np.empty(self.count, np.float32), np.empty(self.count, np.float32)
        step = ctypes.c_int32()
        _ncheck(_lib.rbgs_unet_get_adam(self._h, _vp(m.ctypes.data), _vp(v.ctypes.data), self.count,
                                        ctypes.byref(step), self._stream(stream)))
        return m, v, step.value

    def set_adam(self, m, v, step, stream=None):
        """Restore Adam's state (after set_params, which restarts it)."""
        import numpy as np
        m = np.ascontiguousarray(m, dtype=np.float32)
        v = np.ascontiguousarray(v, dtype=np.float32)
        if m.size != self.count or v.size != self.count:
            raise ValueError(f"expected {self.count} values in m and in v")
        _ncheck(_lib.rbgs_unet_set_adam(self._h, _vp(m.ctypes.data), _vp(v.ctypes.data), self.count,
                                        int(step), self._stream(stream)))

    def _check_batch(self, f):
        if f.dim() != 3 or f.shape[1] != self.n + 2 or f.stride(2) != 1 or f.dtype.itemsize != 8:
            raise ValueError("expected a float64 (batch, n+2, ld) tensor with unit column stride")
        if f.stride(0) != (self.n + 2) * f.stride(1):
            raise ValueError("grids of a batch must be stored back to back")
        return f.shape[0], f.stride(1)

    def forward(self, f, u0, stream=None):
        """u0[b] interior <- the network's guess for f[b]."""
        b, ld = self._check_batch(f)
        if u0.shape != f.shape or u0.stride() != f.stride():
            raise ValueError("u0 must have f's shape and strides")
        _ncheck(_lib.rbgs_unet_forward(self._h, b, _vp(f.data_ptr()), ld, _vp(u0.data_ptr()),
                                       self._stream(stream)))

    def train_step(self, f, u_target, lr, update=True, stream=None):
        b, ld = self._check_batch(f)
        if u_target.shape != f.shape or u_target.stride() != f.stride():
            raise ValueError("u_target must have f's shape and strides")
        loss = ctypes.c_float()
        _ncheck(_lib.rbgs_unet_train_step(self._h, b, _vp(f.data_ptr()), _vp(u_target.data_ptr()),
                                          ld, float(lr), 1 if update else 0, ctypes.byref(loss),
                                          self._stream(stream)))
        return loss.value

    def solve_learned(self, u, f, max_sweeps, rel_tol, check_every=1000, kernel="auto",
                      compare_after=0, workspace=None, stream=None, **tuning):
        """Solve from the better of the caller's start and the network's
        guess (lower relative residual, after compare_after sweeps of both);
        returns rbgs_solve's statistics plus used_guess and rel_start."""
        _same_layout(u, f)
        grid = make_grid(u)
        ws = _workspace(grid, F64, u.device, workspace=workspace)
        opts = rbgs_solve_opts()
        opts.max_sweeps, opts.rel_tol, opts.check_every = int(max_sweeps), float(rel_tol), int(check_every)
        opts.omega = 1.0
        opts.sweep = _sweep_opts(kernel=kernel, **tuning)
        info = rbgs_solve_info()
        used = ctypes.c_int32()
        rel0 = ctypes.c_double()
        rc = _lib.rbgs_solve_learned(self._h, ctypes.byref(grid), _vp(u.data_ptr()),
                                     _vp(f.data_ptr()), ctypes.byref(opts), int(compare_after),
                                     ctypes.byref(info),
                                     ctypes.byref(used), ctypes.byref(rel0), _vp(ws.data_ptr()),
                                     ws.numel(), self._stream(stream))
        _ncheck(rc, allow=(OK, ENOCONV))
        return {"sweeps": info.sweeps, "rel_residual": info.rel_residual, "status": info.status,
                "used_guess": bool(used.value), "rel_start": rel0.value}

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            _lib.rbgs_unet_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
