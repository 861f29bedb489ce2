"""C-ABI host checks that need no GPU: the library loads, exports every
function include/rbgs.h declares, and rejects bad arguments before any
device call."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER_DIR = os.path.join(ROOT, "include")


def declared_functions():
    names = set()
    for fname in os.listdir(HEADER_DIR):
        if not fname.endswith(".h"):
            continue
        text = open(os.path.join(HEADER_DIR, fname)).read()
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        for m in re.finditer(r"\b(rbgs_[a-z0-9_]+)\s*\(", text):
            names.add(m.group(1))
    return names


@pytest.fixture(scope="module")
def lib():
    from paper_2607_01735_amd import rbgs
    return rbgs


def test_library_exports_every_declared_symbol(lib):
    declared = declared_functions()
    assert {"rbgs_sweep", "rbgs_residual", "rbgs_solve", "rbgs_workspace_size"} <= declared
    raw = ctypes.CDLL(lib.LIB_PATH)
    for name in sorted(declared):
        assert hasattr(raw, name), f"{name} declared in include/ but not exported"


def test_binding_names_match_abi(lib):
    import paper_2607_01735_amd as pkg
    for name in ("rbgs_sweep", "rbgs_residual", "rbgs_solve", "rbgs_workspace_size",
                 "rbgs_strerror", "rbgs_last_error"):
        assert callable(getattr(pkg, name))


def test_strerror(lib):
    assert lib.rbgs_strerror(0) == "RBGS_OK"
    for code in (-1, -2, -3, -4, -5, -6, -8):
        assert lib.rbgs_strerror(code).startswith("RBGS_E")
    assert "unknown" in lib.rbgs_strerror(12345)


def _grid(lib, n=31, ld=None, h=None):
    return lib.rbgs_grid(n, n + 2 if ld is None else ld, 1.0 / (n + 1) if h is None else h)


def test_workspace_size(lib):
    g = _grid(lib, 255)
    s64 = lib.rbgs_workspace_size(g, lib.F64)
    s32 = lib.rbgs_workspace_size(g, lib.F32)
    # four split colour arrays (u red/black, f red/black) at least
    assert s64 >= 4 * 257 * 129 * 8 and s32 >= 4 * 257 * 129 * 4
    assert s64 % 256 == 0
    assert lib.rbgs_workspace_size(g, lib.F64, lib.PREC_F32_IR) > s64
    assert lib.rbgs_workspace_size(_grid(lib, 0), lib.F64) == 0
    assert lib.rbgs_workspace_size(_grid(lib, 31, ld=32), lib.F64) == 0
    assert lib.rbgs_workspace_size(_grid(lib, 31, h=-1.0), lib.F64) == 0
    assert lib.rbgs_workspace_size(_grid(lib, 31, h=float("inf")), lib.F64) == 0
    assert lib.rbgs_workspace_size(_grid(lib, 31), 7) == 0


def _sweep(lib, grid, dtype=0, nsweeps=1, opts=None, ws=None, ws_bytes=0):
    o = ctypes.byref(opts) if opts is not None else None
    return lib._lib.rbgs_sweep(ctypes.byref(grid), dtype, None, None, nsweeps, o, ws, ws_bytes,
                               None)


@pytest.mark.parametrize("bad", ["n0", "nbig", "ld", "h0", "hnan", "dtype", "nsweeps", "kernel",
                                 "negopt", "rows_small", "rows_big", "ws_null", "ws_align",
                                 "ws_small", "order", "stamp", "trace_items", "trace_null"])
def test_sweep_validation_before_device_work(lib, bad):
    g = _grid(lib, 31)
    dtype, nsweeps, opts = lib.F64, 1, lib.rbgs_sweep_opts()
    ws, ws_bytes = ctypes.c_void_p(1 << 20), 1 << 30
    expect = lib.EINVAL
    if bad == "n0":
        g = _grid(lib, 0)
    elif bad == "nbig":
        g = lib.rbgs_grid(70000, 70002, 1e-5)
    elif bad == "ld":
        g = _grid(lib, 31, ld=32)
    elif bad == "h0":
        g = _grid(lib, 31, h=0.0)
    elif bad == "hnan":
        g = _grid(lib, 31, h=float("nan"))
    elif bad == "dtype":
        dtype = 5
    elif bad == "nsweeps":
        nsweeps = -1
    elif bad == "kernel":
        opts.kernel = 9
    elif bad == "negopt":
        opts.fuse = -2
    elif bad == "rows_small":
        opts.kernel, opts.tile_rows = 2, 7
    elif bad == "rows_big":  # would overflow the strip count; rejected, not clamped
        opts.kernel, opts.tile_rows = 2, (1 << 31) - 1
    elif bad == "ws_null":
        ws, expect = None, lib.EWORKSPACE
    elif bad == "ws_align":
        ws, expect = ctypes.c_void_p((1 << 20) + 8), lib.EWORKSPACE
    elif bad == "ws_small":
        ws_bytes, expect = 100, lib.EWORKSPACE
    elif bad == "order":
        opts.kernel, opts.debug_tile_order = 2, 3
    elif bad == "stamp":
        opts.kernel, opts.debug_stamp_check = 2, 2
    elif bad == "trace_items":  # a trace array without a record count
        opts.kernel, opts.debug_trace = 2, 1 << 20
    elif bad == "trace_null":   # a record count without an array
        opts.kernel, opts.debug_trace_items = 2, 16
    rc = _sweep(lib, g, dtype, nsweeps, opts, ws, ws_bytes)
    assert rc == expect, lib.rbgs_last_error()
    assert lib.rbgs_last_error()


@pytest.mark.parametrize("bad", ["omega", "omega_range", "sor_f32", "sor_ir", "check", "maxs",
                                 "prec", "ir_f32", "nan_tol", "inner"])
def test_solve_validation_before_device_work(lib, bad):
    g = _grid(lib, 31)
    o = lib.rbgs_solve_opts()
    o.max_sweeps, o.rel_tol, o.check_every, o.omega = 10, 1e-8, 5, 1.0
    dtype = lib.F64
    expect = lib.EINVAL
    if bad == "omega":  # SOR runs without the persistent kernel's verification modes
        o.omega, o.sweep.kernel, expect = 1.5, lib._KERNELS["blocked"], lib.EUNSUPPORTED
        o.sweep.debug_tile_order = 1
    elif bad == "omega_range":
        o.omega = 2.5
    elif bad == "sor_f32":
        o.omega, dtype, expect = 1.5, lib.F32, lib.EUNSUPPORTED
    elif bad == "sor_ir":
        o.omega, o.precision, expect = 1.5, lib.PREC_F32_IR, lib.EUNSUPPORTED
    elif bad == "check":
        o.check_every = 0
    elif bad == "maxs":
        o.max_sweeps = -1
    elif bad == "prec":
        o.precision = 7
    elif bad == "ir_f32":
        o.precision, dtype = lib.PREC_F32_IR, lib.F32
    elif bad == "nan_tol":
        o.rel_tol = float("nan")
    elif bad == "inner":
        o.inner_sweeps = -3
    info = lib.rbgs_solve_info()
    rc = lib._lib.rbgs_solve(ctypes.byref(g), dtype, None, None, ctypes.byref(o),
                             ctypes.byref(info), None, 0, None)
    assert rc == expect, lib.rbgs_last_error()


def test_residual_validation(lib):
    g = _grid(lib, 0)
    a = ctypes.c_double()
    rc = lib._lib.rbgs_residual(ctypes.byref(g), lib.F64, None, None, ctypes.byref(a), None,
                                None, 0, None)
    assert rc == lib.EINVAL
    g = _grid(lib, 15)
    rc = lib._lib.rbgs_residual(ctypes.byref(g), lib.F64, None, None, ctypes.byref(a), None,
                                None, 0, None)
    assert rc == lib.EWORKSPACE


def test_python_binding_rejects_mismatched_tensors(lib):
    torch = pytest.importorskip("torch")
    u = torch.zeros(10, 10, dtype=torch.float64)
    f = torch.zeros(10, 10, dtype=torch.float32)
    with pytest.raises(ValueError):
        lib.rbgs_sweep(u, f, 1)
    with pytest.raises(ValueError):
        lib.make_grid(torch.zeros(10, 5, dtype=torch.float64))
    with pytest.raises(TypeError):
        lib._dtype_code(torch.zeros(3, 3, dtype=torch.int32))


@pytest.mark.parametrize("case", ["batch", "dtype", "sizes", "stride", "null"])
def test_transfer_validation(lib, case):
    fine, coarse = _grid(lib, 15), _grid(lib, 7)
    batch, dt, fs, cs = 2, lib.F64, 17 * 17, 9 * 9
    if case == "batch":
        batch = 0
    elif case == "dtype":
        dt = 7
    elif case == "sizes":
        coarse = _grid(lib, 6)
    elif case == "stride":
        cs = 9 * 9 - 1
    for fn in (lib._lib.rbgs_restrict, lib._lib.rbgs_prolong):
        if fn is lib._lib.rbgs_restrict:
            rc = fn(batch, dt, ctypes.byref(fine), None, fs, ctypes.byref(coarse), None, cs, None)
        else:
            rc = fn(batch, dt, ctypes.byref(coarse), None, cs, ctypes.byref(fine), None, fs, None)
        assert rc == lib.EINVAL, (case, rc)
        if case == "null":
            assert "NULL" in lib.rbgs_last_error()


@pytest.mark.parametrize("bad", ["null_opts", "prec", "omega", "omega0", "omega_range", "tol",
                                 "inner", "check", "count", "null_arrays", "ws", "ws_f64",
                                 "ws_sor"])
def test_solve_batched_validation_before_device_work(lib, bad):
    grids = (lib.rbgs_grid * 2)(_grid(lib, 15), _grid(lib, 31))
    ptrs = (ctypes.c_void_p * 2)(1 << 20, 2 << 20)  # never dereferenced: checks come first
    o = lib.rbgs_solve_opts()
    o.max_sweeps, o.rel_tol, o.check_every, o.inner_sweeps = 100, 1e-8, 10, 10
    o.precision, o.omega = lib.PREC_F32_IR, 1.0
    count, opts, u, f, expect = 2, ctypes.byref(o), ptrs, ptrs, lib.EINVAL
    if bad == "null_opts":
        opts = None
    elif bad == "prec":
        o.precision = 3
    elif bad == "omega":  # SOR runs without refinement
        o.omega, expect = 1.5, lib.EUNSUPPORTED
    elif bad == "omega0":  # 0 asks for each grid's optimal SOR factor
        o.omega, expect = 0.0, lib.EUNSUPPORTED
    elif bad == "omega_range":
        o.omega, o.precision = 2.0, lib.PREC_F64
    elif bad == "ws_sor":  # FP64 SOR passes the option checks
        o.omega, o.precision, expect = 0.0, lib.PREC_F64, lib.EWORKSPACE
    elif bad == "check":
        o.check_every = -1
    elif bad == "ws_f64":  # FP64 solves take the same workspace
        o.precision, expect = lib.PREC_F64, lib.EWORKSPACE
    elif bad == "tol":
        o.rel_tol = 0.0
    elif bad == "inner":
        o.inner_sweeps, o.check_every = 0, 0
    elif bad == "count":
        count = 0
    elif bad == "null_arrays":
        u = None
    elif bad == "ws":
        expect = lib.EWORKSPACE
    rc = lib._lib.rbgs_solve_batched(count, grids, u, f, opts, None, None, 0, None)
    assert rc == expect, lib.rbgs_batch_last_error()
    assert lib._lib.rbgs_batch_solve_workspace_size(0, grids) == 0
    assert lib._lib.rbgs_batch_solve_workspace_size(2, grids) > 0


def test_mg_workspace_size(lib):
    g = _grid(lib, 255)
    full = lib.rbgs_mg_workspace_size(g, lib.F64)
    one = lib.rbgs_mg_workspace_size(g, lib.F64, max_levels=1)
    # every level holds a full single-grid workspace; the coarse levels add
    # about a third of the finest one
    assert one == lib.rbgs_workspace_size(g, lib.F64)
    assert one < full < 1.5 * one
    assert full % 256 == 0
    assert lib.rbgs_mg_workspace_size(g, lib.F32) == 0
    assert lib.rbgs_mg_workspace_size(_grid(lib, 0), lib.F64) == 0
    assert lib.rbgs_mg_workspace_size(g, lib.F64, max_levels=-1) == 0


@pytest.mark.parametrize("bad", ["f32", "dtype", "null_opts", "cycles", "pre", "nosmooth",
                                 "levels", "coarse", "nan_tol", "kernel", "timing", "ws_null"])
def test_mg_validation_before_device_work(lib, bad):
    g = _grid(lib, 63)
    o = lib.rbgs_mg_opts()
    o.max_cycles, o.rel_tol, o.pre_sweeps, o.post_sweeps = 5, 1e-8, 2, 2
    dtype, expect, opts = lib.F64, lib.EINVAL, ctypes.byref(o)
    if bad == "f32":
        dtype, expect = lib.F32, lib.EUNSUPPORTED
    elif bad == "dtype":
        dtype = 9
    elif bad == "null_opts":
        opts = None
    elif bad == "cycles":
        o.max_cycles = -1
    elif bad == "pre":
        o.pre_sweeps = -1
    elif bad == "nosmooth":
        o.pre_sweeps = o.post_sweeps = 0
    elif bad == "levels":
        o.max_levels = -2
    elif bad == "coarse":
        o.coarse_sweeps = -5
    elif bad == "nan_tol":
        o.rel_tol = float("nan")
    elif bad == "kernel":
        o.sweep.kernel = 11
    elif bad == "timing":
        t = lib.rbgs_timing()
        o.sweep.timing = ctypes.pointer(t)
        expect = lib.EUNSUPPORTED
    elif bad == "ws_null":
        expect = lib.EWORKSPACE
    info = lib.rbgs_mg_info()
    rc = lib._lib.rbgs_mg_solve(ctypes.byref(g), dtype, None, None, opts, ctypes.byref(info),
                                None, 0, None)
    assert rc == expect, lib.rbgs_last_error()
    assert lib.rbgs_last_error()


def test_mc9_workspace_and_validation(lib):
    g = _grid(lib, 255)
    size = lib.rbgs_mc9_workspace_size(g)
    # eight colour arrays of 129 rows x 160 doubles at least
    assert size >= 8 * 129 * 128 * 8 and size % 256 == 0
    assert lib.rbgs_mc9_workspace_size(_grid(lib, 0)) == 0
    raw = lib._lib
    gp = ctypes.byref(g)
    assert raw.rbgs_mc9_sweep(gp, None, None, -1, 0, None, 0, None) == lib.EINVAL
    assert raw.rbgs_mc9_sweep(gp, None, None, 1, 9, None, 0, None) == lib.EINVAL
    assert raw.rbgs_mc9_sweep(gp, None, None, 1, 2, None, 0, None) == lib.EWORKSPACE
    assert raw.rbgs_mc9_sweep(gp, None, None, 1, 0, None, 0, None) == lib.EWORKSPACE
    info = lib.rbgs_solve_info()
    assert raw.rbgs_mc9_solve(gp, None, None, 10, 1e-8, 0, 0, ctypes.byref(info), None, 0,
                              None) == lib.EINVAL
    assert raw.rbgs_mc9_solve(gp, None, None, 10, float("nan"), 5, 0, ctypes.byref(info), None,
                              0, None) == lib.EINVAL
    bad = _grid(lib, 31, ld=30)
    assert raw.rbgs_mc9_residual(ctypes.byref(bad), None, None, None, None, None, 0,
                                 None) == lib.EINVAL


def test_rb3_workspace_and_validation(lib):
    g = _grid(lib, 63)
    size = lib.rbgs_rb3_workspace_size(g)
    assert size >= 4 * 65 * 65 * 64 * 8 and size % 256 == 0
    assert lib.rbgs_rb3_workspace_size(lib.rbgs_grid(5000, 5002, 1e-3)) == 0
    raw = lib._lib
    gp = ctypes.byref(g)
    assert raw.rbgs_rb3_sweep(gp, None, None, -1, None, 0, None) == lib.EINVAL
    assert raw.rbgs_rb3_sweep(gp, None, None, 1, None, 0, None) == lib.EWORKSPACE
    info = lib.rbgs_solve_info()
    assert raw.rbgs_rb3_solve(gp, None, None, 10, 1e-8, 0, ctypes.byref(info), None, 0,
                              None) == lib.EINVAL
    bad = _grid(lib, 31, h=0.0)
    assert raw.rbgs_rb3_residual(ctypes.byref(bad), None, None, None, None, None, 0,
                                 None) == lib.EINVAL


@pytest.mark.parametrize("case", ["blocked", "unknown", "delay", "spin", "stall", "sweeps",
                                  "ws", "solve_blocked", "solve_sweeps"])
def test_rb3_kernel_options_validate_before_device_work(lib, case):
    """The 3D calls' kernel choice: PLAIN/AUTO or RESIDENT (the flag-driven
    form); BLOCKED is unsupported; debug fields must be >= 0."""
    g = _grid(lib, 63)
    o = lib.rbgs_rb3_opts()
    o.kernel = lib.KERNEL_RESIDENT
    nsweeps, expect = 4, lib.EINVAL
    if case in ("blocked", "solve_blocked"):
        o.kernel, expect = lib.KERNEL_BLOCKED, lib.EUNSUPPORTED
    elif case == "unknown":
        o.kernel = 9
    elif case == "delay":
        o.debug_delay = -1
    elif case == "spin":
        o.debug_spin_limit = -2
    elif case == "stall":
        o.debug_stall_block = -1
    elif case == "sweeps":
        nsweeps = (1 << 29) + 1
    elif case == "ws":
        expect = lib.EWORKSPACE
    raw = lib._lib
    if case.startswith("solve"):
        info = lib.rbgs_solve_info()
        ms = (1 << 29) + 1 if case == "solve_sweeps" else 10
        rc = raw.rbgs_rb3_solve_ex(ctypes.byref(g), None, None, ms, 1e-8, 5, ctypes.byref(o),
                                   ctypes.byref(info), None, 0, None)
    else:
        rc = raw.rbgs_rb3_sweep_ex(ctypes.byref(g), None, None, nsweeps, ctypes.byref(o), None, 0,
                                   None)
    assert rc == expect, (case, rc, lib.rbgs_last_error())


def test_split_layout_entry_points_validate(lib):
    g = _grid(lib, 255)
    assert lib.rbgs_split_pitch(g, lib.F64) == 160  # ceil(257 / 2) = 129 -> 5 x 32
    assert lib.rbgs_split_pitch(g, lib.F32) == 192  # 129 -> 3 x 64
    assert lib.rbgs_split_pitch(_grid(lib, 0), lib.F64) == 0
    raw = lib._lib
    gp = ctypes.byref(g)
    assert raw.rbgs_pack(gp, 7, None, None, None, None) == lib.EINVAL
    assert raw.rbgs_pack(ctypes.byref(_grid(lib, 31, ld=3)), 0, None, None, None, None) == lib.EINVAL
    assert raw.rbgs_unpack(gp, 7, None, None, None, None) == lib.EINVAL
    o = lib.rbgs_sweep_opts()
    assert raw.rbgs_sweep_split(gp, 0, None, None, None, None, -1, ctypes.byref(o), None, 0,
                                None) == lib.EINVAL
    assert raw.rbgs_sweep_split(gp, 0, None, None, None, None, 3, ctypes.byref(o), None, 0,
                                None) == lib.EWORKSPACE
    t = lib.rbgs_timing()
    o.timing = ctypes.pointer(t)
    assert raw.rbgs_sweep_split(gp, 0, None, None, None, None, 3, ctypes.byref(o), None, 0,
                                None) == lib.EUNSUPPORTED


@pytest.mark.parametrize("rows", [7, 65537, (1 << 31) - 1])
def test_batched_tile_rows_bounds(lib, rows):
    """Tile heights outside [8, 65536] are rejected before any device work
    (a height near INT_MAX would overflow the strip count)."""
    grids = (lib.rbgs_grid * 2)(_grid(lib, 15), _grid(lib, 31))
    ptrs = (ctypes.c_void_p * 2)(1 << 20, 2 << 20)  # never dereferenced: checks come first
    o = lib.rbgs_sweep_opts()
    o.tile_rows = rows
    rc = lib._lib.rbgs_sweep_batched(2, grids, lib.F32, ptrs, ptrs, 10, ctypes.byref(o), None, 0, None)
    assert rc == lib.EINVAL
    assert "tile_rows" in lib.rbgs_batch_last_error()


@pytest.mark.parametrize("case", ["n0", "dtype", "too_big"])
def test_residual_noalloc_validation_before_device_work(lib, case):
    """The no-allocation residual checks its arguments, and that the grid's
    partial sums fit its static scratch, before touching the device."""
    g, dtype = _grid(lib, 31), lib.F64
    if case == "n0":
        g = _grid(lib, 0)
    elif case == "dtype":
        dtype = 9
    elif case == "too_big":
        g = lib.rbgs_grid(32767, 32769, 1.0 / 32768)
    rc = lib._lib.rbgs_residual_noalloc(ctypes.byref(g), dtype, ctypes.c_void_p(256),
                                        ctypes.c_void_p(256), None, None, None)
    assert rc == lib.EINVAL
    if case == "too_big":
        assert "static scratch" in lib.rbgs_last_error()


def test_fallback_option_validation(lib):
    """The refinement's fallback flag is 0 or 1, and batches refuse it."""
    g = _grid(lib, 31)
    o = lib.rbgs_solve_opts()
    o.max_sweeps, o.rel_tol, o.check_every, o.omega = 10, 1e-8, 5, 1.0
    o.precision, o.fallback = lib.PREC_F32_IR, 2
    rc = lib._lib.rbgs_solve(ctypes.byref(g), lib.F64, None, None, ctypes.byref(o), None, None, 0,
                             None)
    assert rc == lib.EINVAL and "fallback" in lib.rbgs_last_error()
    grids = (lib.rbgs_grid * 2)(_grid(lib, 15), _grid(lib, 31))
    ptrs = (ctypes.c_void_p * 2)(1 << 20, 2 << 20)
    o.fallback, o.inner_sweeps = 1, 10
    rc = lib._lib.rbgs_solve_batched(2, grids, ptrs, ptrs, ctypes.byref(o), None, None, 0, None)
    assert rc == lib.EUNSUPPORTED and "fallback" in lib.rbgs_batch_last_error()


@pytest.mark.parametrize("field", ["debug_tile_order", "debug_stamp_check"])
def test_batched_rejects_verification_modes(lib, field):
    """The tile orders, stamp check and trace are single-grid modes."""
    grids = (lib.rbgs_grid * 2)(_grid(lib, 15), _grid(lib, 31))
    ptrs = (ctypes.c_void_p * 2)(1 << 20, 2 << 20)  # never dereferenced: checks come first
    o = lib.rbgs_sweep_opts()
    setattr(o, field, 1)
    rc = lib._lib.rbgs_sweep_batched(2, grids, lib.F32, ptrs, ptrs, 10, ctypes.byref(o), None, 0, None)
    assert rc == lib.EUNSUPPORTED
    assert "single-grid" in lib.rbgs_batch_last_error()


def test_status_strings_cover_every_code(lib):
    for code in (lib.OK, lib.EINVAL, lib.EHIP, lib.ENOCONV, lib.ETIMEOUT, lib.ENONFINITE,
                 lib.EUNSUPPORTED, lib.EWORKSPACE, lib.EORDER):
        assert "unknown" not in lib.rbgs_strerror(code)
