"""Oracle for red-black Gauss-Seidel (test infrastructure only).

Only the tests, the smoke check and the benchmark's CPU-baseline leg may
import this package.  It wraps the plain C oracle (rbgs_oracle.c) for numpy
arrays in the natural layout: an (n+2) x ld row-major array whose ring (row 0,
row n+1, column 0, column n+1) holds the Dirichlet data g.  Nothing here is
shared with, or imported by, the GPU library.

Paper anchors: the point update is Eq. (1) of Section 2; the colouring (red
when i+j is even) is stated in Section 2; one sweep is the red half-sweep
then the black half-sweep, as in Algorithms 1 and 2.
"""
import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None

OK = 0
EINVAL = -1
ENOCONV = -3

_i32 = ctypes.c_int32
_i64 = ctypes.c_int64
_f64 = ctypes.c_double
_vp = ctypes.c_void_p


def _load(path=None):
    """Load liboracle.so (building it if absent).  path: load another build
    of the same source instead (the tests use this for planted mistakes)."""
    global _lib
    if _lib is not None and path is None:
        return _lib
    if path is None and not os.path.exists(_LIB_PATH):
        from . import build as _build
        _build.build()
    lib = ctypes.CDLL(path or _LIB_PATH)
    sig = {
        "rbgs_ref_half_sweep_f64": [_i32, _i64, _f64, _vp, _vp, _i32],
        "rbgs_ref_sweep_f64": [_i32, _i64, _f64, _vp, _vp, _i32],
        "rbgs_ref_half_sweep_f32": [_i32, _i64, _f64, _vp, _vp, _i32],
        "rbgs_ref_sweep_f32": [_i32, _i64, _f64, _vp, _vp, _i32],
        "rbgs_ref_residual_f64": [_i32, _i64, _f64, _vp, _vp, _vp, _vp, _vp],
        "rbgs_ref_residual_f32": [_i32, _i64, _f64, _vp, _vp, _vp, _vp, _vp],
        "rbgs_ref_solve_f64": [_i32, _i64, _f64, _vp, _vp, _i32, _f64, _i32, _vp, _vp],
        "rbgs_ref_ir_solve": [_i32, _i64, _f64, _vp, _vp, _i32, _i32, _i32, _f64, _vp, _vp],
        "rbgs_ref_ir_solve_fallback": [_i32, _i64, _f64, _vp, _vp, _i32, _i32, _i32, _f64, _vp,
                                       _vp, _vp, _vp],
        "rbgs_ref_colour": [_i64, _i64],
        "rbgs_ref_sor_half_sweep_f64": [_i32, _i64, _f64, _f64, _vp, _vp, _i32],
        "rbgs_ref_sor_sweep_f64": [_i32, _i64, _f64, _f64, _vp, _vp, _i32],
        "rbgs_ref_sor_solve_f64": [_i32, _i64, _f64, _f64, _vp, _vp, _i32, _f64, _i32, _vp, _vp],
        "rbgs_ref_mg_levels": [_i32, _i32, _vp],
        "rbgs_ref_mc9_colour": [_i64, _i64],
        "rbgs_ref_rb3_half_sweep_f64": [_i32, _i64, _f64, _vp, _vp, _i32],
        "rbgs_ref_rb3_sweep_f64": [_i32, _i64, _f64, _vp, _vp, _i32],
        "rbgs_ref_rb3_residual_f64": [_i32, _i64, _f64, _vp, _vp, _vp, _vp, _vp],
        "rbgs_ref_rb3_solve_f64": [_i32, _i64, _f64, _vp, _vp, _i32, _f64, _i32, _vp, _vp],
        "rbgs_ref_mc9_quarter_sweep_f64": [_i32, _i64, _f64, _vp, _vp, _i32],
        "rbgs_ref_mc9_sweep_f64": [_i32, _i64, _f64, _vp, _vp, _i32],
        "rbgs_ref_mc9_residual_f64": [_i32, _i64, _f64, _vp, _vp, _vp, _vp, _vp],
        "rbgs_ref_mc9_solve_f64": [_i32, _i64, _f64, _vp, _vp, _i32, _f64, _i32, _vp, _vp],
        "rbgs_ref_mg_restrict_f64": [_i32, _vp, _i64, _vp, _i64],
        "rbgs_ref_mg_prolong_add_f64": [_i32, _vp, _i64, _vp, _i64],
        "rbgs_ref_mg_solve_f64": [_i32, _i64, _f64, _vp, _vp, _i32, _i32, _i32, _i32, _i32, _f64,
                                  _vp, _vp],
    }
    for name, args in sig.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = _i32
    lib.rbgs_ref_threads.argtypes = []
    lib.rbgs_ref_threads.restype = _i32
    lib.rbgs_ref_round_bf16.argtypes = [ctypes.c_float]
    lib.rbgs_ref_round_bf16.restype = ctypes.c_float
    if path is None:
        _lib = lib
    return lib


class use_library:
    """Context manager: route every call of this module to another build of
    the oracle source (used to check that the pins catch planted mistakes)."""

    def __init__(self, path):
        self.path = path

    def __enter__(self):
        global _lib
        self.saved = _lib
        _lib = _load(self.path)
        return self

    def __exit__(self, *exc):
        global _lib
        _lib = self.saved
        return False


def _grid(a):
    if a.ndim != 2 or a.shape[0] < 3 or a.shape[1] < a.shape[0]:
        raise ValueError("expected an (n+2) x ld array with ld >= n+2")
    if not a.flags.c_contiguous:
        raise ValueError("array must be C-contiguous")
    return a.shape[0] - 2, a.shape[1]


def _ptr(a):
    return ctypes.c_void_p(a.ctypes.data)


def _check(rc, name):
    if rc not in (OK, ENOCONV):
        raise RuntimeError(f"{name} returned {rc}")
    return rc


def half_sweep(u, f, h, colour):
    """One half-sweep in place; colour 0 = red (i+j even), 1 = black."""
    n, ld = _grid(u)
    if u.dtype == np.float64:
        assert f.dtype == np.float64 and f.shape == u.shape
        _check(_load().rbgs_ref_half_sweep_f64(n, ld, h, _ptr(u), _ptr(f), colour), "half_sweep_f64")
    elif u.dtype == np.float32:
        assert f.dtype == np.float32 and f.shape == u.shape
        _check(_load().rbgs_ref_half_sweep_f32(n, ld, h, _ptr(u), _ptr(f), colour), "half_sweep_f32")
    else:
        raise TypeError(u.dtype)
    return u


def sweep(u, f, h, nsweeps):
    """nsweeps full red-then-black sweeps in place (FP64, or FP32 emulation)."""
    n, ld = _grid(u)
    if u.dtype == np.float64:
        assert f.dtype == np.float64 and f.shape == u.shape
        _check(_load().rbgs_ref_sweep_f64(n, ld, h, _ptr(u), _ptr(f), nsweeps), "sweep_f64")
    elif u.dtype == np.float32:
        assert f.dtype == np.float32 and f.shape == u.shape
        _check(_load().rbgs_ref_sweep_f32(n, ld, h, _ptr(u), _ptr(f), nsweeps), "sweep_f32")
    else:
        raise TypeError(u.dtype)
    return u


def residual(u, f, h, want_field=False):
    """(||r||_2, ||r||_2/||b||_2[, r]) in FP64 with compensated sums."""
    n, ld = _grid(u)
    a = _f64()
    r = _f64()
    field = np.zeros(u.shape, np.float64) if want_field else None
    fp = _ptr(field) if want_field else None
    if u.dtype == np.float64:
        fn = _load().rbgs_ref_residual_f64
    elif u.dtype == np.float32:
        fn = _load().rbgs_ref_residual_f32
    else:
        raise TypeError(u.dtype)
    assert f.dtype == u.dtype and f.shape == u.shape
    _check(fn(n, ld, h, _ptr(u), _ptr(f), ctypes.byref(a), ctypes.byref(r), fp), "residual")
    if want_field:
        return a.value, r.value, field
    return a.value, r.value


def solve(u, f, h, max_sweeps, rel_tol, check_every):
    """Sweeps until rel <= rel_tol (checked every check_every sweeps).

    Returns (status, sweeps_done, rel)."""
    n, ld = _grid(u)
    assert u.dtype == np.float64 and f.dtype == np.float64
    done = _i32()
    rel = _f64()
    rc = _check(_load().rbgs_ref_solve_f64(n, ld, h, _ptr(u), _ptr(f), max_sweeps, rel_tol,
                                           check_every, ctypes.byref(done), ctypes.byref(rel)),
                "solve_f64")
    return rc, done.value, rel.value


def ir_solve(u, f, h, inner_sweeps, max_outer, rel_tol, rhs_bf16=False):
    """FP64 iterative refinement around FP32 inner sweeps.

    Returns (status, outer_steps, rel)."""
    n, ld = _grid(u)
    assert u.dtype == np.float64 and f.dtype == np.float64
    outer = _i32()
    rel = _f64()
    rc = _check(_load().rbgs_ref_ir_solve(n, ld, h, _ptr(u), _ptr(f), 1 if rhs_bf16 else 0,
                                          inner_sweeps, max_outer, rel_tol,
                                          ctypes.byref(outer), ctypes.byref(rel)),
                "ir_solve")
    return rc, outer.value, rel.value


def ir_solve_fallback(u, f, h, inner_sweeps, max_sweeps, rel_tol, rhs_bf16=False):
    """Refinement whose inner precision widens when it stalls or overflows
    (bfloat16 rhs -> binary32 -> FP64 sweeps).

    Returns (status, outer_steps, sweeps, rel, precision) with precision
    0 = FP64 sweeps, 1 = binary32, 2 = bfloat16 rhs at the end."""
    n, ld = _grid(u)
    assert u.dtype == np.float64 and f.dtype == np.float64
    outer, done, prec = _i32(), _i32(), _i32()
    rel = _f64()
    rc = _check(_load().rbgs_ref_ir_solve_fallback(
        n, ld, h, _ptr(u), _ptr(f), 1 if rhs_bf16 else 0, inner_sweeps, max_sweeps, rel_tol,
        ctypes.byref(outer), ctypes.byref(done), ctypes.byref(rel), ctypes.byref(prec)),
        "ir_solve_fallback")
    return rc, outer.value, done.value, rel.value, prec.value


def omega_opt(n):
    """Optimal SOR factor of the model problem, 2 / (1 + sin(pi h)), h = 1/(n+1)."""
    import math
    return 2.0 / (1.0 + math.sin(math.pi / (n + 1)))


def sor_sweep(u, f, h, omega, nsweeps):
    """nsweeps red-black SOR sweeps in place (FP64)."""
    n, ld = _grid(u)
    assert u.dtype == np.float64 and f.dtype == np.float64 and f.shape == u.shape
    _check(_load().rbgs_ref_sor_sweep_f64(n, ld, h, omega, _ptr(u), _ptr(f), nsweeps),
           "sor_sweep_f64")
    return u


def sor_solve(u, f, h, omega, max_sweeps, rel_tol, check_every):
    """SOR sweeps until rel <= rel_tol (checked every check_every sweeps).

    Returns (status, sweeps_done, rel)."""
    n, ld = _grid(u)
    assert u.dtype == np.float64 and f.dtype == np.float64
    done = _i32()
    rel = _f64()
    rc = _check(_load().rbgs_ref_sor_solve_f64(n, ld, h, omega, _ptr(u), _ptr(f), max_sweeps,
                                               rel_tol, check_every, ctypes.byref(done),
                                               ctypes.byref(rel)), "sor_solve_f64")
    return rc, done.value, rel.value


def mg_levels(n, max_levels=0):
    """Grid sizes of the multigrid hierarchy: n, then (n - 1) / 2 while odd
    and >= 3 (at most max_levels levels when max_levels > 0)."""
    sizes = (ctypes.c_int32 * 32)()
    cnt = _load().rbgs_ref_mg_levels(n, max_levels, sizes)
    if cnt < 1:
        raise ValueError("bad multigrid level request")
    return [sizes[k] for k in range(cnt)]


def mg_default_coarse_sweeps(nc):
    """Sweeps on the coarsest level when the caller leaves the count at 0:
    one when it is a single point (exact), else 2 (nc + 1)^2, enough to bring
    a coarse error down by about e^-20 (Gauss-Seidel's rate 1 - pi^2 h^2)."""
    return 1 if nc == 1 else 2 * (nc + 1) * (nc + 1)


def mg_restrict(r):
    """Full weighting of an (n_f+2)^2 natural-layout field onto a new
    (n_c+2)^2 array (zero ring), n_f = 2 n_c + 1."""
    nf = r.shape[0] - 2
    if nf < 3 or nf % 2 == 0:
        raise ValueError("fine size must be 2 n_c + 1")
    nc = (nf - 1) // 2
    r = np.ascontiguousarray(r, np.float64)
    out = np.zeros((nc + 2, nc + 2))
    _check(_load().rbgs_ref_mg_restrict_f64(nc, _ptr(r), r.shape[1], _ptr(out), out.shape[1]),
           "mg_restrict")
    return out


def mg_prolong_add(ec, u):
    """u += bilinear prolongation of the coarse array ec (ring included), in
    place at the interior of u."""
    nc = ec.shape[0] - 2
    ec = np.ascontiguousarray(ec, np.float64)
    n, ld = _grid(u)
    if n != 2 * nc + 1:
        raise ValueError("fine size must be 2 n_c + 1")
    assert u.dtype == np.float64
    _check(_load().rbgs_ref_mg_prolong_add_f64(nc, _ptr(ec), ec.shape[1], _ptr(u), ld),
           "mg_prolong_add")
    return u


def mg_solve(u, f, h, nu1, nu2, max_cycles, rel_tol, max_levels=0, coarse_sweeps=0):
    """V-cycles with red-black Gauss-Seidel smoothing until rel <= rel_tol
    (checked before the first cycle and after each).  coarse_sweeps = 0 takes
    mg_default_coarse_sweeps of the coarsest size.  Returns (status, cycles,
    rel)."""
    n, ld = _grid(u)
    assert u.dtype == np.float64 and f.dtype == np.float64 and f.shape == u.shape
    if coarse_sweeps == 0:
        coarse_sweeps = mg_default_coarse_sweeps(mg_levels(n, max_levels)[-1])
    cyc = _i32()
    rel = _f64()
    rc = _check(_load().rbgs_ref_mg_solve_f64(n, ld, h, _ptr(u), _ptr(f), nu1, nu2, max_levels,
                                              coarse_sweeps, max_cycles, rel_tol,
                                              ctypes.byref(cyc), ctypes.byref(rel)),
                "mg_solve_f64")
    return rc, cyc.value, rel.value


def mc9_colour(i, j):
    """Colour of point (i, j) for the 9-point stencil: (i & 1) + 2 (j & 1)."""
    return _load().rbgs_ref_mc9_colour(i, j)


def mc9_quarter_sweep(u, f, h, colour):
    """Update every interior point of one of the four colours, in place."""
    n, ld = _grid(u)
    assert u.dtype == np.float64 and f.dtype == np.float64 and f.shape == u.shape
    _check(_load().rbgs_ref_mc9_quarter_sweep_f64(n, ld, h, _ptr(u), _ptr(f), colour),
           "mc9_quarter_sweep")
    return u


def mc9_sweep(u, f, h, nsweeps):
    """nsweeps 4-colour 9-point Gauss-Seidel sweeps (colours 0..3) in place."""
    n, ld = _grid(u)
    assert u.dtype == np.float64 and f.dtype == np.float64 and f.shape == u.shape
    _check(_load().rbgs_ref_mc9_sweep_f64(n, ld, h, _ptr(u), _ptr(f), nsweeps), "mc9_sweep")
    return u


def mc9_residual(u, f, h, want_field=False):
    """(||r||_2, ||r||_2/||b||_2[, r]) of the 9-point system in FP64."""
    n, ld = _grid(u)
    assert u.dtype == np.float64 and f.dtype == np.float64 and f.shape == u.shape
    a, r = _f64(), _f64()
    field = np.zeros(u.shape, np.float64) if want_field else None
    _check(_load().rbgs_ref_mc9_residual_f64(n, ld, h, _ptr(u), _ptr(f), ctypes.byref(a),
                                             ctypes.byref(r), _ptr(field) if want_field else None),
           "mc9_residual")
    return (a.value, r.value, field) if want_field else (a.value, r.value)


def mc9_solve(u, f, h, max_sweeps, rel_tol, check_every):
    """4-colour 9-point sweeps until rel <= rel_tol.  Returns (status, sweeps, rel)."""
    n, ld = _grid(u)
    assert u.dtype == np.float64 and f.dtype == np.float64
    done, rel = _i32(), _f64()
    rc = _check(_load().rbgs_ref_mc9_solve_f64(n, ld, h, _ptr(u), _ptr(f), max_sweeps, rel_tol,
                                               check_every, ctypes.byref(done),
                                               ctypes.byref(rel)), "mc9_solve")
    return rc, done.value, rel.value


def _grid3(a):
    if a.ndim != 3 or a.shape[0] < 3 or a.shape[1] != a.shape[0] or a.shape[2] < a.shape[0]:
        raise ValueError("expected an (n+2) x (n+2) x ld array with ld >= n+2")
    if not a.flags.c_contiguous or a.dtype != np.float64:
        raise ValueError("array must be C-contiguous float64")
    return a.shape[0] - 2, a.shape[2]


def rb3_half_sweep(u, f, h, colour):
    """One 3D red-black half-sweep in place; colour 0 = red (i+j+k even)."""
    n, ld = _grid3(u)
    assert f.shape == u.shape
    _check(_load().rbgs_ref_rb3_half_sweep_f64(n, ld, h, _ptr(u), _ptr(f), colour), "rb3_half")
    return u


def rb3_sweep(u, f, h, nsweeps):
    """nsweeps 3D red-black sweeps (7-point Laplacian) in place."""
    n, ld = _grid3(u)
    assert f.shape == u.shape
    _check(_load().rbgs_ref_rb3_sweep_f64(n, ld, h, _ptr(u), _ptr(f), nsweeps), "rb3_sweep")
    return u


def rb3_residual(u, f, h, want_field=False):
    """(||r||_2, ||r||_2/||b||_2[, r]) of the 3D 7-point system in FP64."""
    n, ld = _grid3(u)
    assert f.shape == u.shape and f.dtype == np.float64
    a, r = _f64(), _f64()
    field = np.zeros(u.shape, np.float64) if want_field else None
    _check(_load().rbgs_ref_rb3_residual_f64(n, ld, h, _ptr(u), _ptr(f), ctypes.byref(a),
                                             ctypes.byref(r), _ptr(field) if want_field else None),
           "rb3_residual")
    return (a.value, r.value, field) if want_field else (a.value, r.value)


def rb3_solve(u, f, h, max_sweeps, rel_tol, check_every):
    """3D red-black sweeps until rel <= rel_tol.  Returns (status, sweeps, rel)."""
    n, ld = _grid3(u)
    done, rel = _i32(), _f64()
    rc = _check(_load().rbgs_ref_rb3_solve_f64(n, ld, h, _ptr(u), _ptr(f), max_sweeps, rel_tol,
                                               check_every, ctypes.byref(done),
                                               ctypes.byref(rel)), "rb3_solve")
    return rc, done.value, rel.value


def threads():
    """OpenMP threads the oracle's parallel loops use."""
    return int(_load().rbgs_ref_threads())


def round_bf16(x):
    """binary32 -> bfloat16 (round to nearest even) -> binary32, elementwise."""
    fn = _load().rbgs_ref_round_bf16
    flat = np.asarray(x, np.float32).ravel()
    out = np.array([fn(float(v)) for v in flat], np.float32)
    return out.reshape(np.shape(x))


def colour(i, j):
    return _load().rbgs_ref_colour(i, j)


def sweep_batched(us, fs, hs, nsweeps):
    """Independent sweeps of many grids: a plain loop over sweep()."""
    for u, f, h in zip(us, fs, hs):
        sweep(u, f, h, nsweeps)
    return us
