"""The blocked sweep's tile pipelines, run on the CPU, against the oracle.

The persistent kernel's device code (`csrc/blocked_pipeline.h`: tiles,
overlapped halos, the row pipeline of L half-sweeps, the LDS ring of h^2 f,
ping-pong buffers, progress flags and tickets) is compiled unchanged for
the host against a small stand-in for HIP's device features
(`tests/emu/hip/hip_runtime.h`: a workgroup = a wave of 64 lanes as fibers,
cross-lane operations and fences as wave barriers).  Since any schedule that honours the tile dependencies
computes the sequential red-black sweep (Section 2.3), the result must
equal the oracle's sweeps bit for bit.

* AddressSanitizer, one workgroup taking every ticket: no access may leave
  the arrays the library allocates.
* ThreadSanitizer, several workgroups as host threads sharing the tickets,
  progress flags and grid arrays through the device code's own atomics:
  every grid access must be ordered by the dependency protocol (a tile
  loads only rows of its 3 x 3 neighbourhood, after the flags say those
  tiles finished the pass before).  This is the check that found loads of
  rows beyond that neighbourhood in the input prefetch of short tiles
  (values that fed nothing stored, but raced with the writers of those
  rows); the loads are now clamped to the tile's region.
* A replay of a removed variant: inputs loaded four steps ahead, on the
  single-tile FP32 grid (n = 7, fuse 5) whose passes are handed between
  workgroups only through the progress flag and the ping-pong buffers.
* The verification modes of the persistent kernel: tiles of a pass taken in
  reversed and in seeded pseudo-random order (tickets stay pass-major), with
  the stamp check on (every neighbour has completed p or p + 1 passes
  around a pass-p item).  And the stamp check's own pin: with the
  dependency wait planted away (CPU build only), four workgroups in
  shuffled order must trip it.

The GPU tests check the same kernels on the device; these check their
indexing and ordering where a fault or a race can be located exactly.
"""
import os
import shutil
import subprocess

import numpy as np
import pytest

import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "tests", "emu", "tile_pipeline_emu.cpp")
INCLUDES = [os.path.join(ROOT, "tests", "emu"), os.path.join(ROOT, "paper_2607_01735_amd", "csrc"),
            os.path.join(ROOT, "include")]

# dtype, fuse, n, rows, passes, workgroups, sanitizer, prefetch steps (0 = the library's),
# tile order within a pass (0 as numbered; 1 reversed and 2 shuffled, both with the stamp check)
CASES = [
    (np.float64, 7, 63, 64, 2, 1, "address", 0, 0),     # one edge tile, taller than the grid
    (np.float64, 7, 520, 16, 2, 1, "address", 0, 0),    # 33 strips x 3 bands, interior tiles
    (np.float64, 1, 37, 8, 3, 1, "address", 0, 0),      # shallowest pipeline (L = 2), smallest ring
    (np.float32, 4, 1030, 16, 2, 1, "address", 0, 0),   # FP32 vectors of 4, interior tiles
    (np.float64, 2, 40, 8, 3, 3, "thread", 0, 0),       # three workgroups, short tiles
    (np.float64, 3, 150, 8, 3, 4, "thread", 0, 0),      # 19 strips x 2 bands, four workgroups
    (np.float64, 7, 130, 16, 3, 3, "thread", 0, 0),     # the 8191^2 depth, 9 strips x 2 bands
    (np.float32, 5, 7, 10, 3, 3, "thread", 4, 0),       # removed four-step prefetch, one tile
    (np.float32, 5, 7, 10, 3, 3, "thread", 0, 0),       # the kept depth on the same grid
    (np.float64, 3, 150, 8, 3, 4, "thread", 0, 1),      # reversed tile order, stamp check
    (np.float64, 2, 40, 8, 4, 3, "thread", 0, 2),       # shuffled tile order, stamp check
]

pytestmark = pytest.mark.skipif(shutil.which("g++") is None, reason="needs g++")


def _key(case):
    dtype, fuse, _, _, _, _, san, pre = case[:8]
    return (np.dtype(dtype).name, fuse, san, pre)


def _build(out, name, fuse, san, pre, extra=()):
    exe = out / (f"emu_{name}_{fuse}_{san}_{pre}" + "".join(d.split("=")[0] for d in extra))
    # no _FORTIFY_SOURCE: its longjmp check rejects the jumps between fiber stacks
    cmd = ["g++", "-std=c++17", "-O1", "-g", "-ffp-contract=off", "-U_FORTIFY_SOURCE",
           f"-fsanitize={san}", "-fno-omit-frame-pointer",
           f"-DEMU_T={'double' if name == 'float64' else 'float'}", f"-DEMU_FUSE={fuse}"]
    if pre:
        cmd.append(f"-DRBGS_EMU_PREFETCH_STEPS={pre}")
    cmd += [f"-D{d}" for d in extra]
    cmd += [f"-I{d}" for d in INCLUDES] + [SRC, "-o", str(exe), "-lpthread"]
    res = subprocess.run(cmd, capture_output=True, text=True)
    assert res.returncode == 0, res.stderr[-3000:]
    return exe


def _inputs(n, dtype):
    u0 = W.random_ring(n, seed=n)
    u0[1:n + 1, 1:n + 1] = W.uniform_rhs(n, seed=n + 1)[1:n + 1, 1:n + 1]
    f = W.uniform_rhs(n, seed=n + 2)
    return u0.astype(dtype), f.astype(dtype)


def _env(order):
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:detect_stack_use_after_return=0",
               TSAN_OPTIONS="halt_on_error=1:report_signal_unsafe=0")
    if order:
        env.update(EMU_TILE_ORDER=str(order), EMU_SEED="7", EMU_STAMP_CHECK="1")
    return env


@pytest.fixture(scope="module")
def emulators(tmp_path_factory):
    out = tmp_path_factory.mktemp("tile_emu")
    built = {}
    for case in CASES:
        key = _key(case)
        if key in built:
            continue
        name, fuse, san, pre = key
        built[key] = _build(out, name, fuse, san, pre)
    return out, built


@pytest.mark.slow
@pytest.mark.parametrize("case", CASES, ids=lambda c: "-".join(str(x) for x in _key(c)) +
                         f"-n{c[2]}-r{c[3]}-p{c[4]}-wg{c[5]}-o{c[8]}")
def test_tile_pipeline_matches_oracle(oracle, emulators, case):
    dtype, fuse, n, rows, passes, wgs, san, pre, order = case
    out, built = emulators
    h = W.spacing(n)
    u0, f = _inputs(n, dtype)
    assert u0.shape == (n + 2, n + 2) and f.shape == (n + 2, n + 2)
    tag = "-".join(str(x) for x in _key(case)) + f"_{n}_{wgs}_{order}"
    fin = out / f"in_{tag}.bin"
    fout = out / f"out_{tag}.bin"
    with open(fin, "wb") as fh:
        fh.write(np.ascontiguousarray(u0).tobytes())
        fh.write(np.ascontiguousarray(f).tobytes())
    res = subprocess.run([str(built[_key(case)]), str(n), str(rows), str(passes), repr(h),
                          str(fin), str(fout), str(wgs)], capture_output=True, text=True,
                         env=_env(order), timeout=600)
    assert res.returncode == 0, (res.stdout + res.stderr)[-4000:]
    assert "ThreadSanitizer" not in res.stderr, res.stderr[-4000:]
    got = np.fromfile(fout, dtype=dtype).reshape(n + 2, n + 2)
    ref = oracle.sweep(u0.copy(), f, h, passes * fuse)
    diff = got.view(np.uint8) != ref.view(np.uint8)
    assert not diff.any(), f"{int(diff.sum())} bytes differ; max |diff| " \
        f"{np.max(np.abs(got.astype(np.float64) - ref))}"


@pytest.mark.slow
def test_stamp_check_catches_a_missing_wait(tmp_path):
    """The stamp check's pin: the same emulation with the dependency wait
    taken out (planted on the CPU only) lets a tile run ahead of its
    neighbours; four workgroups taking a shuffled order must raise the
    error word's order code (2), which the library reports as RBGS_EORDER."""
    exe = _build(tmp_path, "float64", 2, "address", 0, extra=("RBGS_EMU_NO_WAIT",))
    n, passes = 40, 4
    u0, f = _inputs(n, np.float64)
    fin = tmp_path / "in.bin"
    with open(fin, "wb") as fh:
        fh.write(np.ascontiguousarray(u0).tobytes())
        fh.write(np.ascontiguousarray(f).tobytes())
    res = subprocess.run([str(exe), str(n), "8", str(passes), repr(W.spacing(n)), str(fin),
                          str(tmp_path / "out.bin"), "4"], capture_output=True, text=True,
                         env=_env(2), timeout=600)
    assert res.returncode == 4, (res.stdout + res.stderr)[-2000:]
    assert "error word (2)" in res.stderr


@pytest.mark.slow
@pytest.mark.parametrize("n,omega", [(150, 1.6), (7, 0.7)])
def test_sor_pipeline_matches_oracle(oracle, tmp_path, n, omega):
    """The SOR form of the pipeline (levels relax from each point's previous
    version; red read and written by every pass, the second buffer's
    interior poisoned with NaN) on four workgroups under ThreadSanitizer:
    the oracle's SOR sweeps bit for bit."""
    fuse, rows, passes = 3, 8, 3
    exe = _build(tmp_path, "float64", fuse, "thread", 0)
    u0, f = _inputs(n, np.float64)
    fin, fout = tmp_path / "in.bin", tmp_path / "out.bin"
    with open(fin, "wb") as fh:
        fh.write(np.ascontiguousarray(u0).tobytes())
        fh.write(np.ascontiguousarray(f).tobytes())
    h = W.spacing(n)
    res = subprocess.run([str(exe), str(n), str(rows), str(passes), repr(h), str(fin), str(fout), "4"],
                         capture_output=True, text=True, env=dict(_env(0), EMU_OMEGA=repr(omega)),
                         timeout=900)
    assert res.returncode == 0, (res.stdout + res.stderr)[-4000:]
    got = np.fromfile(fout, dtype=np.float64).reshape(n + 2, n + 2)
    ref = oracle.sor_sweep(u0.copy(), f, h, omega, passes * fuse)
    assert np.array_equal(got.view(np.uint8), ref.view(np.uint8))


@pytest.mark.slow
@pytest.mark.parametrize("fuse,n,rows,passes,split", [(7, 130, 16, 4, 2), (3, 150, 8, 3, 1)])
def test_merged_depths_match_oracle(oracle, tmp_path, fuse, n, rows, passes, split):
    """One launch whose passes differ in depth by one sweep (the first
    `split` passes fuse `fuse` sweeps, the rest one fewer, sharing the
    wave's LDS ring), three workgroups under ThreadSanitizer: the oracle's
    sweeps bit for bit."""
    exe = _build(tmp_path, "float64", fuse, "thread", 0, extra=("EMU_MERGED",))
    u0, f = _inputs(n, np.float64)
    fin, fout = tmp_path / "in.bin", tmp_path / "out.bin"
    with open(fin, "wb") as fh:
        fh.write(np.ascontiguousarray(u0).tobytes())
        fh.write(np.ascontiguousarray(f).tobytes())
    h = W.spacing(n)
    res = subprocess.run([str(exe), str(n), str(rows), str(passes), repr(h), str(fin), str(fout), "3"],
                         capture_output=True, text=True, env=dict(_env(0), EMU_SPLIT=str(split)),
                         timeout=1200)
    assert res.returncode == 0, (res.stdout + res.stderr)[-4000:]
    got = np.fromfile(fout, dtype=np.float64).reshape(n + 2, n + 2)
    ref = oracle.sweep(u0.copy(), f, h, split * fuse + (passes - split) * (fuse - 1))
    assert np.array_equal(got.view(np.uint8), ref.view(np.uint8))
