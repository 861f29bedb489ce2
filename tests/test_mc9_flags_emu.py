"""The flag-driven four-colour 9-point sweep, run on the CPU, against the oracle.

The kernel's device code (`csrc/mc9_flags.h`: the block geometry over the
(i >> 1, j >> 1) index grid, the ticket queue of (quarter-sweep, block)
items, the nine-counter dependency wait, the quarter-sweep of a block) is
compiled unchanged for the host against the stand-in for HIP's device
features in `tests/emu/hip`.  Any schedule that honours the block
dependencies computes the sequential four-colour sweep, so the result must
equal the oracle's 9-point sweeps bit for bit.  n = 1 and n = 2 have colours
with no interior point: every block still publishes every quarter-sweep, so
no wait lacks a producer.

* AddressSanitizer, one workgroup walking every block: no access may leave
  the arrays the library allocates (the row padding holds NaN, so a read of
  it would also change the result).
* ThreadSanitizer, several workgroups as host threads sharing the ticket,
  the counters and the grid through the device code's own atomics: every
  grid access must be ordered by the dependency rule (a block reads only its
  own and its eight neighbours' cells, after their counters say they
  finished the previous quarter-sweep).  Small block bounds and more blocks
  than workgroups cover every lane layout (8, 16, 32 and 64 columns per
  row); fewer workgroups than blocks per quarter-sweep is the case a
  schedule that needed every workgroup resident would hang on.
* The watchdog: a block that never publishes makes the waits on it expire;
  every workgroup leaves and the error word is raised.
"""
import os
import shutil
import subprocess

import numpy as np
import pytest

import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "tests", "emu", "mc9_flags_emu.cpp")
INCLUDES = [os.path.join(ROOT, "tests", "emu"), os.path.join(ROOT, "paper_2607_01735_amd", "csrc")]

# n, sweeps, max_blocks, workgroups, sanitizer, delay
CASES = [
    (1, 3, 64, 1, "address", 0),      # one point: colours 1, 2, 3 have none
    (2, 4, 64, 1, "address", 0),      # every colour one point
    (7, 4, 64, 1, "address", 0),      # 8 columns per row of lanes
    (40, 3, 64, 1, "address", 0),     # 32-lane rows, grown blocks
    (200, 2, 64, 1, "address", 0),    # two 64-lane column blocks
    (1, 3, 64, 3, "thread", 0),       # n = 1 with three workgroups
    (33, 5, 64, 4, "thread", 0),      # more blocks than workgroups
    (70, 3, 64, 6, "thread", 0),      # 64-lane rows, several tickets per workgroup
    (150, 2, 200, 8, "thread", 0),    # 8 workgroups
    (33, 3, 64, 4, "thread", 3),      # schedule stress: random stalls per block
]

pytestmark = pytest.mark.skipif(shutil.which("g++") is None, reason="needs g++")


def _build(out, san):
    exe = out / f"mc9_emu_{san}"
    # no _FORTIFY_SOURCE: its longjmp check rejects the jumps between fiber stacks
    cmd = ["g++", "-std=c++17", "-O1", "-g", "-ffp-contract=off", "-U_FORTIFY_SOURCE",
           f"-fsanitize={san}", "-fno-omit-frame-pointer"]
    cmd += [f"-I{d}" for d in INCLUDES] + [SRC, "-o", str(exe), "-lpthread"]
    res = subprocess.run(cmd, capture_output=True, text=True)
    assert res.returncode == 0, res.stderr[-3000:]
    return exe


@pytest.fixture(scope="module")
def emulators(tmp_path_factory):
    out = tmp_path_factory.mktemp("mc9_emu")
    return out, {san: _build(out, san) for san in ("address", "thread")}


def _env():
    return dict(os.environ, ASAN_OPTIONS="detect_leaks=0:detect_stack_use_after_return=0",
                TSAN_OPTIONS="halt_on_error=1:report_signal_unsafe=0")


def _inputs(n):
    u = W.random_ring(n, seed=400 + n)  # nonzero Dirichlet data, corners included
    u[1:n + 1, 1:n + 1] = W.uniform_rhs(n, seed=500 + n)[1:n + 1, 1:n + 1]
    f = W.uniform_rhs(n, seed=600 + n)
    return u, f


def _run(exe, out, n, sweeps, max_blocks, wgs, delay=0, stall=0):
    u, f = _inputs(n)
    tag = f"{n}_{sweeps}_{max_blocks}_{wgs}_{delay}_{stall}_{exe.name}"
    fin, fout = out / f"in_{tag}.bin", out / f"out_{tag}.bin"
    with open(fin, "wb") as fh:
        fh.write(u.tobytes())
        fh.write(f.tobytes())
    h = 1.0 / (n + 1)
    args = [str(exe), str(n), str(sweeps), repr(h), str(fin), str(fout), str(max_blocks), str(wgs)]
    if delay or stall:
        args += [str(delay), str(stall)]
    res = subprocess.run(args, capture_output=True, text=True, env=_env(), timeout=600)
    got = np.fromfile(fout, dtype=np.float64).reshape(u.shape) if res.returncode == 0 else None
    return res, u, f, h, got


@pytest.mark.slow
@pytest.mark.parametrize("case", CASES, ids=lambda c: f"n{c[0]}-s{c[1]}-b{c[2]}-wg{c[3]}-{c[4]}-d{c[5]}")
def test_mc9_flags_matches_oracle(oracle, emulators, case):
    n, sweeps, max_blocks, wgs, san, delay = case
    out, exes = emulators
    res, u, f, h, got = _run(exes[san], out, n, sweeps, max_blocks, wgs, delay)
    assert res.returncode == 0, res.stdout + res.stderr[-4000:]
    # the block shape the kernel used covers the interior exactly, its lanes
    # split rows evenly, and the block count fits the bound
    import re
    m = re.search(r"qw=(\d+) ri=(\d+) blocks=(\d+) \((\d+) x (\d+)\) rows=(\d+) cols=(\d+)",
                  res.stdout)
    qw, ri, nb, ib, qb, rows, cols = map(int, m.groups())
    assert rows == cols == (n + 1) // 2 + 1
    assert nb == ib * qb and (nb <= max_blocks or ri >= rows)
    assert ri % (64 // qw) == 0 and (qb - 1) * qw < cols <= qb * qw
    assert (ib - 1) * ri < rows <= ib * ri
    ref = u.copy()
    oracle.mc9_sweep(ref, f, h, sweeps)
    assert np.array_equal(got.view(np.uint64), ref.view(np.uint64)), \
        f"max diff {np.nanmax(np.abs(got - ref))}; {res.stdout}"


@pytest.mark.slow
def test_mc9_flags_watchdog(emulators):
    """Block 0 never publishes: its neighbours' waits expire, the error word
    is raised and every workgroup leaves (exit status 4, no hang)."""
    out, exes = emulators
    res, *_ = _run(exes["thread"], out, 33, 3, 64, 4, delay=0, stall=1)
    assert res.returncode == 4, res.stdout + res.stderr[-2000:]
    assert "error word" in res.stderr
