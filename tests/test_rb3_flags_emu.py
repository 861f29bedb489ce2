"""The flag-driven 3D sweep, run on the CPU, against the oracle.

The kernel's device code (`csrc/rb3_flags.h`: the block geometry, the
level-by-level walk of each wave's blocks, the seven-counter dependency wait,
the plane-marching half-sweep of a block, with either plane chunk) is
compiled unchanged for the host against the stand-in for HIP's device
features in `tests/emu/hip`.  Any
schedule that honours the block dependencies computes the sequential
red-black sweep, so the result must equal the oracle's 3D sweeps bit for bit.

* AddressSanitizer, one workgroup walking every block: no access may leave
  the arrays the library allocates (the row padding holds NaN, so a read of
  it would also change the result).
* ThreadSanitizer, several workgroups as host threads sharing the ticket,
  the counters and the grid through the device code's own atomics: every
  grid access must be ordered by the dependency rule (a block reads only its
  own and its six face neighbours' cells, after their counters say they
  finished the previous half-sweep).  Small block bounds and more blocks
  than workgroups cover every lane layout (8, 16, 32 and 64 q-columns per
  row); fewer workgroups than blocks per half-sweep is the case a
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
SRC = os.path.join(ROOT, "tests", "emu", "rb3_flags_emu.cpp")
INCLUDES = [os.path.join(ROOT, "tests", "emu"), os.path.join(ROOT, "paper_2607_01735_amd", "csrc")]

# n, sweeps, max_blocks, workgroups, sanitizer, delay, plane chunk
CASES = [
    (1, 3, 64, 1, "address", 0, "deep"),      # one block, 8-lane rows, a single point
    (7, 4, 64, 1, "address", 0, "deep"),      # 8 q-columns of 8 rows per step
    (20, 3, 64, 1, "address", 0, "deep"),     # 16-lane rows, grown blocks
    (37, 2, 64, 1, "address", 0, "deep"),     # 32-lane rows
    (70, 2, 64, 1, "address", 0, "deep"),     # two 64-lane q-blocks
    (9, 5, 64, 4, "thread", 0, "deep"),       # 4 workgroups, more blocks than workgroups
    (21, 3, 64, 5, "thread", 0, "deep"),      # several tickets per workgroup
    (40, 3, 200, 8, "thread", 0, "deep"),     # 32-lane rows, 8 waves
    (66, 2, 64, 6, "thread", 0, "deep"),      # 64-lane rows, two q-blocks
    (21, 3, 64, 4, "thread", 3, "deep"),      # schedule stress: random stalls per block
    (20, 3, 64, 1, "address", 0, "lean"),     # the lean plane chunk
    (37, 2, 64, 1, "address", 0, "lean"),     # 16 + 16 + 5 planes: a chunk cut short
    (40, 3, 200, 8, "thread", 0, "lean"),
    (21, 3, 64, 4, "thread", 3, "lean"),
]

pytestmark = pytest.mark.skipif(shutil.which("g++") is None, reason="needs g++")


def _build(out, san):
    exe = out / f"rb3_emu_{san}"
    # no _FORTIFY_SOURCE: its longjmp check rejects the jumps between fiber stacks
    cmd = ["g++", "-std=c++17", "-O1", "-g", "-ffp-contract=off", "-U_FORTIFY_SOURCE",
           f"-fsanitize={san}", "-fno-omit-frame-pointer"]
    cmd += [f"-I{d}" for d in INCLUDES] + [SRC, "-o", str(exe), "-lpthread"]
    res = subprocess.run(cmd, capture_output=True, text=True)
    assert res.returncode == 0, res.stderr[-3000:]
    return exe


@pytest.fixture(scope="module")
def emulators(tmp_path_factory):
    out = tmp_path_factory.mktemp("rb3_emu")
    return out, {san: _build(out, san) for san in ("address", "thread")}


def _env():
    return dict(os.environ, ASAN_OPTIONS="detect_leaks=0:detect_stack_use_after_return=0",
                TSAN_OPTIONS="halt_on_error=1:report_signal_unsafe=0")


def _inputs(n):
    rng = np.random.default_rng(300 + n)
    u = np.zeros((n + 2,) * 3)
    u[1:-1, 1:-1, 1:-1] = rng.uniform(-1, 1, (n,) * 3)
    for face in (np.s_[0], np.s_[-1]):  # nonzero Dirichlet data on all six faces
        u[face] = rng.uniform(-1, 1, (n + 2, n + 2))
        u[:, face] = rng.uniform(-1, 1, (n + 2, n + 2))
        u[:, :, face] = rng.uniform(-1, 1, (n + 2, n + 2))
    f = np.zeros_like(u)
    f[1:-1, 1:-1, 1:-1] = rng.uniform(-1, 1, (n,) * 3)
    return u, f


def _run(exe, out, n, sweeps, max_blocks, wgs, delay=0, stall=0, chunk="deep"):
    u, f = _inputs(n)
    tag = f"{n}_{sweeps}_{max_blocks}_{wgs}_{delay}_{stall}_{chunk}_{exe.name}"
    fin, fout = out / f"in_{tag}.bin", out / f"out_{tag}.bin"
    with open(fin, "wb") as fh:
        fh.write(u.tobytes())
        fh.write(f.tobytes())
    h = 1.0 / (n + 1)
    args = [str(exe), str(n), str(sweeps), repr(h), str(fin), str(fout), str(max_blocks), str(wgs)]
    if delay or stall:
        args += [str(delay), str(stall)]
    res = subprocess.run(args, capture_output=True, text=True, env=dict(_env(), EMU_CHUNK=chunk),
                         timeout=600)
    got = np.fromfile(fout, dtype=np.float64).reshape(u.shape) if res.returncode == 0 else None
    return res, u, f, h, got


@pytest.mark.slow
@pytest.mark.parametrize("case", CASES,
                         ids=lambda c: f"n{c[0]}-s{c[1]}-b{c[2]}-wg{c[3]}-{c[4]}-d{c[5]}-{c[6]}")
def test_rb3_flags_matches_oracle(oracle, emulators, case):
    n, sweeps, max_blocks, wgs, san, delay, chunk = case
    out, exes = emulators
    res, u, f, h, got = _run(exes[san], out, n, sweeps, max_blocks, wgs, delay, chunk=chunk)
    assert res.returncode == 0, res.stdout + res.stderr[-4000:]
    assert f"chunk={chunk}" in res.stdout
    # the block shape the kernel used covers the interior exactly, its lanes
    # split rows evenly, and the block count fits the bound
    import re
    m = re.search(r"qw=(\d+) rj=(\d+) rz=(\d+) blocks=(\d+) \((\d+) x (\d+) x (\d+)\)", res.stdout)
    qw, rj, rz, nb, qb, jb, zb = map(int, m.groups())
    qs = n // 2 + 1
    assert nb == qb * jb * zb and (nb <= max_blocks or (rj >= n and rz >= n))
    assert rj % (64 // qw) == 0 and (qb - 1) * qw < qs <= qb * qw
    assert (jb - 1) * rj < n <= jb * rj and (zb - 1) * rz < n <= zb * rz
    ref = u.copy()
    oracle.rb3_sweep(ref, f, h, sweeps)
    assert np.array_equal(got.view(np.uint64), ref.view(np.uint64)), \
        f"max diff {np.nanmax(np.abs(got - ref))}; {res.stdout}"


@pytest.mark.slow
def test_rb3_flags_watchdog(emulators):
    """Block 0 never publishes: its neighbours' waits expire, the error word
    is raised and every workgroup leaves (exit status 4, no hang)."""
    out, exes = emulators
    res, *_ = _run(exes["thread"], out, 21, 3, 64, 4, delay=0, stall=1)
    assert res.returncode == 4, res.stdout + res.stderr[-2000:]
    assert "error word" in res.stderr
