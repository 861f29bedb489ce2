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

# dtype, fuse, n, rows, passes, workgroups, sanitizer, prefetch steps (0 = the library's)
CASES = [
    (np.float64, 7, 63, 64, 2, 1, "address", 0),     # one edge tile, taller than the grid
    (np.float64, 7, 520, 16, 2, 1, "address", 0),    # 33 strips x 3 bands, interior tiles
    (np.float64, 1, 37, 8, 3, 1, "address", 0),      # shallowest pipeline (L = 2), smallest ring
    (np.float32, 4, 1030, 16, 2, 1, "address", 0),   # FP32 vectors of 4, interior tiles
    (np.float64, 2, 40, 8, 3, 3, "thread", 0),       # three workgroups, short tiles
    (np.float64, 3, 150, 8, 3, 4, "thread", 0),      # 19 strips x 2 bands, four workgroups
    (np.float64, 7, 130, 16, 3, 3, "thread", 0),     # the 8191^2 depth, 9 strips x 2 bands
    (np.float32, 5, 7, 10, 3, 3, "thread", 4),       # removed four-step prefetch, one tile
    (np.float32, 5, 7, 10, 3, 3, "thread", 0),       # the kept depth on the same grid
]

pytestmark = pytest.mark.skipif(shutil.which("g++") is None, reason="needs g++")


def _key(case):
    dtype, fuse, _, _, _, _, san, pre = case
    return (np.dtype(dtype).name, fuse, san, pre)


@pytest.fixture(scope="module")
def emulators(tmp_path_factory):
    out = tmp_path_factory.mktemp("tile_emu")
    built = {}
    for case in CASES:
        key = _key(case)
        if key in built:
            continue
        name, fuse, san, pre = key
        exe = out / f"emu_{name}_{fuse}_{san}_{pre}"
        # no _FORTIFY_SOURCE: its longjmp check rejects the jumps between fiber stacks
        cmd = ["g++", "-std=c++17", "-O1", "-g", "-ffp-contract=off", "-U_FORTIFY_SOURCE",
               f"-fsanitize={san}", "-fno-omit-frame-pointer",
               f"-DEMU_T={'double' if name == 'float64' else 'float'}", f"-DEMU_FUSE={fuse}"]
        if pre:
            cmd.append(f"-DRBGS_EMU_PREFETCH_STEPS={pre}")
        cmd += [f"-I{d}" for d in INCLUDES] + [SRC, "-o", str(exe), "-lpthread"]
        res = subprocess.run(cmd, capture_output=True, text=True)
        assert res.returncode == 0, res.stderr[-3000:]
        built[key] = exe
    return out, built


@pytest.mark.slow
@pytest.mark.parametrize("case", CASES, ids=lambda c: "-".join(str(x) for x in _key(c)) +
                         f"-n{c[2]}-r{c[3]}-p{c[4]}-wg{c[5]}")
def test_tile_pipeline_matches_oracle(oracle, emulators, case):
    dtype, fuse, n, rows, passes, wgs, san, pre = case
    out, built = emulators
    h = W.spacing(n)
    u0 = W.random_ring(n, seed=n)
    u0[1:n + 1, 1:n + 1] = W.uniform_rhs(n, seed=n + 1)[1:n + 1, 1:n + 1]
    f = W.uniform_rhs(n, seed=n + 2)
    u0, f = u0.astype(dtype), f.astype(dtype)
    assert u0.shape == (n + 2, n + 2) and f.shape == (n + 2, n + 2)
    tag = "-".join(str(x) for x in _key(case)) + f"_{n}_{wgs}"
    fin = out / f"in_{tag}.bin"
    fout = out / f"out_{tag}.bin"
    with open(fin, "wb") as fh:
        fh.write(np.ascontiguousarray(u0).tobytes())
        fh.write(np.ascontiguousarray(f).tobytes())
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:detect_stack_use_after_return=0",
               TSAN_OPTIONS="halt_on_error=1:report_signal_unsafe=0")
    res = subprocess.run([str(built[_key(case)]), str(n), str(rows), str(passes), repr(h),
                          str(fin), str(fout), str(wgs)], capture_output=True, text=True, env=env,
                         timeout=600)
    assert res.returncode == 0, (res.stdout + res.stderr)[-4000:]
    assert "ThreadSanitizer" not in res.stderr, res.stderr[-4000:]
    got = np.fromfile(fout, dtype=dtype).reshape(n + 2, n + 2)
    ref = oracle.sweep(u0.copy(), f, h, passes * fuse)
    diff = got.view(np.uint8) != ref.view(np.uint8)
    assert not diff.any(), f"{int(diff.sum())} bytes differ; max |diff| " \
        f"{np.max(np.abs(got.astype(np.float64) - ref))}"
