"""The blocked sweep's tile pipeline, run on the CPU, against the oracle.

The persistent kernel's device code (`csrc/blocked_pipeline.h`: tiles,
overlapped halos, the row pipeline of L half-sweeps, the LDS ring of h^2 f,
ping-pong buffers, progress flags and tickets) is compiled unchanged for
the host against a small stand-in for HIP's device features
(`tests/emu/hip/hip_runtime.h`: one wave = 64 threads, cross-lane
operations through a barrier), with AddressSanitizer on every array, and
one emulated wave takes every ticket.  Since any schedule that honours the
tile dependencies computes the sequential red-black sweep (Section 2.3),
the result must equal the oracle's sweeps bit for bit, and no access may
leave the arrays the library allocates.  The GPU tests check the same
kernel on the device; this one checks its indexing where a fault can be
located exactly.
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

CASES = [  # dtype, fuse, n, rows, passes
    (np.float64, 7, 63, 64, 2),     # one edge tile, taller than the grid
    (np.float64, 7, 520, 16, 2),    # 33 strips x 3 bands, interior tiles in the middle band
    (np.float64, 1, 37, 8, 3),      # shallowest pipeline (L = 2), smallest ring
    (np.float32, 4, 1030, 16, 2),   # FP32 vectors of 4, interior tiles
]

pytestmark = pytest.mark.skipif(shutil.which("g++") is None, reason="needs g++")


@pytest.fixture(scope="module")
def emulators(tmp_path_factory):
    out = tmp_path_factory.mktemp("tile_emu")
    built = {}
    for dtype, fuse, *_ in CASES:
        key = (dtype, fuse)
        if key in built:
            continue
        exe = out / f"emu_{np.dtype(dtype).name}_{fuse}"
        # no _FORTIFY_SOURCE: its longjmp check rejects the jumps between fiber stacks
        cmd = ["g++", "-std=c++17", "-O1", "-g", "-ffp-contract=off", "-U_FORTIFY_SOURCE", "-fsanitize=address",
               "-fno-omit-frame-pointer",
               f"-DEMU_T={'double' if dtype == np.float64 else 'float'}", f"-DEMU_FUSE={fuse}"]
        cmd += [f"-I{d}" for d in INCLUDES] + [SRC, "-o", str(exe)]
        res = subprocess.run(cmd, capture_output=True, text=True)
        assert res.returncode == 0, res.stderr[-3000:]
        built[key] = exe
    return out, built


@pytest.mark.slow
@pytest.mark.parametrize("dtype,fuse,n,rows,passes", CASES)
def test_tile_pipeline_matches_oracle(oracle, emulators, dtype, fuse, n, rows, passes):
    out, built = emulators
    h = W.spacing(n)
    u0 = W.random_ring(n, seed=n)
    u0[1:n + 1, 1:n + 1] = W.uniform_rhs(n, seed=n + 1)[1:n + 1, 1:n + 1]
    f = W.uniform_rhs(n, seed=n + 2)
    u0, f = u0.astype(dtype), f.astype(dtype)
    assert u0.shape == (n + 2, n + 2) and f.shape == (n + 2, n + 2)
    fin = out / f"in_{n}_{fuse}.bin"
    fout = out / f"out_{n}_{fuse}.bin"
    with open(fin, "wb") as fh:
        fh.write(np.ascontiguousarray(u0).tobytes())
        fh.write(np.ascontiguousarray(f).tobytes())
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:detect_stack_use_after_return=0")
    res = subprocess.run([str(built[(dtype, fuse)]), str(n), str(rows), str(passes), repr(h),
                          str(fin), str(fout)], capture_output=True, text=True, env=env,
                         timeout=600)
    assert res.returncode == 0, (res.stdout + res.stderr)[-4000:]
    got = np.fromfile(fout, dtype=dtype).reshape(n + 2, n + 2)
    ref = oracle.sweep(u0.copy(), f, h, passes * fuse)
    diff = got.view(np.uint8) != ref.view(np.uint8)
    assert not diff.any(), f"{int(diff.sum())} bytes differ; max |diff| " \
        f"{np.max(np.abs(got.astype(np.float64) - ref))}"
