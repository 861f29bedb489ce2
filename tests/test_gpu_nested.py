"""Training targets of the learned guess: nested iteration on the GPU.

learned.nested_targets (FP32 batched sweeps and the library's grid
transfers) is compared with the same nested iteration composed on the CPU
from the oracle's FP64 sweep and the reference transfers: the two differ
only by FP32 rounding, bounded here by 2e-5 relative.  Both are also
compared with the oracle's fully converged solve (relative residual 1e-12),
which they must match to 5e-4 relative: the level sweep counts used here
leave 2-4e-4 in FP64 on these fields, measured against a direct solve.
"""
import numpy as np
import pytest

import workloads as W
from oracle import transfer_ref as T

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

import paper_2607_01735_amd as rb  # noqa: E402
from paper_2607_01735_amd import learned  # noqa: E402

N = 127
LEVELS = (2000, 1000, 1000)
SEEDS = (3, 4, 5)


def cpu_nested(oracle, f):
    rhs = [f]
    for _ in LEVELS[1:]:
        rhs.append(T.restrict(rhs[-1]))
    u = None
    for fl, sweeps in zip(rhs[::-1], LEVELS):
        n = fl.shape[0] - 2
        u = np.zeros_like(fl) if u is None else T.prolong(u)
        oracle.sweep(u, fl, 1.0 / (n + 1), sweeps)
    return u


def test_nested_targets_match_cpu_composition_and_converge(oracle):
    print(f"nested targets n={N} levels={LEVELS}", flush=True)
    f = np.stack([W.grf_rhs(N, seed=s)[0] for s in SEEDS])
    got = learned.nested_targets(rb, torch, torch.from_numpy(f).to("cuda"), LEVELS,
                                 chunk=2, tune=False).cpu().numpy()
    h = 1.0 / (N + 1)
    for b in range(len(SEEDS)):
        ref = cpu_nested(oracle, f[b])
        conv = np.zeros_like(f[b])
        status, _, rel = oracle.solve(conv, f[b], h, 200000, 1e-12, 1000)
        assert rel <= 1e-12
        scale = np.linalg.norm(conv)
        assert np.linalg.norm(got[b] - ref) / scale < 2e-5
        assert np.linalg.norm(ref - conv) / scale < 5e-4
        assert np.linalg.norm(got[b] - conv) / scale < 5e-4
        assert not np.any(got[b][0]) and not np.any(got[b][:, -1])
