"""GPU parity on shapes chosen to reach every default pass A tiling the
library picks by itself: 4-block tasks with deferred stores (rows of >= 512
column groups whose 4-block tasks fill one round of CUs), the packed table
in 1024-lane workgroups (>= 512 groups, >= 256 tasks), the lane table at 256
lanes per row
(256..511 groups), blocks side by side (narrow rows with >= 256 tasks), and
row phases with the shared table (small problems). Each shape runs two calls
(stream state) against the oracle, with a seeded window and estimator."""
from types import SimpleNamespace

import numpy as np
import pytest

import oracle
import synth
from parity import check_result

torch = pytest.importorskip("torch")
sk = pytest.importorskip("paper_1808_10365_amd")

pytestmark = pytest.mark.gpu
DEV = "cuda:0"

# (N, F, M, blocks per call, expected default lanes per row)
SHAPES = [
    (2048, 4, 4, 1024, 512),     # 512 groups, 1024 blocks: 4-block tasks, stores deferred
    (4096, 2, 4, 900, 512),      # the same with a partial last task
    (2048, 4, 16, 256, 1024),    # 512 groups, 256 tasks: packed, 1024 lanes
    (4096, 4, 8, 300, 1024),     # 1024 groups
    (4096, 8, 8, 260, 1024),     # 2048 groups: two 1024-lane chunks per block
    (1024, 4, 8, 256, 256),      # 256 groups: lane table, 256 lanes
    (2048, 3, 16, 192, 256),     # 384 groups, too few blocks for 1024 lanes
    (256, 8, 8, 512, 128),       # 128 groups: 2 blocks side by side
    (64, 1, 2, 16384, 4),        # 4 groups: 64 blocks side by side
    (48, 5, 4, 4096, 16),        # 15 groups padded to 16 lanes, 16 blocks side by side
    (48, 5, 4, 2000, 16),        # the same rows with too few tasks: row phases of 16 lanes
    (16, 1, 256, 16, None),      # tiny: row phases
    (256, 4, 256, 192, 16),      # serving N=256 frame shape: 16 lanes, 16 row phases, 768 workgroups
    (1024, 4, 8, 16, 32),        # 256 groups, 16 blocks: row phases stop at the block's 8 rows
    (2048, 4, 4, 8, 64),         # 512 groups, 8 blocks of 4 rows: 64 lanes (4 phases)
]


@pytest.mark.parametrize("k", range(len(SHAPES)))
def test_default_tile_shapes(k):
    N, F, M, B, want_lpr = SHAPES[k]
    rng = np.random.default_rng(500 + k)
    L = int(rng.choice([0, 1, 2, 7, 64]))
    est = 1 if (L == 1 and rng.random() < 0.5) else 0
    T = B * M
    w = synth.Workload(f"dt{k}", N, F, 2 * T, M, 900 + k, rng.uniform(1.5, 3.5, N), [])
    x = synth.generate(w, nthreads=4)
    print(f"shape N={N} F={F} M={M} B={B} L={L} est={est}", flush=True)
    plan = sk.Plan(N, F, T, M, norm_window=L, estimator=est)
    xs = [torch.from_numpy(np.ascontiguousarray(x[c * T:(c + 1) * T])).to(DEV) for c in range(2)]
    if want_lpr is not None:
        import ctypes
        vec, lpr, wgs = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int64()
        lib = sk.load_library()
        assert lib.sk_plan_get_pass_a_tile(plan.handle, ctypes.c_void_p(xs[0].data_ptr()), ctypes.byref(vec),
                                           ctypes.byref(lpr), ctypes.byref(wgs)) == 0
        assert (vec.value, lpr.value) == (16, want_lpr), (vec.value, lpr.value)
    outs = [plan.compute(xc, want=sk.ALL_OUTPUTS) for xc in xs]
    torch.cuda.synchronize()
    ref = oracle.sk(x, M, L, est)
    cat = {name: torch.cat([getattr(o, name) for o in outs], dim=1) for name in sk.ALL_OUTPUTS}
    check_result(SimpleNamespace(**cat), ref, M, L, est, what=f"default tile shape {k}")
    plan.close()
