"""GPU test of the entry point that allocates nothing (sk_compute_noalloc).

Two calls in a row through the C ABI, the second with a smaller input,
each against a fresh plan's first call (sk_compute: the same kernels, so
every output agrees bit for bit) and against the CPU oracle to the parity
bar. A call whose prefix sums would not fit the static scratch is refused.
"""
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


def _one(N, F, B, M, L, seed, mask=False):
    w = synth.Workload(f"na{seed}", N, F, B * M, M, seed, np.random.default_rng(seed).uniform(1.5, 3.5, N), [])
    x = synth.generate(w, nthreads=4)
    xd = torch.from_numpy(x).to(DEV)
    md = None
    if mask:
        m = (np.random.default_rng(seed + 1).random((F, N)) > 0.1).astype(np.uint8)
        md = torch.from_numpy(m).to(DEV)
    print(f"no-alloc call N={N} F={F} B={B} M={M} L={L} mask={mask}", flush=True)
    plan = sk.Plan(N, F, B * M, M, norm_window=L, k_sigma=5.0)
    ref_out = plan.compute(xd, mask=md, want=sk.ALL_OUTPUTS)
    out = plan.alloc_outputs(DEV, sk.ALL_OUTPUTS)
    sk.compute_noalloc(xd, out, M, norm_window=L, k_sigma=5.0, mask=md)
    torch.cuda.synchronize()
    plan.close()
    for k in sk.ALL_OUTPUTS:
        a, b = getattr(out, k).cpu().numpy(), getattr(ref_out, k).cpu().numpy()
        assert np.array_equal(a, b, equal_nan=a.dtype.kind == "f"), k
    ref = oracle.sk(x, M, L, 0, 5.0, 0.0, 0.0, None if md is None else md.cpu().numpy())
    check_result(out, ref, M, L, what=f"no-alloc N={N} F={F} B={B} M={M} L={L}")


@pytest.mark.parametrize("L", [0, 1, 4, 256])
def test_noalloc_two_calls_second_smaller(L):
    # CHIME-shaped rows at a quarter of the length, then a smaller problem.
    _one(2048, 4, 256, 256, L, 11)
    _one(256, 2, 37, 64, L, 12, mask=True)


def test_noalloc_scratch_limit():
    # F (ceil(B / R) + 1) N int32 beyond the static array: refused, nothing runs.
    assert sk.noalloc_scratch_bytes() == 32 << 20
    N, F, M, B = 16384, 8, 2, 4096
    x = torch.zeros((1, 1, 1), dtype=torch.uint8, device=DEV)
    d = sk.PlanDesc(N, F, B * M, M, 256, 0, 5.0, 0.0, 0.0)
    o = sk.Outputs(*([x.data_ptr()] * 2 + [None] * 7))
    lib = sk.load_library()
    import ctypes
    rc = lib.sk_compute_noalloc(ctypes.byref(d), ctypes.c_void_p(x.data_ptr()), None, ctypes.byref(o), None)
    assert rc == sk.SK_ERR_SHAPE, lib.sk_last_error()
    o2 = sk.Outputs(*([None] * 9))
    assert lib.sk_compute_noalloc(ctypes.byref(d), ctypes.c_void_p(x.data_ptr()), None, ctypes.byref(o2), None) \
        == sk.SK_ERR_INVALID_ARG
