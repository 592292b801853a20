"""The per-phase profiling events: every call, or every stride-th call, is
recorded, and the recorded phase durations are positive and no longer than
the whole loop."""
import ctypes

import numpy as np
import pytest

import synth

torch = pytest.importorskip("torch")
sk = pytest.importorskip("paper_1808_10365_amd")

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


@pytest.mark.parametrize("stride,calls", [(1, 6), (3, 10), (4, 8)])
def test_profile_stride(stride, calls):
    N, F, M, B, L = 256, 4, 64, 40, 16
    T = M * B
    x = synth.generate(synth.Workload("prof", N, F, T, M, 31, np.full(N, 2.5), []), nthreads=2)
    plan = sk.Plan(N, F, T, M, norm_window=L)
    xd = torch.from_numpy(x).to(DEV)
    out = plan.alloc_outputs(DEV)
    lib = sk.load_library()
    want = (calls + stride - 1) // stride
    assert lib.sk_profile_enable(plan.handle, ctypes.c_int32(want + 5)) == 0
    assert lib.sk_profile_set_stride(plan.handle, ctypes.c_int32(stride)) == 0
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record()
    for _ in range(calls):
        plan.compute_into(xd, out)
    e1.record()
    torch.cuda.synchronize()
    total = e0.elapsed_time(e1)
    ms_a = (ctypes.c_float * (want + 5))()
    ms_b = (ctypes.c_float * (want + 5))()
    n = ctypes.c_int32()
    assert lib.sk_profile_read(plan.handle, ms_a, ms_b, want + 5, ctypes.byref(n)) == 0
    assert n.value == want
    a = np.array(ms_a[:want])
    b = np.array(ms_b[:want])
    assert np.all(a > 0) and np.all(b > 0)
    assert (a + b).sum() <= total * 1.001
    assert lib.sk_profile_set_stride(plan.handle, ctypes.c_int32(0)) != 0
    assert lib.sk_profile_enable(plan.handle, ctypes.c_int32(0)) == 0
    plan.close()
