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


@pytest.mark.parametrize("balance", [True, False])
def test_pass_a_timeline(balance):
    # One timeline launch per setting on wide rows with the deferred-store
    # variant: a record per wavefront of every task, stamps in order, ids in
    # range; and the plan's stream afterwards equals a plan that never ran
    # a timeline, bit for bit (the timeline leaves the normaliser alone).
    N, F, M, B, L = 2048, 4, 32, 24, 5
    T = M * B
    x = synth.generate(synth.Workload("tl", N, F, 2 * T, M, 37, np.full(N, 2.2), []), nthreads=2)
    frames = [torch.from_numpy(np.ascontiguousarray(x[k * T:(k + 1) * T])).to(DEV) for k in range(2)]
    plan, plain = sk.Plan(N, F, T, M, norm_window=L), sk.Plan(N, F, T, M, norm_window=L)
    for p in (plan, plain):
        p.set_pass_a_variant(4, 0)
        p.set_pass_a_blocks(4)
    r0 = plan.compute(frames[0], want=sk.ALL_OUTPUTS)
    tl = plan.pass_a_timeline(frames[1], simd_balance=balance)
    r1 = plan.compute(frames[1], want=sk.ALL_OUTPUTS)
    q0 = plain.compute(frames[0], want=sk.ALL_OUTPUTS)
    q1 = plain.compute(frames[1], want=sk.ALL_OUTPUTS)
    torch.cuda.synchronize()
    tasks = B // 4 * (F * N // 16 // 512)
    assert tl.shape == (8 * tasks, 6)
    assert np.all(tl[:, 0] <= tl[:, 1]) and np.all(tl[:, 1] <= tl[:, 2])
    assert np.all((tl[:, 3] >= 0) & (tl[:, 3] < 8)) and np.all((tl[:, 5] >= 0) & (tl[:, 5] < 4))
    assert (tl[:, 2].max() - tl[:, 0].min()) < 100 * 10**6   # under a second of 100 MHz ticks
    for a, b in ((r0, q0), (r1, q1)):
        for key in sk.ALL_OUTPUTS:
            u, v = getattr(a, key).cpu().numpy(), getattr(b, key).cpu().numpy()
            assert np.array_equal(u, v, equal_nan=u.dtype.kind == "f"), key
    # Another variant is refused.
    plan.set_pass_a_variant(2, 0)
    with pytest.raises(sk.SKError):
        plan.pass_a_timeline(frames[0])
    plan.close()
    plain.close()
