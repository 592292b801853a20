"""The plan autotuner (sk_plan_autotune): it times its candidates on a frame,
keeps one of them, and leaves the stream's results untouched. A plan tuned
between two calls gives, on the second call, the same outputs bit for bit as
an untuned plan fed the same two frames (the normaliser history is exported
before tuning and imported after; integer sums are exact and the combine's
order does not depend on the chunk length), and both match the oracle over
the two-frame stream."""
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


# (N, F, M, B, L): wide rows (>= 512 groups of 16 inputs: the deferred-store
# candidates), mid-width rows, narrow rows (blocks side by side), and N not a
# multiple of 16 (only the library's pass A).
SHAPES = [(2048, 4, 64, 40, 8), (1024, 4, 64, 33, 5), (64, 2, 32, 90, 12), (100, 3, 16, 50, 6)]


@pytest.mark.parametrize("N,F,M,B,L", SHAPES)
def test_autotune_keeps_stream_results(N, F, M, B, L):
    T = M * B
    w = synth.Workload(f"tune{N}", N, F, 3 * T, M, 400 + N, np.linspace(1.8, 3.2, N), [])
    x = synth.generate(w, nthreads=2)
    frames = [torch.from_numpy(np.ascontiguousarray(x[k * T:(k + 1) * T])).to(DEV) for k in range(3)]
    print(f"autotune shape N={N} F={F} M={M} B={B} L={L}", flush=True)
    tuned = sk.Plan(N, F, T, M, norm_window=L, k_sigma=4.0)
    plain = sk.Plan(N, F, T, M, norm_window=L, k_sigma=4.0)
    got = {"tuned": [], "plain": []}
    for k in range(2):
        for name, plan in (("tuned", tuned), ("plain", plain)):
            r = plan.compute(frames[k], want=sk.ALL_OUTPUTS)
            got[name].append({key: getattr(r, key).cpu().numpy().copy() for key in sk.ALL_OUTPUTS})
        torch.cuda.synchronize()
        if k == 0:
            # Tune on a different frame between the two calls.
            pick = tuned.autotune(frames[2], reps=2)
            print("pick:", pick, flush=True)
            wide = N % 16 == 0 and N * F // 16 >= 512
            mid = N % 16 == 0 and N * F // 16 >= 256
            n_a = 1 + (3 + 1 if wide else 0) + (2 if mid else 0) + (1 if N % 16 == 0 and N * F // 16 < 256 else 0)
            # Wide rows also time 2- and 4-block tasks without chunk sums,
            # each at its own chunk length only.
            assert pick["candidates"] == 3 * n_a + (2 if wide else 0)
            assert pick["pass_a_chunk_sums"] in (0, 1)
            if pick["pass_a_chunk_sums"]:
                assert pick["pass_a_variant"] == 4 and pick["pass_a_blocks"] == pick["pass_b_chunk"]
            assert pick["pass_b_chunk"] in (1, 2, 4)
            assert pick["pass_b_vec"] in (1, 4)
            assert pick["ms_pass_a"] > 0 and pick["ms_pass_b"] > 0
            assert pick["ms_pass_a"] + pick["ms_pass_b"] <= \
                (pick["ms_library_pass_a"] + pick["ms_library_pass_b"]) * (1 + 1e-6) or pick["ms_library_pass_a"] == 0
            if N % 16:
                assert pick["pass_a_variant"] == 0
    for k in range(2):
        for key in sk.ALL_OUTPUTS:
            a, b = got["tuned"][k][key], got["plain"][k][key]
            assert np.array_equal(a, b, equal_nan=a.dtype.kind == "f"), (k, key)
    ref = oracle.sk(x[:2 * T], M, L, 0, 4.0, 0.0, 0.0)
    cat = {key: torch.from_numpy(np.concatenate([got["tuned"][0][key], got["tuned"][1][key]], axis=1))
           for key in sk.ALL_OUTPUTS}
    check_result(SimpleNamespace(**cat), ref, M, L, 0, 4.0, 0.0, 0.0, what=f"tuned plan N={N} F={F} M={M}")
    tuned.close()
    plain.close()


def test_autotune_rejects_bad_arguments():
    plan = sk.Plan(64, 1, 64 * 4, 64, norm_window=2)
    x = torch.zeros((64 * 4, 1, 64), dtype=torch.uint8, device=DEV)
    with pytest.raises(sk.SKError):
        plan.autotune(x, reps=0)
    with pytest.raises(ValueError):
        plan.autotune(torch.zeros((64 * 4, 1, 63), dtype=torch.uint8, device=DEV))
    plan.close()
