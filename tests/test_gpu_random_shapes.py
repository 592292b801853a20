"""GPU parity over seeded random shapes: the library's own tile choices
(no forced variants) on shapes drawn from a wide range, against the oracle.

Each case draws N (multiples of 16 and 4 and neither), F, M, the blocks per
call, the window L, the estimator, a mask or none, quantised-Gaussian or
uniform random bytes, and 1..3 consecutive calls on one plan (stream mode).
A second test draws every tuning control at random on the same shapes. The
cases are fixed by their seeds, so a failure names a reproducible shape."""
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

N_CHOICES = [1, 3, 16, 17, 48, 64, 100, 256, 272, 512, 1000, 1024, 1040, 2048, 2064, 4096]
F_CHOICES = [1, 2, 3, 4, 8]
M_CHOICES = [2, 3, 8, 16, 31, 64, 256, 1024]
L_CHOICES = [0, 1, 2, 3, 7, 16, 64, 300]
MAX_CALL_BYTES = 1 << 24


def draw(case):
    rng = np.random.default_rng(1000 + case)
    N = int(rng.choice(N_CHOICES))
    F = int(rng.choice(F_CHOICES))
    M = int(rng.choice(M_CHOICES))
    while N * F * M > MAX_CALL_BYTES and M > 2:
        M //= 2
    b_max = max(1, min(200, MAX_CALL_BYTES // (N * F * M)))
    B = int(rng.integers(1, b_max + 1))
    L = int(rng.choice(L_CHOICES))
    est = 1 if (L == 1 and rng.random() < 0.5) else 0
    calls = int(rng.integers(1, 4))
    use_mask = rng.random() < 0.3
    uniform = rng.random() < 0.2
    return dict(N=N, F=F, M=M, B=B, L=L, est=est, calls=calls, use_mask=use_mask, uniform=uniform,
                seed=int(rng.integers(1, 1 << 30)))


@pytest.mark.parametrize("case", range(48))
def test_random_shape(case):
    c = draw(case)
    N, F, M, B, L, est, calls = c["N"], c["F"], c["M"], c["B"], c["L"], c["est"], c["calls"]
    T = M * B
    print(f"case {case}: {c}", flush=True)
    rng = np.random.default_rng(c["seed"])
    if c["uniform"]:
        x = rng.integers(0, 256, size=(calls * T, F, N), dtype=np.uint8)
    else:
        w = synth.Workload(f"rand{case}", N, F, calls * T, M, c["seed"], rng.uniform(1.5, 3.5, N), [])
        x = synth.generate(w, nthreads=4)
    mask = (rng.random((F, N)) > 0.1).astype(np.uint8) if c["use_mask"] else None
    plan = sk.Plan(N, F, T, M, norm_window=L, estimator=est, k_sigma=5.0)
    md = None if mask is None else torch.from_numpy(mask).to(DEV)
    outs = []
    for k in range(calls):
        xd = torch.from_numpy(np.ascontiguousarray(x[k * T:(k + 1) * T])).to(DEV)
        outs.append(plan.compute(xd, mask=md, want=sk.ALL_OUTPUTS))
    torch.cuda.synchronize()
    plan.close()
    got = SimpleNamespace(**{name: torch.cat([getattr(o, name) for o in outs], dim=1) for name in sk.ALL_OUTPUTS})
    ref = oracle.sk(x, M, L, est, 5.0, 0.0, 0.0, mask)
    check_result(got, ref, M, L, est, 5.0, 0.0, 0.0, what=f"random case {case} {c}")


def draw_knobs(case):
    r = np.random.default_rng(77000 + case)
    return dict(chunk=int(r.choice([0, 1, 2, 4])), vec=int(r.choice([0, 1, 4])),
                variant=int(r.integers(-1, 5)), lpr=int(r.choice([0, 1, 4, 16, 64, 256, 512, 1024])),
                grid=int(r.choice([0, 0, 64, 300])), ablocks=int(r.choice([0, 0, 2, 4])))


@pytest.mark.parametrize("case", range(40))
def test_random_shape_and_tuning(case):
    # The same seeded shapes with every tuning control drawn at random:
    # pass B chunk and lane width, pass A variant, lanes per row, persistent
    # grid and blocks per task.
    c, kn = draw(case), draw_knobs(case)
    N, F, M, B, L, est, calls = c["N"], c["F"], c["M"], c["B"], c["L"], c["est"], c["calls"]
    T = M * B
    print(f"case {case}: {c} {kn}", flush=True)
    rng = np.random.default_rng(c["seed"])
    if c["uniform"]:
        x = rng.integers(0, 256, size=(calls * T, F, N), dtype=np.uint8)
    else:
        w = synth.Workload(f"knob{case}", N, F, calls * T, M, c["seed"], rng.uniform(1.5, 3.5, N), [])
        x = synth.generate(w, nthreads=4)
    mask = (rng.random((F, N)) > 0.1).astype(np.uint8) if c["use_mask"] else None
    plan = sk.Plan(N, F, T, M, norm_window=L, estimator=est, k_sigma=5.0)
    if kn["chunk"] or kn["vec"]:
        plan.set_pass_b_tile(kn["chunk"], kn["vec"])
    if kn["lpr"]:
        plan.set_pass_a_tile(kn["lpr"])
    if kn["variant"] >= 0 or kn["grid"]:
        plan.set_pass_a_variant(kn["variant"], kn["grid"])
    if kn["ablocks"]:
        plan.set_pass_a_blocks(kn["ablocks"])
    md = None if mask is None else torch.from_numpy(mask).to(DEV)
    outs = []
    for k in range(calls):
        xd = torch.from_numpy(np.ascontiguousarray(x[k * T:(k + 1) * T])).to(DEV)
        outs.append(plan.compute(xd, mask=md, want=sk.ALL_OUTPUTS))
    torch.cuda.synchronize()
    plan.close()
    got = SimpleNamespace(**{name: torch.cat([getattr(o, name) for o in outs], dim=1) for name in sk.ALL_OUTPUTS})
    ref = oracle.sk(x, M, L, est, 5.0, 0.0, 0.0, mask)
    check_result(got, ref, M, L, est, 5.0, 0.0, 0.0, what=f"random case {case} with tuning {kn}")
