"""GPU parity of the single-launch path (one cooperative kernel per call:
pass A, the window prefix scans across workgroups, the combine, V and flags).
Each case runs three calls (history carried, including windows longer than a
call) and compares with the oracle to the usual bar and with the two-pass path
of the same plan shape: integer outputs identical, V within 1e-12."""
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

# (N, F, M, B, L): 1..4 blocks per workgroup at 256 CUs, windows shorter
# and longer than a call.
CASES = [
    (2048, 4, 8, 1024, 256),
    (2048, 4, 8, 1000, 5),
    (2048, 4, 4, 700, 64),
    (2048, 4, 4, 300, 450),
    (2048, 4, 16, 100, 2),
    (1024, 8, 4, 900, 37),
    (1024, 2, 8, 513, 1200),
]


def _run(plan, xs, want):
    outs = [plan.compute(x, want=want) for x in xs]
    torch.cuda.synchronize()
    return {name: torch.cat([getattr(o, name) for o in outs], dim=1) for name in want}


@pytest.mark.parametrize("k", range(len(CASES)))
def test_fused_matches_oracle_and_two_pass(k):
    N, F, M, B, L = CASES[k]
    T = B * M
    rng = np.random.default_rng(700 + k)
    w = synth.Workload(f"fu{k}", N, F, 3 * T, M, 40 + k, rng.uniform(1.5, 3.5, N), [])
    x = synth.generate(w, nthreads=4)
    xs = [torch.from_numpy(np.ascontiguousarray(x[c * T:(c + 1) * T])).to(DEV) for c in range(3)]
    print(f"case N={N} F={F} M={M} B={B} L={L}", flush=True)
    fused = sk.Plan(N, F, T, M, norm_window=L)
    fused.set_fused(1)
    got = _run(fused, xs, sk.ALL_OUTPUTS)
    assert fused.last_fused()
    twop = sk.Plan(N, F, T, M, norm_window=L)
    twop.set_fused(0)
    ref2 = _run(twop, xs, sk.ALL_OUTPUTS)
    assert not twop.last_fused()
    ref = oracle.sk(x, M, L)
    check_result(SimpleNamespace(**got), ref, M, L, what=f"fused case {k}")
    for name in ("s1", "s2", "r1", "r2", "n_eff"):
        assert torch.equal(got[name], ref2[name]), name
    v1, v2 = got["v"].cpu().numpy().astype(np.float64), ref2["v"].cpu().numpy().astype(np.float64)
    assert np.array_equal(np.isnan(v1), np.isnan(v2))
    ok = ~np.isnan(v1)
    assert np.all(np.abs(v1[ok] - v2[ok]) <= 1e-6 * np.maximum(1.0, np.abs(v2[ok])))
    fused.close()
    twop.close()


def test_fused_mask_and_no_s2_export():
    N, F, M, B, L = 2048, 4, 8, 1024, 64
    T = B * M
    rng = np.random.default_rng(9)
    w = synth.Workload("fumask", N, F, 2 * T, M, 77, rng.uniform(1.5, 3.5, N), [])
    x = synth.generate(w, nthreads=4)
    mask = (rng.random((F, N)) > 0.1).astype(np.uint8)
    md = torch.from_numpy(mask).to(DEV)
    plan = sk.Plan(N, F, T, M, norm_window=L)
    plan.set_fused(1)
    outs = []
    for c in range(2):
        xc = torch.from_numpy(np.ascontiguousarray(x[c * T:(c + 1) * T])).to(DEV)
        outs.append(plan.compute(xc, mask=md, want=("v", "flags", "n_eff", "r1", "r2", "s1")))
        assert plan.last_fused()
    torch.cuda.synchronize()
    got = SimpleNamespace(s1=torch.cat([o.s1 for o in outs], 1), s2=None,
                          r1=torch.cat([o.r1 for o in outs], 1), r2=torch.cat([o.r2 for o in outs], 1),
                          v=torch.cat([o.v for o in outs], 1), flags=torch.cat([o.flags for o in outs], 1),
                          n_eff=torch.cat([o.n_eff for o in outs], 1))
    ref = oracle.sk(x, M, L, mask=mask)
    check_result(got, ref, M, L, what="fused with mask, S2 not exported")
    plan.close()


def test_fused_off_by_default_and_shape_gate():
    # Default plan: two-pass. Switched on for a shape it does not serve
    # (N % 1024 != 0): the call still runs, two-pass, and matches the oracle.
    N, F, M, B, L = 2048, 4, 8, 64, 16
    T = B * M
    w = synth.Workload("fuoff", N, F, T, M, 78, np.full(N, 2.5), [])
    x = synth.generate(w, nthreads=4)
    plan = sk.Plan(N, F, T, M, norm_window=L)
    plan.compute(torch.from_numpy(x).to(DEV))
    torch.cuda.synchronize()
    assert not plan.last_fused()
    plan.close()

    N = 1536
    w = synth.Workload("fugate", N, F, T, M, 79, np.full(N, 2.5), [])
    x = synth.generate(w, nthreads=4)
    plan = sk.Plan(N, F, T, M, norm_window=L)
    plan.set_fused(1)
    got = plan.compute(torch.from_numpy(x).to(DEV), want=sk.ALL_OUTPUTS)
    torch.cuda.synchronize()
    assert not plan.last_fused()
    check_result(got, oracle.sk(x, M, L), M, L, what="fused switched on, shape not served")
    with pytest.raises(Exception):
        plan.set_fused(2)
    plan.close()
