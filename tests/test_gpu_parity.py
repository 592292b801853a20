"""GPU parity: the HIP path (through the C ABI) against the CPU oracle.

Small shapes span several tiles and ragged tails; the workload tests run the
Pathfinder- and CHIME-shaped inputs at their full sizes in the launch
configuration the benchmark times.
"""
import os
import sys

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


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def run_gpu(x, M, L=1, est=0, k=5.0, delta=0.0, sigma_override=0.0, mask=None, lpr=0, variant=None, grid=0):
    T, F, N = x.shape
    plan = sk.Plan(N, F, T, M, norm_window=L, estimator=est, k_sigma=k, expect_offset=delta,
                   sigma_override=sigma_override)
    if lpr:
        plan.set_pass_a_tile(lpr)
    if variant is not None or grid:
        plan.set_pass_a_variant(-1 if variant is None else variant, grid)
    xd = torch.from_numpy(np.ascontiguousarray(x)).to(DEV)
    md = None if mask is None else torch.from_numpy(np.ascontiguousarray(mask)).to(DEV)
    out = plan.compute(xd, mask=md, want=sk.ALL_OUTPUTS)
    torch.cuda.synchronize()
    plan.close()
    return out


def both(x, M, L=1, est=0, what="", **kw):
    _say(f"case {what}: shape={x.shape} M={M} L={L} est={est}")
    g = run_gpu(x, M, L, est, **kw)
    mask = kw.get("mask")
    r = oracle.sk(x, M, L, est, kw.get("k", 5.0), kw.get("delta", 0.0), kw.get("sigma_override", 0.0), mask)
    check_result(g, r, M, L, est, kw.get("k", 5.0), kw.get("delta", 0.0), kw.get("sigma_override", 0.0), what)
    return g, r


# ----------------------------------------------------------------------------- tiny workload

@pytest.mark.parametrize("L,est", [(1, 0), (1, 1), (4, 0), (0, 0), (2, 0), (16, 0)])
def test_tiny_workload(L, est):
    w = synth.tiny(seed=1)
    x = synth.generate(w, nthreads=1)
    g, r = both(x, w.block_len, L, est, what=f"tiny L={L}")
    # The tone in blocks 3-5 is flagged low (a tone lowers the estimator).
    if L in (1, 0):
        assert np.all(r.flags[0, 3:6] & 1)


# ----------------------------------------------------------------------------- ragged shapes

RAGGED = [
    # (T, F, N, M)      covers: 1-byte lanes, 4-byte lanes, 16-byte lanes, odd row counts, tails
    (2 * 3, 1, 1, 3),
    (64, 3, 5, 16),
    (99, 2, 17, 33),
    (128, 1, 48, 64),
    (256, 3, 100, 32),
    (96, 5, 160, 24),
    (64, 2, 4096, 8),
    (130, 1, 64, 65),
    (40, 7, 2064, 10),
]


@pytest.mark.parametrize("shape", RAGGED)
@pytest.mark.parametrize("L", [0, 1, 3])
def test_ragged_random_bytes(shape, L):
    # Uniform random bytes: every code, including code 0 (decodes to -8).
    T, F, N, M = shape
    rng = np.random.default_rng(T * 7 + F * 3 + N + M + L)
    x = rng.integers(0, 256, size=(T, F, N), dtype=np.uint8)
    both(x, M, L, what=f"ragged {shape}")


PASS_A_TILES = ([(0, lpr) for lpr in (1, 2, 4, 8, 16, 32, 64, 128, 256, 512, 1024)]
                + [(v, lpr) for v in (1, 2) for lpr in (256, 512, 1024)] + [(3, 0), (4, 0)])


@pytest.mark.parametrize("variant,lpr", PASS_A_TILES)
def test_every_pass_a_tile(variant, lpr):
    # M = 48 and M = 100 leave partial batches and odd row counts for every
    # row-phase count of the shared table (variant 0). The packed lane table
    # (1, 2) takes 256..1024 lanes per row; M = 100 and 48 leave packed runs
    # shorter than 16 rows, and the 32-group row leaves most lanes of a
    # 256-lane row idle. Variant 3 sets its own lanes per row (blocks side by
    # side); 4 uses 512 lanes and holds the sums of several blocks before
    # storing them.
    rng = np.random.default_rng(lpr + 7 * variant)
    for T, F, N, M in ((96, 3, 512, 48), (200, 2, 256, 100), (64, 4, 2048, 32)):
        x = rng.integers(0, 256, size=(T, F, N), dtype=np.uint8)
        both(x, M, 2, what=f"tile lpr={lpr} variant={variant}", lpr=lpr, variant=variant)


@pytest.mark.parametrize("grid", [1, 3, 7])
def test_pass_a_persistent_grid(grid):
    # Fewer workgroups than tasks: each loops over several (block, chunk) tasks.
    rng = np.random.default_rng(grid)
    T, F, N, M = 512, 2, 1024, 64
    x = rng.integers(0, 256, size=(T, F, N), dtype=np.uint8)
    for variant in (0, 1, 2, 3, 4):
        both(x, M, 3, what=f"grid={grid} variant={variant}", lpr=64, variant=variant, grid=grid)


def test_unaligned_input_pointer():
    # An input view starting one byte into an allocation takes the 1-byte lane path.
    rng = np.random.default_rng(3)
    T, F, N, M = 64, 2, 32, 16
    x = rng.integers(0, 256, size=(T * F * N + 1,), dtype=np.uint8)
    xd = torch.from_numpy(x).to(DEV)[1:].view(T, F, N)
    plan = sk.Plan(N, F, T, M, norm_window=1)
    out = plan.compute(xd)
    torch.cuda.synchronize()
    r = oracle.sk(x[1:].reshape(T, F, N), M, 1)
    check_result(out, r, M, 1, what="unaligned")


def test_mask_and_dead_inputs():
    T, F, N, M = 512, 3, 64, 64
    w = synth.Workload("m", N, F, T, M, 77, np.full(N, 2.0), [])
    x = synth.generate(w, nthreads=2)
    x[:, :, 5] = 0x88           # zero power
    x[:128, 1, 9] = 0x88        # zero power for two blocks of channel 1
    mask = np.ones((F, N), np.uint8)
    mask[0, :7] = 0
    mask[2, 60] = 0
    for L in (0, 1, 2, 4):
        both(x, M, L, what=f"mask L={L}", mask=mask)
    # Fully masked channel: invalid everywhere.
    mask[1, :] = 0
    g, r = both(x, M, 1, what="masked channel", mask=mask)
    assert np.all(g.flags.cpu().numpy()[1] == sk.FLAG_INVALID)


def test_cw_lattice_gives_zero():
    x = synth.lattice_cw(n_inputs=32, n_channels=2, n_samples=64 * 16, seed=5)
    for L in (0, 1, 4):
        g, r = both(x, 64, L, what=f"cw L={L}")
        v = g.v.cpu().numpy()
        full = np.arange(v.shape[1]) >= max(L - 1, 0)
        assert np.all(v[:, full] == 0.0)


def test_gain_invariance_gpu():
    T, F, N, M = 64 * 8, 2, 32, 64
    re, im = synth.uniform_small(N, F, T, seed=21, vmax=3)
    a = run_gpu(synth.encode(re, im), M, 3)
    re[:, :, [1, 4, 17]] *= 2
    im[:, :, [1, 4, 17]] *= 2
    b = run_gpu(synth.encode(re, im), M, 3)
    assert np.array_equal(a.v.cpu().numpy(), b.v.cpu().numpy())


def test_flag_parameters():
    w = synth.tiny(seed=9)
    x = synth.generate(w, nthreads=1)
    for kw in (dict(k=3.0), dict(k=5.0, delta=-0.06), dict(k=2.0, sigma_override=0.02)):
        both(x, 256, 1, what=f"flags {kw}", **kw)
        both(x, 256, 1, 1, what=f"flags tilde {kw}", **kw)


def test_flags_entry_point():
    rng = np.random.default_rng(4)
    v = rng.normal(1.0, 0.05, size=(3, 1000)).astype(np.float32)
    v[0, :5] = np.nan
    ne = rng.integers(0, 64, size=(3, 1000)).astype(np.int32)
    plan = sk.Plan(64, 3, 0, 256, norm_window=1, k_sigma=3.0, expect_offset=0.01)
    fl = plan.flags(torch.from_numpy(v).to(DEV), torch.from_numpy(ne).to(DEV)).cpu().numpy()
    ref = oracle.flags(v.astype(np.float64), ne, 256, 1, 0, 3.0, 0.01)
    assert np.array_equal(fl, ref)


@pytest.mark.parametrize("variant", [None, 0, 1, 2, 3, 4])
def test_largest_block_no_overflow(variant):
    # M = 131071 with every sample at power 128: S2 = M * 2^14 = 2^31 - 2^14.
    # The packed table (1, 2) holds 16 such rows per run: 2^11 + 2^30.
    T, F, N, M = 131071 * 2, 1, 16, 131071
    x = np.zeros((T, F, N), np.uint8)
    x[:, :, 1::2] = 0xFF
    g, r = both(x, M, 1, what=f"max M variant={variant}", variant=variant)
    assert int(g.s2.cpu().numpy()[0, 0, 0]) == M * 128 * 128


def test_empty_call():
    plan = sk.Plan(16, 1, 0, 256, norm_window=4)
    out = plan.compute(torch.empty((0, 1, 16), dtype=torch.uint8, device=DEV))
    torch.cuda.synchronize()
    assert out.v.numel() == 0


# ----------------------------------------------------------------------------- stream semantics

@pytest.mark.parametrize("L", [2, 3, 5, 17, 64])
def test_stream_frames_equal_one_shot(L):
    # Any cut of the stream into frames gives the outputs of one long call.
    N, F, M = 48, 3, 32
    cuts = [4, 1, 7, 2, 16, 3]                # frame lengths in blocks
    T = sum(cuts) * M
    w = synth.Workload("s", N, F, T, M, 31, np.random.default_rng(2).uniform(1.5, 3.5, N), [])
    x = synth.generate(w, nthreads=2)
    ref = oracle.sk(x, M, L)
    t0 = 0
    got_v, got_s1 = [], []
    plans = {}
    for c in cuts:
        if c not in plans:
            plans[c] = sk.Plan(N, F, c * M, M, norm_window=L)
    state = None
    for c in cuts:
        p = plans[c]
        if state is not None:
            p.import_state(state)
        out = p.compute(torch.from_numpy(x[t0:t0 + c * M].copy()).to(DEV))
        torch.cuda.synchronize()
        state = p.export_state()
        got_v.append(out.v.cpu().numpy())
        got_s1.append(out.s1.cpu().numpy())
        t0 += c * M
    v = np.concatenate(got_v, axis=1)
    err = np.abs(v - ref.V) / np.maximum(1, np.abs(ref.V))
    assert err.max() <= 1e-6
    assert np.array_equal(np.concatenate(got_s1, axis=1), ref.S1)


def test_state_reset_and_continuation():
    N, F, M, L = 32, 2, 64, 8
    T = 6 * M
    x = synth.generate(synth.Workload("r", N, F, 2 * T, M, 5, np.full(N, 2.0), []), nthreads=2)
    p = sk.Plan(N, F, T, M, norm_window=L)
    a = p.compute(torch.from_numpy(x[:T].copy()).to(DEV))
    b = p.compute(torch.from_numpy(x[T:].copy()).to(DEV))
    torch.cuda.synchronize()
    ref = oracle.sk(x, M, L)
    assert np.allclose(np.concatenate([a.v.cpu().numpy(), b.v.cpu().numpy()], 1), ref.V, rtol=0, atol=1e-6)
    p.reset()
    c = p.compute(torch.from_numpy(x[T:].copy()).to(DEV))
    torch.cuda.synchronize()
    ref2 = oracle.sk(x[T:], M, L)
    assert np.allclose(c.v.cpu().numpy(), ref2.V, rtol=0, atol=1e-6)
    # A blob from another shape is refused.
    q = sk.Plan(N + 1, F, T, M, norm_window=L)
    with pytest.raises(sk.SKError):
        q.import_state(p.export_state())


# ----------------------------------------------------------------------------- size limits

def test_max_inputs():
    # N = 16384, the largest a plan accepts: each combine wavefront walks 8
    # groups of 256 inputs (8 wavefronts per chunk) and the raw sums need 64
    # bits; wide rows of 2048 column groups in pass A.
    N, F, M, B, L = 16384, 2, 64, 13, 5
    w = synth.Workload("maxn", N, F, M * B, M, 61, np.random.default_rng(3).uniform(1.5, 3.5, N), [])
    both(synth.generate(w, nthreads=4), M, L, what="N = 16384")


def test_window_much_longer_than_calls():
    # L = 2^12 blocks of M = 16 (window power sum 2^12 * 16 * 128 = 2^23), in
    # calls of 40 blocks: the history is carried for 100 calls before the
    # window fills, then slides; every call is checked against the oracle
    # over the whole stream at the end.
    N, F, M, B, L, calls = 32, 2, 16, 40, 1 << 12, 110
    T = M * B
    w = synth.Workload("longw", N, F, calls * T, M, 62, np.random.default_rng(4).uniform(1.5, 3.5, N), [])
    x = synth.generate(w, nthreads=4)
    _say(f"case long window: N={N} F={F} M={M} L={L}, {calls} calls of {B} blocks")
    plan = sk.Plan(N, F, T, M, norm_window=L, k_sigma=5.0)
    xd = torch.from_numpy(x).to(DEV)
    outs = [plan.compute(xd[k * T:(k + 1) * T], want=sk.ALL_OUTPUTS) for k in range(calls)]
    torch.cuda.synchronize()
    cat = {k: torch.cat([getattr(o, k).cpu() for o in outs], dim=1) for k in sk.ALL_OUTPUTS}
    plan.close()
    ref = oracle.sk(x, M, L, 0, 5.0, 0.0, 0.0)
    check_result(SimpleNamespace(**cat), ref, M, L, 0, 5.0, 0.0, 0.0, what="long window")


# ----------------------------------------------------------------------------- full-size workloads

def _workload_parity(w, L, reps=1):
    _say(f"generate {w.name}: N={w.n_inputs} F={w.n_channels} T={w.n_samples} M={w.block_len} L={L}")
    x = synth.generate(w)
    delta, sig = oracle.digitised_expectation(w.sigma, w.block_len)   # thresholds from the oracle's model
    plan = sk.Plan(w.n_inputs, w.n_channels, w.n_samples, w.block_len, norm_window=L, k_sigma=5.0,
                   expect_offset=delta, sigma_override=sig)
    xd = torch.from_numpy(x).to(DEV)
    out = plan.compute(xd)
    torch.cuda.synchronize()
    _say(f"oracle {w.name}")
    ref = oracle.sk(x, w.block_len, L, 0, 5.0, delta, sig)
    clear, total = check_result(out, ref, w.block_len, L, 0, 5.0, delta, sig, w.name)
    _say(f"{w.name}: parity ok, flags compared on {clear}/{total}, flagged {(ref.flags != 0).mean():.3%}")
    plan.close()
    return out, ref


def test_pathfinder_full():
    w = synth.pathfinder(seed=2)
    out, ref = _workload_parity(w, w.norm_window)
    # Sanity (not parity): the tone channels are flagged nearly everywhere.
    tone_ch = [e.channel for e in w.events if e.kind == synth.TONE]
    for c in tone_ch:
        assert (ref.flags[c] != 0).mean() > 0.9


@pytest.mark.parametrize("M", [256, 1024])
def test_chime_full(M):
    w = synth.chime(seed=3, block_len=M)
    _workload_parity(w, w.norm_window)


@pytest.mark.parametrize("L,est", [(1, 1), (1, 0), (4, 0)])
def test_false_alarm_thresholds(L, est):
    # Small K (N = 3 inputs, M = 32): thresholds from the false-alarm
    # probability, checked against the oracle's independent quantiles.
    rng = np.random.default_rng(10 + L)
    T, F, N, M = 32 * 200, 2, 3, 32
    x = synth.generate(synth.Workload("f", N, F, T, M, 12, np.full(N, 2.0), []), nthreads=2)
    x[:, 1, 2] = 0x88                                     # one dead input: N_eff = 2 in channel 1
    plan = sk.Plan(N, F, T, M, norm_window=L, estimator=est, k_sigma=5.0)
    plan.set_false_alarm(0.005)
    for n in range(N + 1):
        lo, hi = plan.thresholds(n)
        if n == 0:
            continue
        fl, olo, ohi = oracle.flags_fap(np.array([1.0]), np.array([n], np.int32), M, L, est, fap=0.005)
        assert abs(lo - olo[0]) < 1e-7 and abs(hi - ohi[0]) < 1e-7
    out = plan.compute(torch.from_numpy(x).to(DEV))
    torch.cuda.synchronize()
    ref = oracle.sk(x, M, L, est)
    v = out.v.cpu().numpy().astype(np.float64)
    assert np.allclose(v, ref.V, rtol=0, atol=1e-6, equal_nan=True)
    f0, lo0, hi0 = oracle.flags_fap(ref.V, ref.n_eff, M, L, est, fap=0.005)
    clear = ~(np.isclose(ref.V, lo0, rtol=0, atol=1e-6) | np.isclose(ref.V, hi0, rtol=0, atol=1e-6))
    g = out.flags.cpu().numpy()
    assert np.array_equal(g[clear], f0[clear])
    assert (g != 0).mean() < 0.1
    fl2 = plan.flags(out.v, out.n_eff).cpu().numpy()
    assert np.array_equal(fl2[clear], f0[clear])


@pytest.mark.parametrize("vec", [1, 4])
@pytest.mark.parametrize("N", [96, 1040, 2112])
@pytest.mark.parametrize("L", [0, 1, 2, 4, 5, 9, 40])
def test_pass_b_tiles(vec, N, L):
    # Every chunk length R gives the oracle's results and the same outputs bit
    # for bit (the sums follow one fixed order), across calls of 3, 1, 20 and
    # 2 blocks: the history carry, calls shorter than R and than the window,
    # and windows shorter and longer than R. N = 1040 leaves a partial group
    # of inputs for both lane widths; N = 2112 gives wavefronts two input
    # groups each.
    F, M = 3, 32
    cuts = [3, 1, 20, 2]
    x = synth.generate(synth.Workload("pb", N, F, sum(cuts) * M, M, 8 + L, np.full(N, 2.2), []), nthreads=2)
    ref = oracle.sk(x, M, L)
    res = {}
    for R in (1, 2, 4):
        plans = {c: sk.Plan(N, F, c * M, M, norm_window=L) for c in set(cuts)}
        for p in plans.values():
            p.set_pass_b_tile(R, vec)
        outs, t0, state = [], 0, None
        for c in cuts:
            p = plans[c]
            if state is not None:
                p.import_state(state)
            outs.append(p.compute(torch.from_numpy(x[t0:t0 + c * M].copy()).to(DEV), want=sk.ALL_OUTPUTS))
            torch.cuda.synchronize()
            state = p.export_state()
            t0 += c * M
        cat = {name: torch.cat([getattr(o, name) for o in outs], dim=1) for name in sk.ALL_OUTPUTS}
        check_result(SimpleNamespace(**cat), ref, M, L, what=f"pass B R={R} vec={vec} N={N} L={L}")
        res[R] = cat
        for p in plans.values():
            p.close()
    for name in sk.ALL_OUTPUTS:
        a, b = res[1][name].cpu().numpy(), res[4][name].cpu().numpy()
        assert np.array_equal(a, b, equal_nan=a.dtype.kind == "f"), name
        a = res[2][name].cpu().numpy()
        assert np.array_equal(a, b, equal_nan=a.dtype.kind == "f"), name


@pytest.mark.parametrize("L", [2, 3, 4])
def test_pass_b_small_window_without_scan(L):
    # Windows of at most one chunk (L <= R) in calls at least as long as the
    # window skip the prefix scan: the combine takes the window start from
    # edge rows and the next history's suffix sums from the rows, including
    # the rows of the next chunk when the history starts in an earlier one
    # (calls of 6, 5, 7, 3 and 9 blocks at R = 4). One plan per chunk length,
    # carried from call to call; R = 1 (which scans) is the reference, bit
    # for bit, and the oracle checks all of them.
    N, F, M = 320, 2, 16
    cuts = [6, 5, 7, 3, 9]
    x = synth.generate(synth.Workload("sw", N, F, sum(cuts) * M, M, 70 + L, np.full(N, 2.4), []), nthreads=2)
    ref = oracle.sk(x, M, L)
    res = {}
    for R in (1, 2, 4):
        plans = {c: sk.Plan(N, F, c * M, M, norm_window=L) for c in set(cuts)}
        for p in plans.values():
            p.set_pass_b_tile(R, 0)
        outs, t0, state = [], 0, None
        for c in cuts:
            p = plans[c]
            if state is not None:
                p.import_state(state)
            outs.append(p.compute(torch.from_numpy(x[t0:t0 + c * M].copy()).to(DEV), want=sk.ALL_OUTPUTS))
            torch.cuda.synchronize()
            state = p.export_state()
            t0 += c * M
        cat = {name: torch.cat([getattr(o, name) for o in outs], dim=1) for name in sk.ALL_OUTPUTS}
        check_result(SimpleNamespace(**cat), ref, M, L, what=f"small window R={R} L={L}")
        res[R] = cat
        for p in plans.values():
            p.close()
    for R in (2, 4):
        for name in sk.ALL_OUTPUTS:
            a, b = res[1][name].cpu().numpy(), res[R][name].cpu().numpy()
            assert np.array_equal(a, b, equal_nan=a.dtype.kind == "f"), (R, name)


@pytest.mark.parametrize("R", [1, 2, 4])
@pytest.mark.parametrize("L", [2, 7, 256])
def test_pass_b_one_plan_many_calls(R, L):
    # One plan, five calls of 37 blocks: the device-resident history (suffix
    # sums) carried from call to call with no export, against one long run.
    N, F, M = 256, 2, 16
    T = 37 * M
    x = synth.generate(synth.Workload("mc", N, F, 5 * T, M, 40 + L, np.full(N, 2.0), []), nthreads=2)
    ref = oracle.sk(x, M, L)
    p = sk.Plan(N, F, T, M, norm_window=L)
    p.set_pass_b_tile(R, 0)
    outs = [p.compute(torch.from_numpy(x[c * T:(c + 1) * T].copy()).to(DEV), want=sk.ALL_OUTPUTS) for c in range(5)]
    torch.cuda.synchronize()
    cat = {name: torch.cat([getattr(o, name) for o in outs], dim=1) for name in sk.ALL_OUTPUTS}
    check_result(SimpleNamespace(**cat), ref, M, L, what=f"many calls R={R} L={L}")
    p.close()


@pytest.mark.parametrize("variant", [1, 2, 3, 4])
@pytest.mark.parametrize("Q", [2, 3, 4, 7, 64])
def test_packed_multi_block_tasks(variant, Q):
    # Packed-table pass A tasks walking Q consecutive blocks: B = 37 leaves a
    # short last task for every Q. Variant 3 ignores Q: its 64-group rows put
    # 4 blocks side by side. Variant 4 takes Q in 1..4 and sizes its tasks
    # itself otherwise.
    rng = np.random.default_rng(Q * 10 + variant)
    T, F, N, M = 48 * 37, 2, 512, 48
    x = rng.integers(0, 256, size=(2 * T, F, N), dtype=np.uint8)
    ref = oracle.sk(x, M, 5)
    p = sk.Plan(N, F, T, M, norm_window=5)
    p.set_pass_a_variant(variant, 0)
    p.set_pass_a_blocks(Q)
    outs = [p.compute(torch.from_numpy(x[c * T:(c + 1) * T].copy()).to(DEV), want=sk.ALL_OUTPUTS) for c in range(2)]
    torch.cuda.synchronize()
    cat = {name: torch.cat([getattr(o, name) for o in outs], dim=1) for name in sk.ALL_OUTPUTS}
    check_result(SimpleNamespace(**cat), ref, M, 5, what=f"packed variant={variant} Q={Q}")
    p.close()
