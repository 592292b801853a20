"""GPU parity of the batched form: many uneven problems per graph launch.

Every problem's results equal its own single-plan results bit for bit (the
integer sums are exact and the FP64 combine runs in the same fixed order),
and match the CPU oracle over the concatenated stream to the usual bar."""
import numpy as np
import pytest

import oracle
import synth
from parity import check_result

torch = pytest.importorskip("torch")
sk = pytest.importorskip("paper_1808_10365_amd")

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def _problems(seed, n, max_t=1 << 12):
    rng = np.random.default_rng(seed)
    out = []
    for p in range(n):
        N = int(rng.choice([16, 64, 256, 1024]))
        M = int(rng.choice([16, 64, 256]))
        F = int(rng.choice([1, 3, 4]))
        T = M * int(rng.integers(1, max_t // M + 1))
        L = int(rng.choice([0, 1, 2, 5, 64]))
        est = 1 if (L == 1 and rng.random() < 0.5) else 0
        w = synth.Workload(f"p{p}", N, F, 2 * T, M, seed * 100 + p, rng.uniform(1.5, 3.5, N), [])
        out.append((w, dict(n_inputs=N, n_channels=F, n_samples=T, block_len=M, norm_window=L, estimator=est,
                            k_sigma=4.0, expect_offset=-0.05, sigma_override=0.0)))
    return out


@pytest.mark.parametrize("graph,autotune", [(False, False), (True, False), (False, True), (True, True)])
def test_batch_state_advances_once_per_call(graph, autotune, tmp_path):
    probs = _problems(11, 9)
    xs = [torch.from_numpy(np.ascontiguousarray(synth.generate(w, nthreads=2)[:kw["n_samples"]])).to(DEV)
          for w, kw in probs]
    batch = sk.Batch([kw for _, kw in probs], xs, autotune=autotune, use_graph=graph,
                     tune_cache=str(tmp_path / "tune.json"))
    h0 = [batch.hist_len(j) for j in range(len(probs))]
    print("history after create:", h0, flush=True)
    assert h0 == [0] * len(probs)
    for call in (1, 2):
        batch.compute()
        torch.cuda.synchronize()
        h = [batch.hist_len(j) for j in range(len(probs))]
        expect = [min(max(kw["norm_window"] - 1, 0), call * (kw["n_samples"] // kw["block_len"])) for _, kw in probs]
        print(f"history after call {call}:", h, "expected", expect, flush=True)
        assert h == expect


@pytest.mark.parametrize("graph,autotune", [(False, False), (True, False), (True, True)])
def test_batch_two_calls_match_oracle_and_plans(graph, autotune, tmp_path):
    probs = _problems(11, 9)
    xs = [synth.generate(w, nthreads=2) for w, _ in probs]
    first = [torch.from_numpy(np.ascontiguousarray(x[:kw["n_samples"]])).to(DEV) for x, (_, kw) in zip(xs, probs)]
    second = [torch.from_numpy(np.ascontiguousarray(x[kw["n_samples"]:])).to(DEV) for x, (_, kw) in zip(xs, probs)]
    batch = sk.Batch([kw for _, kw in probs], first, autotune=autotune, use_graph=graph,
                     tune_cache=str(tmp_path / "tune.json"), want=sk.ALL_OUTPUTS)
    plans = [sk.Plan(**kw) for _, kw in probs]
    res_batch, res_plan = [], []
    for inputs in (first, second):
        outs = batch.compute(inputs)
        torch.cuda.synchronize()
        res_batch.append([{k: getattr(o, k).cpu().numpy().copy() for k in sk.ALL_OUTPUTS} for o in outs])
        outs_plan = [p.compute(x, want=sk.ALL_OUTPUTS) for p, x in zip(plans, inputs)]   # one call per plan
        res_plan.append([{k: getattr(o, k).cpu().numpy() for k in sk.ALL_OUTPUTS} for o in outs_plan])
        torch.cuda.synchronize()
    for j, (w, kw) in enumerate(probs):
        M, L, est = kw["block_len"], kw["norm_window"], kw["estimator"]
        for call in range(2):
            for k in sk.ALL_OUTPUTS:
                a, b = res_batch[call][j][k], res_plan[call][j][k]
                assert np.array_equal(a, b, equal_nan=(k == "v")), (j, call, k)
        ref = oracle.sk(xs[j], M, L, est, 4.0, -0.05, 0.0)
        B = kw["n_samples"] // M

        class G:
            pass
        g = G()
        for k in sk.ALL_OUTPUTS:
            full = np.concatenate([res_batch[0][j][k], res_batch[1][j][k]], axis=1)
            setattr(g, k, torch.from_numpy(full))
        check_result(g, ref, M, L, est, 4.0, -0.05, 0.0, what=f"batch problem {j} {kw}")


def test_batch_tiles_and_cache(tmp_path):
    # The autotuner times every candidate of each (N, M, F) class, records the
    # times and the pick in the cache, and the pick is the fastest recorded
    # candidate; a second batch of the same classes takes the picks from the
    # cache without timing.
    import json
    probs = _problems(5, 4)
    probs.append((probs[0][0], dict(probs[0][1])))         # two problems of one class
    xs = [torch.from_numpy(synth.generate(w, nthreads=2)[:kw["n_samples"]].copy()).to(DEV) for w, kw in probs]
    cache = tmp_path / "tune.json"
    b1 = sk.Batch([kw for _, kw in probs], xs, autotune=True, tune_cache=str(cache))
    tiles = [b1.tiles(j) for j in range(len(probs))]
    tun1 = [b1.tuning(j) for j in range(len(probs))]
    print("tuning:", tun1, flush=True)
    assert not any(t["from_cache"] for t in tun1)
    assert tun1[0] == tun1[-1]
    c = json.loads(cache.read_text())
    classes = {(kw["n_inputs"], kw["block_len"], kw["n_channels"]) for _, kw in probs}
    picks = [k for k in c if k.endswith("|pick")]
    assert len(picks) == len(classes)
    for j, (_, kw) in enumerate(probs):
        key = next(k for k in picks if f"|N={kw['n_inputs']}|M={kw['block_len']}|F={kw['n_channels']}|" in k)
        cls = key[:-len("|pick")]
        a_times = {k: v for k, v in c.items() if k.startswith(cls + "|A|")}
        ab_times = {k: v for k, v in c.items() if k.startswith(cls + "|AB|")}
        wide = kw["n_inputs"] * kw["n_channels"] // 16 >= 256
        assert len(a_times) == (6 if wide else 2)
        assert 3 <= len(ab_times) <= (5 if wide and kw["norm_window"] >= 2 else 3)
        t = tun1[j]
        q = t["blocks"] if wide else 1
        assert c[key] == t["rows"] * 100 + q * 10 + t["chunk"]
        # Step 1 keeps the rows of the fastest pass A; step 2 keeps the
        # fastest whole call.
        a_best = min(a_times, key=a_times.get)
        assert f"|A|rows={t['rows']}|" in a_best
        assert ab_times[f"{cls}|AB|rows={t['rows']}|blocks={q}|chunk={t['chunk']}"] == min(ab_times.values())
    b1.close()
    b2 = sk.Batch([kw for _, kw in probs], xs, autotune=True, tune_cache=str(cache))
    tun2 = [b2.tuning(j) for j in range(len(probs))]
    assert all(t["from_cache"] for t in tun2)
    assert [{k: v for k, v in t.items() if k != "from_cache"} for t in tun2] == \
        [{k: v for k, v in t.items() if k != "from_cache"} for t in tun1]
    assert [b2.tiles(j) for j in range(len(probs))] == tiles
    for (lpr, grid), (_, kw) in zip(tiles, probs):
        groups = kw["n_inputs"] * kw["n_channels"] // 16
        want = 512 if groups >= 512 else 256 if groups >= 256 else 1 << max(0, (groups - 1).bit_length())
        assert lpr == want and grid > 0
    b2.close()


def test_batch_wide_and_narrow_rows(tmp_path):
    # Default outputs (no SK_i or significance computed). Rows of 512 column
    # groups (one 512-group task per block, run by a whole workgroup with
    # deferred stores), of 1 group
    # (256 blocks side by side per workgroup) and of 48 groups (a block row
    # padded to 64 lanes), with a block count that leaves a partial last task.
    shapes = [(2048, 4, 64 * 9, 64, 3), (16, 1, 16 * 301, 16, 4), (256, 3, 32 * 45, 32, 2)]
    probs, xs, outs = [], [], []
    for k, (N, F, T, M, L) in enumerate(shapes):
        w = synth.Workload(f"wide{k}", N, F, T, M, 70 + k, np.full(N, 2.3), [])
        x = synth.generate(w, nthreads=2)
        probs.append(dict(n_inputs=N, n_channels=F, n_samples=T, block_len=M, norm_window=L, k_sigma=5.0))
        xs.append(x)
    dx = [torch.from_numpy(x).to(DEV) for x in xs]
    batch = sk.Batch(probs, dx, autotune=True, use_graph=True, tune_cache=str(tmp_path / "t.json"))
    res = batch.compute()
    torch.cuda.synchronize()
    for j, (x, kw) in enumerate(zip(xs, probs)):
        ref = oracle.sk(x, kw["block_len"], kw["norm_window"], 0, 5.0, 0.0, 0.0)
        check_result(res[j], ref, kw["block_len"], kw["norm_window"], what=f"wide/narrow problem {j}")
    batch.close()


def test_batch_rejects_unsupported():
    x = torch.zeros((64, 1, 20), dtype=torch.uint8, device=DEV)
    with pytest.raises(sk.SKError):
        sk.Batch([dict(n_inputs=20, n_channels=1, n_samples=64, block_len=16)], [x])


def test_batch_time_pass_a_leaves_calls_intact(tmp_path):
    # Timing pass A alone between two calls rewrites S1/S2 from the inputs
    # only: the second call still continues the first call's history, and both
    # calls match the oracle over the concatenated stream.
    probs = _problems(13, 5)
    xs = [synth.generate(w, nthreads=2) for w, _ in probs]
    first = [torch.from_numpy(np.ascontiguousarray(x[:kw["n_samples"]])).to(DEV) for x, (_, kw) in zip(xs, probs)]
    second = [torch.from_numpy(np.ascontiguousarray(x[kw["n_samples"]:])).to(DEV) for x, (_, kw) in zip(xs, probs)]
    batch = sk.Batch([kw for _, kw in probs], first, autotune=False, use_graph=True,
                     tune_cache=str(tmp_path / "tune.json"), want=sk.ALL_OUTPUTS)
    res = []
    for call, inputs in enumerate((first, second)):
        outs = batch.compute(inputs)
        torch.cuda.synchronize()
        res.append([{k: getattr(o, k).cpu().numpy().copy() for k in sk.ALL_OUTPUTS} for o in outs])
        if call == 0:
            ms = batch.time_pass_a()
            print("batched pass A alone:", ms, "ms", flush=True)
            assert 0.0 < ms < 1000.0
            h = [batch.hist_len(j) for j in range(len(probs))]
            expect = [min(max(kw["norm_window"] - 1, 0), kw["n_samples"] // kw["block_len"]) for _, kw in probs]
            assert h == expect
    for j, (w, kw) in enumerate(probs):
        M, L, est = kw["block_len"], kw["norm_window"], kw["estimator"]
        ref = oracle.sk(xs[j], M, L, est, 4.0, -0.05, 0.0)

        class G:
            pass
        g = G()
        for k in sk.ALL_OUTPUTS:
            setattr(g, k, torch.from_numpy(np.concatenate([res[0][j][k], res[1][j][k]], axis=1)))
        check_result(g, ref, M, L, est, 4.0, -0.05, 0.0, what=f"timed batch problem {j} {kw}")


@pytest.mark.parametrize("q", [2, 4])
def test_batch_chunk_sums_from_pass_a(q, tmp_path):
    # Wide rows whose pass A tasks walk exactly one pass B chunk: pass A
    # writes the chunk sums and the scan reads them instead of the rows. The
    # pick is forced through the tuning cache; results equal the single
    # plan's bit for bit over two calls and match the oracle.
    import json
    arch = torch.cuda.get_device_properties(0).gcnArchName
    # Rows of 256 column groups (256-lane tasks on half a workgroup) and of
    # 512 and 768 (512-group tasks on a whole workgroup; the second chunk of
    # the 768-group rows half idle).
    shapes = [(1024, 4, 64, 37, 9), (2048, 2, 32, 50, 20), (4096, 1, 16, 23, 64), (2048, 4, 32, 29, 7),
              (2048, 6, 16, 18, 5)]
    cache = {}
    for N, F, M, B, L in shapes:
        cache[f"{arch}|batch|N={N}|M={M}|F={F}|pick"] = 8 * 100 + q * 10 + q
    path = tmp_path / "tune.json"
    path.write_text(json.dumps(cache))
    probs, xs = [], []
    for k, (N, F, M, B, L) in enumerate(shapes):
        w = synth.Workload(f"cs{k}", N, F, 2 * M * B, M, 90 + k, np.linspace(1.7, 3.1, N), [])
        xs.append(synth.generate(w, nthreads=2))
        probs.append(dict(n_inputs=N, n_channels=F, n_samples=M * B, block_len=M, norm_window=L, k_sigma=4.5))
    first = [torch.from_numpy(np.ascontiguousarray(x[:kw["n_samples"]])).to(DEV) for x, kw in zip(xs, probs)]
    second = [torch.from_numpy(np.ascontiguousarray(x[kw["n_samples"]:])).to(DEV) for x, kw in zip(xs, probs)]
    batch = sk.Batch(probs, first, autotune=True, use_graph=True, tune_cache=str(path), want=sk.ALL_OUTPUTS)
    for j in range(len(probs)):
        t = batch.tuning(j)
        print("problem", j, t, flush=True)
        assert t["from_cache"] and t["blocks"] == q and t["chunk"] == q and t["rows"] == 8
    plans = [sk.Plan(**kw) for kw in probs]
    res = []
    for inputs in (first, second):
        outs = batch.compute(inputs)
        torch.cuda.synchronize()
        rb = [{k: getattr(o, k).cpu().numpy().copy() for k in sk.ALL_OUTPUTS} for o in outs]
        op = [p.compute(x, want=sk.ALL_OUTPUTS) for p, x in zip(plans, inputs)]   # one call per plan
        rp = [{k: getattr(o, k).cpu().numpy() for k in sk.ALL_OUTPUTS} for o in op]
        torch.cuda.synchronize()
        for j in range(len(probs)):
            for k in sk.ALL_OUTPUTS:
                assert np.array_equal(rb[j][k], rp[j][k], equal_nan=(k == "v")), (j, k)
        res.append(rb)
    for j, kw in enumerate(probs):
        ref = oracle.sk(xs[j], kw["block_len"], kw["norm_window"], 0, 4.5, 0.0, 0.0)
        from types import SimpleNamespace
        cat = {k: torch.from_numpy(np.concatenate([res[0][j][k], res[1][j][k]], axis=1)) for k in sk.ALL_OUTPUTS}
        check_result(SimpleNamespace(**cat), ref, kw["block_len"], kw["norm_window"], 0, 4.5, 0.0, 0.0,
                     what=f"chunk-sum problem {j} {kw}")
    batch.close()
    for p in plans:
        p.close()
