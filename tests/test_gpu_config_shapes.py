"""GPU parity at the benchmark's own batched and serving shapes.

* The batched draw the benchmark times (32 problems, seed 4: N in
  {64, 256, 1024, 2048}, M in {64, 256, 1024}, F in {1, 4, 8}, T up to 2^17,
  L = 2^16 / M; about 9 GB per call) runs through one Batch over two calls;
  every problem is compared with the oracle over its two-call stream.
* The two serving arrays the benchmark drives (N = 256 and N = 2048, F = 4,
  49152-sample frames, M = 256, L = 256) take three frames each, submitted
  interleaved to one server: each frame equals the array's own plan fed its
  frames in order, bit for bit, and each array's stream equals the oracle's.

Flag thresholds come from the oracle's App. B model (delta, sigma_V at the
generator's per-input RMS).
"""
import sys
import time
from concurrent.futures import ThreadPoolExecutor
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


def _oracle_thresholds(w):
    return oracle.digitised_expectation(w.sigma, w.block_len)


def test_batched_draw_two_calls():
    ws = synth.batched(seed=4)
    t0 = time.perf_counter()
    streams, plans = [], []
    for w in ws:
        # Two calls of T samples: one seeded draw of 2T samples, cut in half.
        w2 = synth.Workload(w.name, w.n_inputs, w.n_channels, 2 * w.n_samples, w.block_len, w.seed, w.sigma,
                            [], w.norm_window)
        streams.append(synth.generate(w2))
        delta, sig = _oracle_thresholds(w)
        plans.append(dict(n_inputs=w.n_inputs, n_channels=w.n_channels, n_samples=w.n_samples,
                          block_len=w.block_len, norm_window=w.norm_window, k_sigma=5.0,
                          expect_offset=delta, sigma_override=sig))
    total = sum(x.nbytes for x in streams)
    shapes = sorted({(w.n_inputs, w.block_len, w.n_channels) for w in ws})
    _say(f"batched draw: {len(ws)} problems, {total / 1e9:.2f} GB over two calls, generated in "
         f"{time.perf_counter() - t0:.1f} s; (N, M, F) classes {shapes}")
    assert any(w.block_len == 1024 for w in ws) and any(w.n_inputs == 2048 for w in ws)
    firsts = [torch.from_numpy(x[:w.n_samples]).to(DEV) for x, w in zip(streams, ws)]
    seconds = [torch.from_numpy(x[w.n_samples:]).to(DEV) for x, w in zip(streams, ws)]
    batch = sk.Batch(plans, firsts, autotune=False, use_graph=True, want=sk.ALL_OUTPUTS)
    got = [[], []]
    for call, xs in enumerate((firsts, seconds)):
        outs = batch.compute(xs if call else None)
        torch.cuda.synchronize()
        got[call] = [{k: getattr(o, k).cpu() for k in sk.ALL_OUTPUTS} for o in outs]
        _say(f"batched call {call + 1} done")
    batch.close()
    del firsts, seconds
    torch.cuda.empty_cache()

    def ref(j):
        w = ws[j]
        return oracle.sk(streams[j], w.block_len, w.norm_window, 0, 5.0, plans[j]["expect_offset"],
                         plans[j]["sigma_override"])

    with ThreadPoolExecutor(max_workers=8) as ex:
        refs = list(ex.map(ref, range(len(ws))))
    _say("oracle done")
    for j, w in enumerate(ws):
        cat = {k: torch.cat([got[0][j][k], got[1][j][k]], dim=1) for k in sk.ALL_OUTPUTS}
        check_result(SimpleNamespace(**cat), refs[j], w.block_len, w.norm_window, 0, 5.0,
                     plans[j]["expect_offset"], plans[j]["sigma_override"],
                     what=f"batched problem {j} N={w.n_inputs} M={w.block_len} F={w.n_channels} T={w.n_samples}")


def test_serving_arrays_alone_equals_mix_and_oracle():
    n_frames = 3
    arrays = []
    for N in (256, 2048):
        w = synth.serving_array(N)
        frames = [synth.generate(synth.serving_array(N, frame=k)) for k in range(n_frames)]
        delta, sig = _oracle_thresholds(w)
        kw = dict(n_inputs=N, n_channels=w.n_channels, n_samples=w.n_samples, block_len=w.block_len,
                  norm_window=w.norm_window, k_sigma=5.0, expect_offset=delta, sigma_override=sig)
        arrays.append(dict(w=w, frames=frames, kw=kw))
    _say("serving arrays: " + ", ".join(f"N={a['kw']['n_inputs']} F={a['kw']['n_channels']} "
                                        f"T={a['kw']['n_samples']} M={a['kw']['block_len']} "
                                        f"L={a['kw']['norm_window']}" for a in arrays))
    # Alone: each array's own plan fed its frames in order.
    alone = []
    for a in arrays:
        p = sk.Plan(**a["kw"])
        outs = []
        for f in a["frames"]:
            r = p.compute(torch.from_numpy(f).to(DEV), want=sk.ALL_OUTPUTS)
            outs.append({k: getattr(r, k).cpu().numpy() for k in sk.ALL_OUTPUTS})
        torch.cuda.synchronize()
        p.close()
        alone.append(outs)
    # Mix: frames of both arrays submitted interleaved (each array's in order).
    srv = sk.Server(hbm_budget_bytes=4 << 30, max_inflight=4, n_streams=2)
    ids = [srv.add_array(**a["kw"]) for a in arrays]
    dev = [[torch.from_numpy(f).to(DEV) for f in a["frames"]] for a in arrays]
    order = [0, 1, 1, 0, 0, 1]
    nxt = [0, 0]
    tickets = []
    for a in order:
        k = nxt[a]
        nxt[a] += 1
        out = srv.alloc_outputs(ids[a], DEV, want=sk.ALL_OUTPUTS)
        t = srv.submit(ids[a], dev[a][k], out, tag=a * 10 + k)
        assert t is not None
        tickets.append((a, k, t, out))
    srv.drain()
    for a, k, t, out in tickets:
        r = srv.poll(t)
        assert r is not None and r.status == 0 and r.tag == a * 10 + k
        for key in sk.ALL_OUTPUTS:
            g = getattr(out, key).cpu().numpy()
            assert np.array_equal(g, alone[a][k][key], equal_nan=g.dtype.kind == "f"), (a, k, key)
    srv.close()
    _say("serving: alone equals mix")
    for a, outs in zip(arrays, alone):
        kw = a["kw"]
        x = np.concatenate(a["frames"], axis=0)
        ref = oracle.sk(x, kw["block_len"], kw["norm_window"], 0, 5.0, kw["expect_offset"], kw["sigma_override"])
        cat = {key: torch.from_numpy(np.concatenate([o[key] for o in outs], axis=1)) for key in sk.ALL_OUTPUTS}
        check_result(SimpleNamespace(**cat), ref, kw["block_len"], kw["norm_window"], 0, 5.0, kw["expect_offset"],
                     kw["sigma_override"], what=f"serving array N={kw['n_inputs']}")
