"""GPU tests of the continuous-batching server.

Each frame's results are the same alone (a plan fed the array's frames in
order) and in the mix (frames of several arrays submitted as they arrive,
admitted by device-memory footprint, overlapping on the device), bit for bit;
one array is also checked against the CPU oracle over its whole stream."""
import time

import numpy as np
import pytest

import oracle
import synth
from parity import check_result

torch = pytest.importorskip("torch")
sk = pytest.importorskip("paper_1808_10365_amd")

pytestmark = pytest.mark.gpu
DEV = "cuda:0"

ARRAYS = [
    dict(n_inputs=64, n_channels=2, n_samples=4096, block_len=256, norm_window=16, k_sigma=5.0),
    dict(n_inputs=512, n_channels=4, n_samples=2048, block_len=256, norm_window=16, k_sigma=5.0),
    dict(n_inputs=48, n_channels=3, n_samples=1024, block_len=64, norm_window=1, k_sigma=4.0),
]


def _frames(kw, n, seed):
    w = synth.Workload("a", kw["n_inputs"], kw["n_channels"], kw["n_samples"] * n, kw["block_len"], seed,
                       np.random.default_rng(seed).uniform(1.5, 3.5, kw["n_inputs"]), [])
    x = synth.generate(w, nthreads=4)
    T = kw["n_samples"]
    return x, [np.ascontiguousarray(x[k * T:(k + 1) * T]) for k in range(n)]


def _alone(kw, frames):
    p = sk.Plan(**kw)
    outs = []
    for f in frames:
        r = p.compute(torch.from_numpy(f).to(DEV), want=sk.ALL_OUTPUTS)
        outs.append({k: getattr(r, k).cpu().numpy() for k in sk.ALL_OUTPUTS})
    torch.cuda.synchronize()
    p.close()
    return outs


@pytest.mark.parametrize("budget_frames,inflight", [(1, 1), (3, 4), (64, 16)])
def test_alone_equals_mix(budget_frames, inflight):
    nfr = 6
    data = [_frames(kw, nfr, 40 + j) for j, kw in enumerate(ARRAYS)]
    alone = [_alone(kw, fr) for kw, (_, fr) in zip(ARRAYS, data)]
    big = max(kw["n_samples"] * kw["n_channels"] * kw["n_inputs"] * 2 for kw in ARRAYS)
    srv = sk.Server(hbm_budget_bytes=budget_frames * big, max_inflight=inflight, n_streams=3)
    ids = [srv.add_array(**kw) for kw in ARRAYS]
    # Interleave submissions in a seeded random order that keeps each array's
    # frames in order (as arrivals from independent arrays would).
    rng = np.random.default_rng(7)
    order = np.repeat(np.arange(len(ARRAYS)), nfr)
    rng.shuffle(order)
    nxt = [0] * len(ARRAYS)
    dev_frames = [[torch.from_numpy(f).to(DEV) for f in fr] for _, fr in data]
    torch.cuda.synchronize()
    tickets = []
    for a in order:
        k = nxt[a]
        nxt[a] += 1
        out = srv.alloc_outputs(ids[a], DEV, want=sk.ALL_OUTPUTS)
        t = srv.submit(ids[a], dev_frames[a][k], out, tag=a * 100 + k)
        assert t is not None
        tickets.append((a, k, t, out))
        time.sleep(float(rng.exponential(2e-4)))
    srv.drain()
    for a, k, t, out in tickets:
        r = srv.poll(t)
        assert r is not None and r.status == 0 and r.tag == a * 100 + k
        assert r.t_submit <= r.t_admit <= r.t_done
        for key in sk.ALL_OUTPUTS:
            g = getattr(out, key).cpu().numpy()
            assert np.array_equal(g, alone[a][k][key], equal_nan=(key == "v")), (a, k, key)
    st = srv.stats()
    assert st.completed == len(order) and st.peak_inflight <= inflight
    assert st.peak_bytes <= budget_frames * big
    if budget_frames == 1:
        assert st.peak_inflight == 1
    srv.close()
    # Oracle over the first array's whole stream.
    x, _ = data[0]
    kw = ARRAYS[0]
    ref = oracle.sk(x, kw["block_len"], kw["norm_window"], 0, kw["k_sigma"])

    class G:
        pass
    g = G()
    for key in sk.ALL_OUTPUTS:
        setattr(g, key, torch.from_numpy(np.concatenate([alone[0][k][key] for k in range(nfr)], axis=1)))
    check_result(g, ref, kw["block_len"], kw["norm_window"], 0, kw["k_sigma"], what="server array 0")


def test_host_staged_frames():
    kw = ARRAYS[1]
    _, frames = _frames(kw, 4, 99)
    alone = _alone(kw, frames)
    srv = sk.Server(hbm_budget_bytes=1 << 30, max_inflight=4, n_streams=2)
    aid = srv.add_array(**kw)
    pinned = [torch.from_numpy(f).pin_memory() for f in frames]
    outs = [srv.alloc_outputs(aid, DEV, want=sk.ALL_OUTPUTS) for _ in frames]
    ts = [srv.submit(aid, p, o, tag=j) for j, (p, o) in enumerate(zip(pinned, outs))]
    srv.drain()
    for j, (t, o) in enumerate(zip(ts, outs)):
        assert srv.poll(t).status == 0
        for key in sk.ALL_OUTPUTS:
            assert np.array_equal(getattr(o, key).cpu().numpy(), alone[j][key], equal_nan=(key == "v"))
    srv.close()


def test_queue_capacity_and_errors():
    kw = ARRAYS[2]
    _, frames = _frames(kw, 1, 5)
    srv = sk.Server(hbm_budget_bytes=1 << 28, max_inflight=1, n_streams=1, queue_capacity=1)
    aid = srv.add_array(**kw)
    f = torch.from_numpy(frames[0]).to(DEV)
    accepted = rejected = 0
    tickets = []
    for j in range(40):
        o = srv.alloc_outputs(aid, DEV)
        t = srv.submit(aid, f, o, tag=j)
        if t is None:
            rejected += 1
        else:
            accepted += 1
            tickets.append(t)
    srv.drain()
    assert accepted + rejected == 40 and accepted >= 1
    assert srv.stats().rejected_full == rejected
    for t in tickets:
        assert srv.poll(t).status == 0
    with pytest.raises(sk.SKError):
        srv.poll(tickets[0])                 # already collected
    with pytest.raises(ValueError):
        srv.submit(7, f, srv.alloc_outputs(aid, DEV))   # unknown array
    tiny = sk.Server(hbm_budget_bytes=1024, max_inflight=1, n_streams=1)
    tid = tiny.add_array(**kw)
    with pytest.raises(sk.SKError):
        tiny.submit(tid, f, tiny.alloc_outputs(tid, DEV))   # frame larger than the budget
    tiny.close()
    srv.close()
