"""GPU parity of the App. A diagnostic (per-channel mean, variance and
effective receiver count of the estimator), and the synthetic reproduction of
App. A's trend: the effective count falls from N toward 1 as a common-mode
signal grows."""
import numpy as np
import pytest

import oracle
import synth

torch = pytest.importorskip("torch")
sk = pytest.importorskip("paper_1808_10365_amd")

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def test_channel_stats_parity():
    rng = np.random.default_rng(2)
    v = rng.normal(0.95, 0.02, size=(5, 3001)).astype(np.float32)
    v[2, ::5] = np.nan
    v[4, :] = np.nan
    v[3, 1:] = np.nan
    mean, var, ne, cnt = [t.cpu().numpy() for t in sk.channel_stats(torch.from_numpy(v).to(DEV), 256)]
    rm, rv, rn, rc = oracle.channel_stats(v.astype(np.float64), 256)
    assert np.array_equal(cnt, rc)
    for g, r in ((mean, rm), (var, rv), (ne, rn)):
        assert np.array_equal(np.isnan(g), np.isnan(r))
        ok = ~np.isnan(r)
        assert np.all(np.abs(g[ok] - r[ok]) <= 1e-9 * np.maximum(1.0, np.abs(r[ok])))


def test_common_mode_sweep_on_gpu():
    N, M, B = 64, 256, 400
    effs = []
    for amp in (0.0, 1.0, 2.0):
        w = synth.common_mode(N, B, M, amp, seed=13, sigma=1.0, n_channels=2)
        x = synth.generate(w, nthreads=4)
        plan = sk.Plan(N, 2, B * M, M, norm_window=1, estimator=sk.EST_TILDE)
        out = plan.compute(torch.from_numpy(x).to(DEV))
        mean, var, ne, cnt = [t.cpu().numpy() for t in sk.channel_stats(out.v, M)]
        ref = oracle.channel_stats(out.v.cpu().numpy().astype(np.float64), M)
        assert np.allclose(ne, ref[2], rtol=1e-9)
        effs.append(float(ne.mean()))
    assert 0.8 * N < effs[0] < 1.25 * N
    assert effs[0] > effs[1] > effs[2]
