"""GPU parity of the App. B Monte-Carlo calibration: every simulated estimate
equals the oracle's (same counter-based generator, exact integer sums), and
the moments agree."""
import numpy as np
import pytest

import oracle

torch = pytest.importorskip("torch")
sk = pytest.importorskip("paper_1808_10365_amd")

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("N,M,sigma,est", [(16, 256, 2.5, 1), (300, 64, 1.52, 0), (5, 1000, 3.5, 1)])
def test_mc_values_match_oracle(N, M, sigma, est):
    n_sim = 300
    m, vals = sk.calibrate_mc(N, M, sigma, n_sim, seed=19, estimator=est, return_values=True)
    g = vals.cpu().numpy()
    r = oracle.mc_calibrate(N, M, sigma, n_sim, seed=19, est=est)
    assert np.all(np.abs(g - r) <= 1e-12 * np.maximum(1.0, np.abs(r)))
    assert abs(m[0] - r.mean()) < 1e-12 and abs(m[1] / r.var(ddof=1) - 1) < 1e-9


def test_mc_large_run_moments():
    # CHIME-like: N = 2048 receivers, n = 256, RMS 1.52 counts (App. B).
    m = sk.calibrate_mc(2048, 256, 1.52, 2000, seed=3)
    K = 2048 * 256
    assert abs(m[0] - 1.0) < 0.01
    assert abs(m[1] / (4 / K) - 1) < 0.15
