"""Comparison helpers for GPU-vs-oracle parity tests.

Bar: integer outputs (S1, S2, R1, R2, N_eff) bit-exact; V within
1e-6 * max(1, |V_oracle|); flags identical wherever the oracle's V lies more
than 1e-6 from a threshold (decided by re-flagging V +- 1e-6 with the oracle:
if the three decisions agree, no threshold is within 1e-6).
"""
import numpy as np

import oracle

V_TOL = 1e-6


def check_result(gpu, ref, M, L, est=0, k=5.0, delta=0.0, sigma_override=0.0, what=""):
    tag = f"[{what}] " if what else ""
    for name, g, r in (("S1", gpu.s1, ref.S1), ("S2", gpu.s2, ref.S2), ("R1", gpu.r1, ref.R1),
                       ("R2", gpu.r2, ref.R2), ("n_eff", gpu.n_eff, ref.n_eff)):
        if g is None:
            continue
        g = g.cpu().numpy()
        if not np.array_equal(g.astype(np.int64), np.asarray(r).astype(np.int64)):
            bad = np.argwhere(g.astype(np.int64) != np.asarray(r).astype(np.int64))
            raise AssertionError(f"{tag}{name} differs at {len(bad)} places, first {bad[:3].tolist()}: "
                                 f"gpu {g[tuple(bad[0])]} oracle {np.asarray(r)[tuple(bad[0])]}")
    if gpu.v is not None:
        v = gpu.v.cpu().numpy().astype(np.float64)
        nan_g, nan_r = np.isnan(v), np.isnan(ref.V)
        assert np.array_equal(nan_g, nan_r), f"{tag}NaN pattern differs"
        ok = ~nan_r
        err = np.abs(v[ok] - ref.V[ok]) / np.maximum(1.0, np.abs(ref.V[ok]))
        if err.size:
            assert err.max() <= V_TOL, f"{tag}V max rel err {err.max():.3e} at {np.argwhere(ok)[err.argmax()]}"
    sk_i = getattr(gpu, "sk_i", None)
    if sk_i is not None:
        g = sk_i.cpu().numpy().astype(np.float64)
        r = oracle.sk_per_input(ref.S1, ref.S2, M)
        assert np.array_equal(np.isnan(g), np.isnan(r)), f"{tag}sk_i NaN pattern differs"
        ok = ~np.isnan(r)
        if ok.any():
            err = np.abs(g[ok] - r[ok]) / np.maximum(1.0, np.abs(r[ok]))
            assert err.max() <= V_TOL, f"{tag}sk_i max rel err {err.max():.3e}"
    sig = getattr(gpu, "significance", None)
    if sig is not None:
        g = sig.cpu().numpy().astype(np.float64)
        r = oracle.significance(ref.V, ref.n_eff, M, L, est, delta, sigma_override)
        assert np.array_equal(np.isnan(g), np.isnan(r)), f"{tag}significance NaN pattern differs"
        ok = ~np.isnan(r)
        if ok.any():
            err = np.abs(g[ok] - r[ok]) / np.maximum(1.0, np.abs(r[ok]))
            assert err.max() <= V_TOL, f"{tag}significance max rel err {err.max():.3e}"
    if gpu.flags is not None:
        fl = gpu.flags.cpu().numpy()
        Vr = ref.V
        ne = ref.n_eff
        f0 = oracle.flags(Vr, ne, M, L, est, k, delta, sigma_override)
        fm = oracle.flags(Vr - V_TOL, ne, M, L, est, k, delta, sigma_override)
        fp = oracle.flags(Vr + V_TOL, ne, M, L, est, k, delta, sigma_override)
        assert np.array_equal(f0, ref.flags)
        clear = (f0 == fm) & (f0 == fp)
        assert np.array_equal(fl[clear], ref.flags[clear]), f"{tag}flags differ at {np.argwhere((fl != ref.flags) & clear)[:5].tolist()}"
        return int(clear.sum()), int(fl.size)
    return None
