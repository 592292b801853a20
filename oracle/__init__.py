"""CPU oracle for the multi-receiver spectral-kurtosis estimator (TEST INFRASTRUCTURE).

Only the test suite, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package. The GPU library never imports it, and
it imports nothing of the GPU library. The arithmetic lives in plain C
(``sk_oracle.c``: int64 sums, FP64 everything else, sums in input order);
this module marshals numpy arrays into it, and adds only the App. B
threshold model's few FP64 formulas over the C code's PMF moments
(``digitised_expectation``). ``exact.py`` recomputes tiny
cases in exact rationals.

Paper: Taylor et al., arXiv:1808.10365, Sec. 2.1-2.2.1 (estimator),
Sec. 3.2 (detection significance), App. B (digitisation).

Every function of the oracle is pinned by a CPU test against something other
than itself; see ``tests/test_oracle_pins.py``.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
# A test may point the oracle at a deliberately broken build (mutation test).
_LIB_PATH = os.environ.get("SK_ORACLE_LIB") or os.path.join(_HERE, "liboracle_sk.so")
_lib = None

EST_HAT, EST_TILDE = 0, 1
FLAG_LOW, FLAG_HIGH, FLAG_INVALID = 1, 2, 4

_i64p = ctypes.POINTER(ctypes.c_int64)
_f64p = ctypes.POINTER(ctypes.c_double)
_i32p = ctypes.POINTER(ctypes.c_int32)
_u8p = ctypes.POINTER(ctypes.c_uint8)


def build(verbose: bool = False, extra_flags=()) -> str:
    """Compile liboracle_sk.so with gcc (always recompiles)."""
    src = os.path.join(_HERE, "sk_oracle.c")
    tmp = _LIB_PATH + ".tmp"
    cmd = ["gcc", "-O2", "-std=gnu11", "-fPIC", "-shared", *extra_flags, src, "-o", tmp, "-lm"]
    if verbose:
        print(" ".join(cmd))
    subprocess.run(cmd, check=True)
    os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build()
        lib = ctypes.CDLL(_LIB_PATH)
        I64, F64, I32, VP = ctypes.c_int64, ctypes.c_double, ctypes.c_int, ctypes.c_void_p
        lib.orc_power.argtypes = [ctypes.c_uint8]
        lib.orc_power.restype = ctypes.c_int
        lib.orc_block_sums.argtypes = [VP, I64, I64, I64, I64, VP, VP]
        lib.orc_block_sums_f64.argtypes = [VP, I64, I64, I64, I64, VP, VP]
        lib.orc_window.argtypes = [VP, VP, I64, I64, I64, I64, I64, VP]
        lib.orc_window_f64.argtypes = [VP, I64, I64, I64, I64, VP]
        lib.orc_flags.argtypes = [VP, VP, I64, I64, I64, I32, F64, F64, F64, VP]
        lib.orc_combine.argtypes = [VP, VP, VP, VP, I64, I64, I64, I64, I64, I32, F64, F64, F64,
                                    VP, VP, VP, VP, VP, VP, VP]
        lib.orc_combine_f64.argtypes = [VP, VP, VP, I64, I64, I64, I64, I64, I32, VP]
        lib.orc_sk_per_input.argtypes = [VP, VP, I64, I64, VP]
        lib.orc_sk.argtypes = [VP, VP, I64, I64, I64, I64, I64, I32, F64, F64, F64, VP, I64,
                               VP, VP, VP, VP, VP, VP, VP, VP]
        lib.orc_sk.restype = ctypes.c_int
        lib.orc_quantised_power_moments.argtypes = [F64, I32, VP]
        lib.orc_mc_codes.argtypes = [I64, I64, I32, F64, ctypes.c_uint64, I64, I64, VP, VP]
        lib.orc_mc_calibrate.argtypes = [I64, I64, I32, I32, F64, I64, ctypes.c_uint64, VP]
        lib.orc_pearson3_quantile.argtypes = [F64, F64, F64, F64]
        lib.orc_pearson3_quantile.restype = ctypes.c_double
        lib.orc_flags_fap.argtypes = [VP, VP, I64, I64, I64, I32, F64, F64, F64, VP, VP, VP]
        lib.orc_channel_stats.argtypes = [VP, I64, I64, I64, VP, VP, VP, VP]
        lib.orc_significance.argtypes = [VP, VP, I64, I64, I64, I32, F64, F64, VP]
        _lib = lib
    return _lib


def _ptr(a: Optional[np.ndarray]):
    return None if a is None else a.ctypes.data


def power(byte: int) -> int:
    """Power of one offset-encoded sample (Sec. 2.2.3, 'Calculating Power')."""
    return int(_load().orc_power(int(byte)))


def power_table() -> np.ndarray:
    return np.array([power(b) for b in range(256)], dtype=np.int64)


def block_sums(x: np.ndarray, M: int):
    """Eq. singlesums for every (f, b, i). x: uint8 [T, F, N] -> S1, S2 int64 [F, B, N]."""
    x = np.ascontiguousarray(x, dtype=np.uint8)
    T, F, N = x.shape
    B = T // M
    S1 = np.empty((F, B, N), np.int64)
    S2 = np.empty((F, B, N), np.int64)
    _load().orc_block_sums(_ptr(x), N, F, T, M, _ptr(S1), _ptr(S2))
    return S1, S2


def block_sums_f64(p: np.ndarray, M: int):
    p = np.ascontiguousarray(p, dtype=np.float64)
    T, F, N = p.shape
    B = T // M
    S1 = np.empty((F, B, N), np.float64)
    S2 = np.empty((F, B, N), np.float64)
    _load().orc_block_sums_f64(_ptr(p), N, F, T, M, _ptr(S1), _ptr(S2))
    return S1, S2


def window(S1: np.ndarray, L: int, hist: Optional[np.ndarray] = None) -> np.ndarray:
    """Normaliser window sums P [F, B, N]; hist is [F, H, N] (oldest first) or None."""
    S1 = np.ascontiguousarray(S1, dtype=np.int64)
    F, B, N = S1.shape
    if hist is None:
        hist = np.zeros((F, 0, N), np.int64)
    hist = np.ascontiguousarray(hist, dtype=np.int64)
    P = np.empty_like(S1)
    _load().orc_window(_ptr(S1), _ptr(hist), hist.shape[1], N, F, B, L, _ptr(P))
    return P


def window_f64(S1: np.ndarray, L: int) -> np.ndarray:
    S1 = np.ascontiguousarray(S1, dtype=np.float64)
    F, B, N = S1.shape
    P = np.empty_like(S1)
    _load().orc_window_f64(_ptr(S1), N, F, B, L, _ptr(P))
    return P


@dataclass
class Result:
    S1: np.ndarray
    S2: np.ndarray
    P: np.ndarray
    A: np.ndarray
    Bq: np.ndarray
    R1: np.ndarray
    R2: np.ndarray
    n_eff: np.ndarray
    V: np.ndarray
    flags: np.ndarray


def combine(S1, S2, P, M, L, est=EST_HAT, k=5.0, delta=0.0, sigma_override=0.0, mask=None) -> Result:
    S1 = np.ascontiguousarray(S1, dtype=np.int64)
    S2 = np.ascontiguousarray(S2, dtype=np.int64)
    P = np.ascontiguousarray(P, dtype=np.int64)
    F, B, N = S1.shape
    if mask is not None:
        mask = np.ascontiguousarray(mask, dtype=np.uint8)
        assert mask.shape == (F, N)
    A = np.empty((F, B)); Bq = np.empty((F, B)); V = np.empty((F, B))
    R1 = np.empty((F, B), np.int64); R2 = np.empty((F, B), np.int64)
    ne = np.empty((F, B), np.int32); fl = np.empty((F, B), np.uint8)
    _load().orc_combine(_ptr(S1), _ptr(S2), _ptr(P), _ptr(mask), N, F, B, M, L, est, k, delta,
                        sigma_override, _ptr(A), _ptr(Bq), _ptr(R1), _ptr(R2), _ptr(ne), _ptr(V), _ptr(fl))
    return Result(S1, S2, P, A, Bq, R1, R2, ne, V, fl)


def sk(x: np.ndarray, M: int, L: int = 1, est: int = EST_HAT, k: float = 5.0, delta: float = 0.0,
       sigma_override: float = 0.0, mask: Optional[np.ndarray] = None,
       hist: Optional[np.ndarray] = None) -> Result:
    """The whole path for one call on bytes x [T, F, N]."""
    x = np.ascontiguousarray(x, dtype=np.uint8)
    T, F, N = x.shape
    if M < 2 or T % M != 0:
        raise ValueError("T must be a multiple of M >= 2")
    if est == EST_TILDE and L != 1:
        raise ValueError("the rescaled estimator is defined for L = 1")
    S1, S2 = block_sums(x, M)
    P = window(S1, L, hist)
    return combine(S1, S2, P, M, L, est, k, delta, sigma_override, mask)


def sk_f64(p: np.ndarray, M: int, L: int = 1, est: int = EST_HAT) -> np.ndarray:
    """V [F, B] from real-valued power p [T, F, N] (continuous chi-squared tests)."""
    S1, S2 = block_sums_f64(p, M)
    P = window_f64(S1, L)
    F, B, N = S1.shape
    V = np.empty((F, B))
    _load().orc_combine_f64(_ptr(S1), _ptr(S2), _ptr(P), N, F, B, M, L, est, _ptr(V))
    return V


def sk_per_input(S1: np.ndarray, S2: np.ndarray, M: int) -> np.ndarray:
    """Eq. originalSK for every entry."""
    S1 = np.ascontiguousarray(S1, dtype=np.int64)
    S2 = np.ascontiguousarray(S2, dtype=np.int64)
    out = np.empty(S1.shape, np.float64)
    _load().orc_sk_per_input(_ptr(S1), _ptr(S2), S1.size, M, _ptr(out))
    return out


def flags(V: np.ndarray, n_eff: np.ndarray, M: int, L: int, est: int = EST_HAT, k: float = 5.0,
          delta: float = 0.0, sigma_override: float = 0.0) -> np.ndarray:
    V = np.ascontiguousarray(V, dtype=np.float64)
    ne = np.ascontiguousarray(n_eff, dtype=np.int32)
    out = np.empty(V.shape, np.uint8)
    _load().orc_flags(_ptr(V), _ptr(ne), V.size, M, L, est, k, delta, sigma_override, _ptr(out))
    return out


def significance(V: np.ndarray, n_eff: np.ndarray, M: int, L: int, est: int = EST_HAT, delta: float = 0.0,
                 sigma_override: float = 0.0) -> np.ndarray:
    """Detection significance (Sec. 3.2): (V - E) / sigma."""
    V = np.ascontiguousarray(V, dtype=np.float64)
    ne = np.ascontiguousarray(n_eff, dtype=np.int32)
    out = np.empty(V.shape, np.float64)
    _load().orc_significance(_ptr(V), _ptr(ne), V.size, M, L, est, delta, sigma_override, _ptr(out))
    return out


def quantised_power_moments(sigma: float, clip: int = 7) -> np.ndarray:
    """[E p, E p^2, E p^3, E p^4] of p = re^2 + im^2 for round-and-clip(N(0, sigma^2)) components."""
    m = np.empty(4)
    _load().orc_quantised_power_moments(float(sigma), int(clip), _ptr(m))
    return m


def digitised_expectation(sigma, M: int, clip: int = 7):
    """App. B threshold model from the exact round-and-clip PMF
    (quantised_power_moments): (delta, sigma_V) for inputs of per-component
    RMS sigma[i] and block length M.

    With q = p / E[p] per input, kappa_i = E[q^2] (2 for chi-squared power):
      delta = mean_i kappa_i - 2  (the offset of the mean of V from 1; App. B
              adds it to the expectation of the thresholds);
      sigma_V from the first-order delta method on V + 1 = K sum q^2 / (sum q)^2,
              Var V = (M / K^2) sum_i [Var(q^2) - 4 kbar Cov(q, q^2) + 4 kbar^2 Var(q)],
              times (K + 1) / (K - 1) as in Eq. avgSK; for chi-squared power
              it reduces to the paper's 4/K (Eq. final).
    Plain per-input loops in FP64."""
    sig = np.atleast_1d(np.asarray(sigma, dtype=np.float64))
    n = sig.size
    k2 = np.empty(n)
    k3 = np.empty(n)
    k4 = np.empty(n)
    for i in range(n):
        m = quantised_power_moments(float(sig[i]), clip)
        mu = m[0]
        k2[i] = m[1] / mu ** 2
        k3[i] = m[2] / mu ** 3
        k4[i] = m[3] / mu ** 4
    kbar = float(k2.mean())
    acc = 0.0
    for i in range(n):
        var_q = k2[i] - 1.0
        var_q2 = k4[i] - k2[i] ** 2
        cov = k3[i] - k2[i]
        acc += var_q2 - 4.0 * kbar * cov + 4.0 * kbar ** 2 * var_q
    K = float(n * M)
    return kbar - 2.0, (K + 1.0) / (K - 1.0) * float(np.sqrt(M / (K * K) * acc))


def stream(frames, M: int, L: int, **kw) -> Result:
    """Oracle over a stream cut into frames: the frames are concatenated in time
    and evaluated in one call, so the window sees every earlier block."""
    x = np.concatenate([np.asarray(f, dtype=np.uint8) for f in frames], axis=0)
    return sk(x, M, L, **kw)


def channel_stats(V: np.ndarray, M: int):
    """App. A diagnostic per channel: mean, unbiased variance of V over blocks,
    N_eff = 4 / (M var), and the number of valid blocks."""
    V = np.ascontiguousarray(V, dtype=np.float64)
    F, B = V.shape
    mean, var, ne = np.empty(F), np.empty(F), np.empty(F)
    cnt = np.empty(F, np.int64)
    _load().orc_channel_stats(_ptr(V), F, B, M, _ptr(mean), _ptr(var), _ptr(ne), _ptr(cnt))
    return mean, var, ne, cnt


def mc_codes(N: int, M: int, sigma: float, seed: int, s: int, i: int, clip: int = 7):
    """Simulated component codes (re, im) of input i in estimate s (App. B simulation)."""
    re = np.empty(M, np.int32)
    im = np.empty(M, np.int32)
    _load().orc_mc_codes(N, M, clip, float(sigma), seed & 0xFFFFFFFFFFFFFFFF, s, i, _ptr(re), _ptr(im))
    return re, im


def mc_calibrate(N: int, M: int, sigma: float, n_sim: int, seed: int, est: int = EST_TILDE, clip: int = 7):
    """Estimator values of n_sim simulated digitised blocks (App. B), own-block normalisation."""
    v = np.empty(n_sim)
    _load().orc_mc_calibrate(N, M, est, clip, float(sigma), n_sim, seed & 0xFFFFFFFFFFFFFFFF, _ptr(v))
    return v


def pearson3_quantile(mean: float, sd: float, skew: float, p: float) -> float:
    return float(_load().orc_pearson3_quantile(mean, sd, skew, p))


def flags_fap(V, n_eff, M: int, L: int, est: int = EST_HAT, fap: float = 1e-3, delta: float = 0.0,
              sigma_override: float = 0.0):
    """Flags with false-alarm thresholds; returns (flags, lo, hi)."""
    V = np.ascontiguousarray(V, dtype=np.float64)
    ne = np.ascontiguousarray(n_eff, dtype=np.int32)
    fl = np.empty(V.shape, np.uint8)
    lo = np.empty(V.shape)
    hi = np.empty(V.shape)
    _load().orc_flags_fap(_ptr(V), _ptr(ne), V.size, M, L, est, fap, delta, sigma_override, _ptr(lo), _ptr(hi), _ptr(fl))
    return fl, lo, hi
