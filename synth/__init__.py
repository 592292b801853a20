"""Seeded synthetic inputs: 4+4-bit offset-encoded complex voltages, [T][F][N] bytes.

This module holds no spectral-kurtosis arithmetic. It makes input bytes (and
the per-input Gaussian RMS it used) that both the CPU oracle and the GPU
library consume. The byte generator is C (``synth.c``), counter-based, so the
bytes do not depend on the thread count.

Workloads (the paper's instruments, restated as synthetic inputs; the
on-sky data of Sec. 3.2 is not available):

* ``tiny``       N=16, F=1, T=4096, sigma=2.5, a tone of amplitude 5 in 256-sample
                 blocks 3-5 on every input.
* ``pathfinder`` N=256, F=8, T=2^17, sigma_i ~ U[1.5, 3.5], 4 inputs at gain x2,
                 tones in 2 channels, 20 impulsive 8-sample bursts (amplitude 7)
                 in 1 channel (Sec. 3.1: the Pathfinder has 256 receivers).
* ``chime``      N=2048, F=4, T=2^18, sigma_i ~ U[1.5, 3.5], a tone whose offset
                 sweeps across 1 channel in the middle third of T, and on/off noise bursts in 5 % of the
                 256-sample blocks (Sec. 3.1: each CHIME GPU chip sees all 2048
                 receivers).
* ``batched``    32 problems, N in {64,256,1024,2048}, M in {64,256,1024},
                 F in {1,4,8}, T = M * U{1..2^17/M}.
* ``serving``    frames of F=4 x 49152 samples from arrays of N=256 and N=2048.

App. B fixes the data model: Gaussian components bounded to [-7, 7], with
CHIME's RMS of about 1.52 counts per component.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass, field
from typing import List, Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "libsynth.so")
_lib = None

TONE, NOISE, BURST, COMMON = 1, 2, 3, 4


class _Event(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("channel", ctypes.c_int32),
                ("t0", ctypes.c_int64), ("t1", ctypes.c_int64),
                ("amplitude", ctypes.c_double), ("nu0", ctypes.c_double),
                ("nu1", ctypes.c_double)]


class _Desc(ctypes.Structure):
    _fields_ = [("n_inputs", ctypes.c_int32), ("n_channels", ctypes.c_int32),
                ("n_samples", ctypes.c_int64), ("seed", ctypes.c_uint64),
                ("sigma", ctypes.POINTER(ctypes.c_double)),
                ("events", ctypes.POINTER(_Event)), ("n_events", ctypes.c_int32),
                ("clip", ctypes.c_int32)]


def build(verbose: bool = False) -> str:
    """Compile libsynth.so with gcc (always recompiles)."""
    import subprocess
    src = os.path.join(_HERE, "synth.c")
    tmp = _LIB_PATH + ".tmp"
    cmd = ["gcc", "-O2", "-std=c11", "-D_GNU_SOURCE", "-fPIC", "-shared", src, "-o", tmp, "-lm", "-lpthread"]
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
        lib.synth_fill.argtypes = [ctypes.POINTER(_Desc), ctypes.c_void_p, ctypes.c_int]
        lib.synth_fill.restype = ctypes.c_int
        lib.synth_thresholds.argtypes = [ctypes.c_double, ctypes.c_int, ctypes.POINTER(ctypes.c_uint32)]
        lib.synth_thresholds.restype = None
        lib.synth_splitmix64.argtypes = [ctypes.c_uint64, ctypes.c_uint64]
        lib.synth_splitmix64.restype = ctypes.c_uint64
        _lib = lib
    return _lib


@dataclass
class Event:
    kind: int
    channel: int
    t0: int
    t1: int
    amplitude: float
    nu0: float = 0.0
    nu1: float = 0.0


@dataclass
class Workload:
    """One synthetic input stream: shape, per-input RMS and RFI events."""
    name: str
    n_inputs: int
    n_channels: int
    n_samples: int
    block_len: int
    seed: int
    sigma: np.ndarray                      # [N] per-component RMS in counts (gain applied)
    events: List[Event] = field(default_factory=list)
    norm_window: int = 1                   # running-normaliser window in blocks
    clip: int = 7

    @property
    def nbytes(self) -> int:
        return self.n_inputs * self.n_channels * self.n_samples


def generate(w: Workload, nthreads: Optional[int] = None, out: Optional[np.ndarray] = None) -> np.ndarray:
    """Return the packed bytes of ``w`` as a uint8 array of shape [T, F, N]."""
    lib = _load()
    N, F, T = w.n_inputs, w.n_channels, w.n_samples
    if out is None:
        out = np.empty((T, F, N), dtype=np.uint8)
    assert out.shape == (T, F, N) and out.dtype == np.uint8 and out.flags.c_contiguous
    sig = np.ascontiguousarray(w.sigma, dtype=np.float64)
    assert sig.shape == (N,)
    ev = (_Event * max(1, len(w.events)))()
    for k, e in enumerate(w.events):
        ev[k] = _Event(e.kind, e.channel, e.t0, e.t1, e.amplitude, e.nu0, e.nu1)
    d = _Desc(N, F, T, w.seed & 0xFFFFFFFFFFFFFFFF,
              sig.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), ev, len(w.events), w.clip)
    if nthreads is None:
        nthreads = min(16, os.cpu_count() or 1)
    rc = lib.synth_fill(ctypes.byref(d), out.ctypes.data, int(nthreads))
    if rc != 0:
        raise RuntimeError(f"synth_fill failed: {rc}")
    return out


def thresholds(sigma: float, clip: int = 7) -> np.ndarray:
    lib = _load()
    thr = (ctypes.c_uint32 * (2 * clip))()
    lib.synth_thresholds(float(sigma), int(clip), thr)
    return np.array(thr, dtype=np.uint64)


def splitmix64(key: int, n: int) -> int:
    return int(_load().synth_splitmix64(key, n))


# ----------------------------------------------------------------------------- workloads

def tiny(seed: int = 1, norm_window: int = 1) -> Workload:
    rng = np.random.default_rng(seed)
    nu = float(rng.uniform(-0.5, 0.5))
    M = 256
    ev = [Event(TONE, 0, 3 * M, 6 * M, 5.0, nu, nu)]
    return Workload("tiny", 16, 1, 4096, M, seed, np.full(16, 2.5), ev, norm_window)


def pathfinder(seed: int = 2, norm_window: int = 256) -> Workload:
    N, F, T, M = 256, 8, 1 << 17, 256
    rng = np.random.default_rng(seed)
    sigma = rng.uniform(1.5, 3.5, size=N)
    gain_inputs = rng.choice(N, size=4, replace=False)
    sigma[gain_inputs] *= 2.0
    tone_ch = rng.choice(F, size=2, replace=False)
    ev = [Event(TONE, int(c), 0, T, 5.0, float(nu), float(nu))
          for c, nu in zip(tone_ch, rng.uniform(-0.5, 0.5, size=2))]
    burst_ch = int(rng.integers(0, F))
    for t0 in np.sort(rng.choice(T // 8, size=20, replace=False)) * 8:
        ev.append(Event(BURST, burst_ch, int(t0), int(t0) + 8, 7.0))
    return Workload("pathfinder", N, F, T, M, seed, sigma, ev, norm_window)


def chime(seed: int = 3, block_len: int = 256) -> Workload:
    N, F, T = 2048, 4, 1 << 18
    rng = np.random.default_rng(seed)
    sigma = rng.uniform(1.5, 3.5, size=N)
    sweep_ch = int(rng.integers(0, F))
    # The tone's offset sweeps across the channel during the middle third of T.
    ev = [Event(TONE, sweep_ch, T // 3, 2 * T // 3, 5.0, -0.5, 0.5)]
    # On/off noise bursts: 5 % of (channel, 256-sample block) cells, in runs.
    G = 256
    nb = T // G
    target = int(round(0.05 * F * nb))
    on = np.zeros((F, nb), dtype=bool)
    while on.sum() < target:
        f = int(rng.integers(0, F))
        b0 = int(rng.integers(0, nb))
        run = int(rng.integers(1, 9))
        on[f, b0:b0 + run] = True
    for f in range(F):
        b = 0
        while b < nb:
            if on[f, b]:
                e = b
                while e < nb and on[f, e]:
                    e += 1
                ev.append(Event(NOISE, f, b * G, e * G, 5.0))
                b = e
            else:
                b += 1
    L = (1 << 16) // block_len
    return Workload(f"chime_m{block_len}", N, F, T, block_len, seed, sigma, ev, L)


def batched(seed: int = 4, n_problems: int = 32, max_t: int = 1 << 17) -> List[Workload]:
    rng = np.random.default_rng(seed)
    out = []
    for p in range(n_problems):
        N = int(rng.choice([64, 256, 1024, 2048]))
        M = int(rng.choice([64, 256, 1024]))
        F = int(rng.choice([1, 4, 8]))
        T = M * int(rng.integers(1, max_t // M + 1))
        sigma = rng.uniform(1.5, 3.5, size=N)
        L = max(1, (1 << 16) // M)
        out.append(Workload(f"batch{p}", N, F, T, M, seed * 1000 + p, sigma, [], L))
    return out


def serving_array(n_inputs: int, seed: int = 5, n_channels: int = 4, frame_samples: int = 49152,
                  block_len: int = 256, frame: int = 0) -> Workload:
    """Frame ``frame`` of one serving array (each frame is its own seeded draw)."""
    rng = np.random.default_rng(seed * 7919 + n_inputs)
    sigma = rng.uniform(1.5, 3.5, size=n_inputs)
    return Workload(f"serve_n{n_inputs}_f{frame}", n_inputs, n_channels, frame_samples, block_len,
                    (seed << 32) ^ (n_inputs << 20) ^ frame, sigma, [], (1 << 16) // block_len)


def lattice_cw(n_inputs: int, n_channels: int, n_samples: int, seed: int = 11) -> np.ndarray:
    """Constant-modulus input: every sample is one of the 12 integer points with
    Re^2 + Im^2 = 25, so each sample's power is exactly 25."""
    pts = np.array([(5, 0), (-5, 0), (0, 5), (0, -5), (3, 4), (3, -4), (-3, 4), (-3, -4),
                    (4, 3), (4, -3), (-4, 3), (-4, -3)], dtype=np.int64)
    rng = np.random.default_rng(seed)
    k = rng.integers(0, 12, size=(n_samples, n_channels, n_inputs))
    re, im = pts[k, 0], pts[k, 1]
    return (((re + 8) << 4) | (im + 8)).astype(np.uint8)


def encode(re: np.ndarray, im: np.ndarray) -> np.ndarray:
    """Offset-encode integer components in [-8, 7] into bytes (hi = Re+8, lo = Im+8)."""
    re = np.asarray(re, dtype=np.int64)
    im = np.asarray(im, dtype=np.int64)
    assert re.min(initial=0) >= -8 and re.max(initial=0) <= 7 and im.min(initial=0) >= -8 and im.max(initial=0) <= 7
    return (((re + 8) << 4) | (im + 8)).astype(np.uint8)


def uniform_small(n_inputs: int, n_channels: int, n_samples: int, seed: int, vmax: int = 3) -> np.ndarray:
    """Integer components drawn uniformly from [-vmax, vmax], returned as (re, im) int arrays."""
    rng = np.random.default_rng(seed)
    re = rng.integers(-vmax, vmax + 1, size=(n_samples, n_channels, n_inputs))
    im = rng.integers(-vmax, vmax + 1, size=(n_samples, n_channels, n_inputs))
    return re, im


def common_mode(n_inputs: int, n_blocks: int, block_len: int, amplitude: float, seed: int,
                sigma: float = 2.0, n_channels: int = 1) -> Workload:
    """Independent Gaussian inputs of RMS ``sigma`` plus a common-mode Gaussian
    of RMS ``amplitude`` shared by every input (App. A's simulation)."""
    T = n_blocks * block_len
    ev = [Event(COMMON, f, 0, T, float(amplitude)) for f in range(n_channels)] if amplitude > 0 else []
    return Workload(f"cm{amplitude}", n_inputs, n_channels, T, block_len, seed, np.full(n_inputs, float(sigma)), ev, 1)
