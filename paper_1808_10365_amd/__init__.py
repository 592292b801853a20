"""MI355X multi-receiver spectral-kurtosis library: Python binding.

Thin ctypes binding over ``libsk.so`` (C ABI in ``include/sk.h``). It only
marshals arguments: torch tensors give device pointers and HIP streams; every
step of the computation runs in the library's HIP kernels. Importing this
package on a machine without the built library raises immediately; there is
no CPU fallback.

Method: Taylor et al., arXiv:1808.10365, Sec. 2.2.1 (multi-receiver
estimator, Eq. avgSK / final), Sec. 3.2 (flags), App. B (digitisation).
"""
from __future__ import annotations

import ctypes
import os
import sys
from dataclasses import dataclass
from typing import Dict, Optional, Sequence

import torch  # noqa: F401  (loads the HIP runtime the library binds to)

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libsk.so")

SK_OK = 0
SK_ERR_INVALID_ARG, SK_ERR_SHAPE, SK_ERR_NOMEM, SK_ERR_DEVICE, SK_ERR_AGAIN, SK_ERR_STATE = -1, -2, -3, -4, -5, -6
EST_HAT, EST_TILDE = 0, 1
FLAG_LOW, FLAG_HIGH, FLAG_INVALID = 1, 2, 4


class SKError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"sk error {code}: {msg}")
        self.code = code


class PlanDesc(ctypes.Structure):
    _fields_ = [("n_inputs", ctypes.c_int32), ("n_channels", ctypes.c_int32),
                ("n_samples", ctypes.c_int64), ("block_len", ctypes.c_int32),
                ("norm_window_blocks", ctypes.c_int32), ("estimator", ctypes.c_int32),
                ("k_sigma", ctypes.c_double), ("expect_offset", ctypes.c_double),
                ("sigma_override", ctypes.c_double)]


class Outputs(ctypes.Structure):
    _fields_ = [("s1", ctypes.c_void_p), ("s2", ctypes.c_void_p), ("r1", ctypes.c_void_p),
                ("r2", ctypes.c_void_p), ("v", ctypes.c_void_p), ("flags", ctypes.c_void_p),
                ("n_eff", ctypes.c_void_p), ("sk_i", ctypes.c_void_p), ("significance", ctypes.c_void_p)]


class PlanTuning(ctypes.Structure):
    _fields_ = [("pass_a_variant", ctypes.c_int32), ("pass_a_lanes", ctypes.c_int32),
                ("pass_a_blocks", ctypes.c_int32), ("pass_a_chunk_sums", ctypes.c_int32),
                ("pass_b_chunk", ctypes.c_int32),
                ("pass_b_vec", ctypes.c_int32), ("candidates", ctypes.c_int32),
                ("ms_pass_a", ctypes.c_float), ("ms_pass_b", ctypes.c_float),
                ("ms_library_pass_a", ctypes.c_float), ("ms_library_pass_b", ctypes.c_float)]


class McDesc(ctypes.Structure):
    _fields_ = [("n_inputs", ctypes.c_int32), ("block_len", ctypes.c_int32), ("estimator", ctypes.c_int32),
                ("clip", ctypes.c_int32), ("sigma", ctypes.c_double), ("n_sim", ctypes.c_int64),
                ("seed", ctypes.c_uint64)]


class ServerDesc(ctypes.Structure):
    _fields_ = [("hbm_budget_bytes", ctypes.c_size_t), ("max_inflight", ctypes.c_int32),
                ("n_streams", ctypes.c_int32), ("queue_capacity", ctypes.c_int32)]


class ServerResult(ctypes.Structure):
    _fields_ = [("tag", ctypes.c_uint64), ("array_id", ctypes.c_int32), ("status", ctypes.c_int32),
                ("t_submit", ctypes.c_double), ("t_admit", ctypes.c_double), ("t_done", ctypes.c_double)]


class ServerStats(ctypes.Structure):
    _fields_ = [("submitted", ctypes.c_uint64), ("completed", ctypes.c_uint64), ("rejected_full", ctypes.c_uint64),
                ("peak_inflight", ctypes.c_int32), ("peak_bytes", ctypes.c_size_t), ("busy_seconds", ctypes.c_double)]


class BatchOpts(ctypes.Structure):
    _fields_ = [("autotune", ctypes.c_int32), ("use_graph", ctypes.c_int32), ("tune_cache", ctypes.c_char_p)]


_lib = None


def load_library():
    """Load libsk.so (built by ``__graft_entry__.build()``); raise if absent."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is not built; run __graft_entry__.build() (the HIP library is required)")
    lib = ctypes.CDLL(LIB_PATH)
    VP, I32, I64, F64, SZ = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_double, ctypes.c_size_t
    lib.sk_last_error.restype = ctypes.c_char_p
    lib.sk_plan_create.argtypes = [ctypes.POINTER(PlanDesc), ctypes.POINTER(VP)]
    lib.sk_plan_destroy.argtypes = [VP]
    lib.sk_plan_device_bytes.argtypes = [VP, ctypes.POINTER(SZ)]
    lib.sk_compute.argtypes = [VP, VP, VP, ctypes.POINTER(Outputs), VP]
    lib.sk_flags.argtypes = [VP, VP, VP, VP, I64, VP]
    lib.sk_compute_noalloc.argtypes = [ctypes.POINTER(PlanDesc), VP, VP, ctypes.POINTER(Outputs), VP]
    lib.sk_compute_noalloc.restype = ctypes.c_int
    lib.sk_noalloc_scratch_bytes.restype = ctypes.c_size_t
    lib.sk_state_reset.argtypes = [VP]
    lib.sk_state_size.argtypes = [VP, ctypes.POINTER(SZ)]
    lib.sk_state_export.argtypes = [VP, VP, SZ, VP]
    lib.sk_state_import.argtypes = [VP, VP, SZ, VP]
    lib.sk_digitised_expectation.argtypes = [VP, I32, I32, I32, ctypes.POINTER(F64), ctypes.POINTER(F64)]
    lib.sk_plan_set_pass_a_tile.argtypes = [VP, I32]
    lib.sk_plan_get_pass_a_tile.argtypes = [VP, VP, ctypes.POINTER(I32), ctypes.POINTER(I32), ctypes.POINTER(I64)]
    lib.sk_plan_set_pass_a_variant.argtypes = [VP, I32, I32]
    lib.sk_plan_set_pass_b_tile.argtypes = [VP, I32, I32]
    lib.sk_plan_set_pass_b_tile.restype = ctypes.c_int
    lib.sk_plan_autotune.argtypes = [VP, VP, I32, VP, ctypes.POINTER(PlanTuning)]
    lib.sk_plan_autotune.restype = ctypes.c_int
    lib.sk_profile_enable.argtypes = [VP, I32]
    lib.sk_profile_set_stride.argtypes = [VP, I32]
    lib.sk_profile_read.argtypes = [VP, VP, VP, I32, ctypes.POINTER(I32)]
    lib.sk_batch_create.argtypes = [ctypes.POINTER(PlanDesc), I32, ctypes.POINTER(BatchOpts), VP, ctypes.POINTER(Outputs), ctypes.POINTER(VP)]
    lib.sk_batch_compute.argtypes = [VP, VP, VP]
    lib.sk_batch_state_reset.argtypes = [VP, VP]
    lib.sk_batch_get_tiles.argtypes = [VP, I32, ctypes.POINTER(I32), ctypes.POINTER(I32)]
    lib.sk_batch_time_pass_a.argtypes = [VP, VP, ctypes.POINTER(ctypes.c_float)]
    lib.sk_batch_get_tuning.argtypes = [VP, I32, ctypes.POINTER(I32), ctypes.POINTER(I32), ctypes.POINTER(I32),
                                        ctypes.POINTER(I32)]
    lib.sk_batch_destroy.argtypes = [VP]
    lib.sk_batch_get_state.argtypes = [VP, I32, ctypes.POINTER(I32)]
    lib.sk_read_probe.argtypes = [VP, I64, I32, VP, VP]
    lib.sk_plan_set_pass_a_blocks.argtypes = [VP, I32]
    lib.sk_plan_pass_a_timeline.argtypes = [VP, VP, I32, VP, I64, ctypes.POINTER(I64), VP]
    lib.sk_server_now.restype = ctypes.c_double
    lib.sk_server_create.argtypes = [ctypes.POINTER(ServerDesc), ctypes.POINTER(VP)]
    lib.sk_server_add_array.argtypes = [VP, ctypes.POINTER(PlanDesc), ctypes.POINTER(I32)]
    lib.sk_stream_submit.argtypes = [VP, I32, VP, I32, ctypes.POINTER(Outputs), ctypes.c_uint64, VP,
                                     ctypes.POINTER(ctypes.c_uint64)]
    lib.sk_stream_poll.argtypes = [VP, ctypes.c_uint64, ctypes.POINTER(ServerResult)]
    lib.sk_server_drain.argtypes = [VP]
    lib.sk_server_get_stats.argtypes = [VP, ctypes.POINTER(ServerStats)]
    lib.sk_server_destroy.argtypes = [VP]
    lib.sk_pearson3_quantile.argtypes = [F64, F64, F64, F64, ctypes.POINTER(F64)]
    lib.sk_pearson3_quantile.restype = ctypes.c_int
    lib.sk_plan_set_false_alarm.argtypes = [VP, F64]
    lib.sk_plan_set_false_alarm.restype = ctypes.c_int
    lib.sk_plan_get_thresholds.argtypes = [VP, I32, ctypes.POINTER(F64), ctypes.POINTER(F64)]
    lib.sk_plan_get_thresholds.restype = ctypes.c_int
    lib.sk_calibrate_mc.argtypes = [ctypes.POINTER(McDesc), VP, VP, VP]
    lib.sk_calibrate_mc.restype = ctypes.c_int
    lib.sk_channel_stats.argtypes = [VP, I32, I64, I32, VP, VP, VP, VP, VP]
    lib.sk_channel_stats.restype = ctypes.c_int
    for name in ("sk_server_create", "sk_server_add_array", "sk_stream_submit", "sk_stream_poll",
                 "sk_server_drain", "sk_server_get_stats", "sk_server_destroy"):
        getattr(lib, name).restype = ctypes.c_int
    for name in ("sk_batch_create", "sk_batch_compute", "sk_batch_state_reset", "sk_batch_get_tiles", "sk_batch_destroy", "sk_batch_get_state", "sk_batch_time_pass_a",
                 "sk_batch_get_tuning"):
        getattr(lib, name).restype = ctypes.c_int
    for name in ("sk_plan_create", "sk_plan_destroy", "sk_plan_device_bytes", "sk_compute", "sk_flags",
                 "sk_state_reset", "sk_state_size", "sk_state_export", "sk_state_import",
                 "sk_digitised_expectation", "sk_plan_set_pass_a_tile", "sk_plan_get_pass_a_tile",
                 "sk_profile_enable", "sk_profile_set_stride", "sk_profile_read", "sk_plan_set_pass_a_variant", "sk_read_probe",
                 "sk_plan_set_pass_a_blocks", "sk_plan_pass_a_timeline"):
        getattr(lib, name).restype = ctypes.c_int
    _lib = lib
    return lib


def _check(rc: int):
    if rc != SK_OK:
        msg = load_library().sk_last_error()
        raise SKError(rc, msg.decode() if msg else "")


def _ptr(t: Optional[torch.Tensor]):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _stream_handle(stream: Optional[torch.cuda.Stream]):
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def _device_tensor(t, name: str, dtype, shape, device_index: int):
    """Raise ValueError unless t is a contiguous tensor on GPU `device_index`
    with this dtype and exact shape: the library receives raw pointers and
    trusts their extent."""
    if not isinstance(t, torch.Tensor):
        raise ValueError(f"{name} must be a torch tensor")
    if not t.is_cuda or t.device.index != device_index:
        raise ValueError(f"{name} must live on cuda:{device_index}, got {t.device}")
    if t.dtype != dtype:
        raise ValueError(f"{name} must be {dtype}, got {t.dtype}")
    if tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} must have shape {tuple(shape)}, got {tuple(t.shape)}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    return t


def _output_specs(F: int, B: int, N: int):
    return {"s1": ((F, B, N), torch.int32), "s2": ((F, B, N), torch.int32), "r1": ((F, B), torch.int64),
            "r2": ((F, B), torch.int64), "v": ((F, B), torch.float32), "flags": ((F, B), torch.uint8),
            "n_eff": ((F, B), torch.int32), "sk_i": ((F, B, N), torch.float32),
            "significance": ((F, B), torch.float32)}


def _check_outputs(out, F: int, B: int, N: int, device_index: int):
    specs = _output_specs(F, B, N)
    for k in ALL_OUTPUTS:
        t = getattr(out, k)
        if t is not None:
            _device_tensor(t, f"output {k}", specs[k][1], specs[k][0], device_index)


def digitised_expectation(sigma: Sequence[float], block_len: int, clip: int = 7):
    """App. B model: (delta, sigma_V) for inputs of per-component RMS ``sigma``."""
    import numpy as np
    s = np.ascontiguousarray(sigma, dtype=np.float64)
    d, sv = ctypes.c_double(), ctypes.c_double()
    _check(load_library().sk_digitised_expectation(s.ctypes.data, len(s), int(block_len), int(clip),
                                                   ctypes.byref(d), ctypes.byref(sv)))
    return d.value, sv.value


def pearson3_quantile(mean: float, sd: float, skew: float, p: float) -> float:
    out = ctypes.c_double()
    _check(load_library().sk_pearson3_quantile(float(mean), float(sd), float(skew), float(p), ctypes.byref(out)))
    return out.value


def calibrate_mc(n_inputs: int, block_len: int, sigma: float, n_sim: int, seed: int, estimator: int = EST_TILDE,
                 clip: int = 7, device="cuda:0", return_values: bool = False):
    """App. B Monte-Carlo on the GPU: moments (mean, var, skew, excess kurtosis) of the
    estimator over n_sim simulated digitised blocks; optionally every value."""
    import numpy as np
    d = McDesc(n_inputs, block_len, estimator, clip, float(sigma), int(n_sim), int(seed) & 0xFFFFFFFFFFFFFFFF)
    m = np.empty(4)
    vals = torch.empty(int(n_sim), dtype=torch.float64, device=device) if return_values else None
    _check(load_library().sk_calibrate_mc(ctypes.byref(d), m.ctypes.data, _ptr(vals), _stream_handle(None)))
    return (m, vals) if return_values else m


def read_probe(x: torch.Tensor, workgroups: int, sink: torch.Tensor,
               stream: Optional[torch.cuda.Stream] = None):
    """Launch the read-only stream probe over the bytes of ``x`` (16-byte
    aligned, size a multiple of 16) on ``stream``; ``sink`` is a device int32
    tensor of at least workgroups * 256 elements."""
    if not (x.is_cuda and x.is_contiguous()) or not (sink.is_cuda and sink.is_contiguous()):
        raise ValueError("x and sink must be contiguous device tensors")
    if sink.dtype != torch.int32 or sink.numel() < workgroups * 256:
        raise ValueError("sink must be int32 with at least workgroups * 256 elements")
    _check(load_library().sk_read_probe(_ptr(x), x.numel() * x.element_size(), int(workgroups), _ptr(sink),
                                        _stream_handle(stream)))


def channel_stats(v: torch.Tensor, block_len: int, stream: Optional[torch.cuda.Stream] = None):
    """App. A diagnostic per channel of v [F][B]: (mean, var, n_eff, count) device tensors."""
    if not isinstance(v, torch.Tensor) or not v.is_cuda or v.dtype != torch.float32 or v.dim() != 2:
        raise ValueError("v must be a float32 device tensor [F][B]")
    v = v.contiguous()
    F, B = v.shape
    mean = torch.empty(F, dtype=torch.float64, device=v.device)
    var = torch.empty_like(mean)
    ne = torch.empty_like(mean)
    cnt = torch.empty(F, dtype=torch.int64, device=v.device)
    _check(load_library().sk_channel_stats(_ptr(v), F, B, int(block_len), _ptr(mean), _ptr(var), _ptr(ne),
                                            _ptr(cnt), _stream_handle(stream)))
    return mean, var, ne, cnt


@dataclass
class Result:
    s1: Optional[torch.Tensor]
    s2: Optional[torch.Tensor]
    r1: Optional[torch.Tensor]
    r2: Optional[torch.Tensor]
    v: Optional[torch.Tensor]
    flags: Optional[torch.Tensor]
    n_eff: Optional[torch.Tensor]
    sk_i: Optional[torch.Tensor] = None
    significance: Optional[torch.Tensor] = None


ALL_OUTPUTS = ("s1", "s2", "r1", "r2", "v", "flags", "n_eff", "sk_i", "significance")
DEFAULT_OUTPUTS = ("s1", "s2", "r1", "r2", "v", "flags", "n_eff")


class Plan:
    """One stream of [T][F][N] frames with its own normaliser state (a ``sk_plan_t``)."""

    def __init__(self, n_inputs: int, n_channels: int, n_samples: int, block_len: int,
                 norm_window: int = 1, estimator: int = EST_HAT, k_sigma: float = 5.0,
                 expect_offset: float = 0.0, sigma_override: float = 0.0):
        self._lib = load_library()
        self.desc = PlanDesc(n_inputs, n_channels, n_samples, block_len, norm_window, estimator,
                             k_sigma, expect_offset, sigma_override)
        self.device_index = torch.cuda.current_device()
        h = ctypes.c_void_p()
        _check(self._lib.sk_plan_create(ctypes.byref(self.desc), ctypes.byref(h)))
        self.handle = h

    @property
    def n_blocks(self) -> int:
        return self.desc.n_samples // self.desc.block_len

    def close(self):
        if self.handle:
            _check(self._lib.sk_plan_destroy(self.handle))
            self.handle = None

    def __del__(self, _finalizing=sys.is_finalizing):
        # At interpreter shutdown the HIP runtime may already be gone: leave
        # the memory to the process exit instead of calling into it.
        if _finalizing():
            return
        try:
            self.close()
        except Exception:
            pass

    def device_bytes(self) -> int:
        n = ctypes.c_size_t()
        _check(self._lib.sk_plan_device_bytes(self.handle, ctypes.byref(n)))
        return n.value

    def set_pass_a_tile(self, lanes_per_row: int):
        _check(self._lib.sk_plan_set_pass_a_tile(self.handle, int(lanes_per_row)))

    def set_pass_b_tile(self, chunk: int = 0, inputs_per_lane: int = 0):
        """Pass B blocks per combine workgroup (1, 2, 4; 0: library choice) and
        inputs per lane (1, 4; 0: library choice)."""
        _check(self._lib.sk_plan_set_pass_b_tile(self.handle, int(chunk), int(inputs_per_lane)))

    def autotune(self, x: torch.Tensor, reps: int = 2, stream: Optional[torch.cuda.Stream] = None) -> dict:
        """Time the plan's tile candidates on the input ``x`` ([T][F][N] uint8 on
        the plan's device) and keep the fastest (``sk_plan_autotune``); the
        normaliser state is kept. Returns the kept settings and their times."""
        d = self.desc
        _device_tensor(x, "x", torch.uint8, (d.n_samples, d.n_channels, d.n_inputs), self.device_index)
        r = PlanTuning()
        _check(self._lib.sk_plan_autotune(self.handle, ctypes.c_void_p(x.data_ptr()), int(reps),
                                          _stream_handle(stream), ctypes.byref(r)))
        return {k: (round(float(getattr(r, k)), 5) if k.startswith("ms_") else int(getattr(r, k)))
                for k, _ in PlanTuning._fields_}

    def set_false_alarm(self, fap: float):
        """Flag at the fap and 1 - fap quantiles of a Pearson III law (0: symmetric k sigma)."""
        _check(self._lib.sk_plan_set_false_alarm(self.handle, float(fap)))

    def thresholds(self, n_eff: int):
        lo, hi = ctypes.c_double(), ctypes.c_double()
        _check(self._lib.sk_plan_get_thresholds(self.handle, int(n_eff), ctypes.byref(lo), ctypes.byref(hi)))
        return lo.value, hi.value

    def pass_a_timeline(self, x: torch.Tensor, simd_balance: bool = True,
                        stream: Optional[torch.cuda.Stream] = None) -> "numpy.ndarray":
        """Per-wavefront timeline of one pass A launch (``sk_plan_pass_a_timeline``):
        int64 rows of (start, reads done, end) in 100 MHz clock ticks, XCD id,
        HW_ID and SIMD. The plan's pass A must be the deferred-store variant."""
        d = self.desc
        _device_tensor(x, "x", torch.uint8, (d.n_samples, d.n_channels, d.n_inputs), self.device_index)
        B = d.n_samples // d.block_len
        cap = 8 * (B * ((d.n_channels * d.n_inputs // 16 + 511) // 512) + 1)
        out = torch.zeros((cap, 6), dtype=torch.int64, device=x.device)
        n = ctypes.c_int64()
        _check(self._lib.sk_plan_pass_a_timeline(self.handle, ctypes.c_void_p(x.data_ptr()), int(bool(simd_balance)),
                                                 ctypes.c_void_p(out.data_ptr()), cap, ctypes.byref(n),
                                                 _stream_handle(stream)))
        (stream or torch.cuda.current_stream(x.device)).synchronize()
        return out[:n.value].cpu().numpy()

    def set_pass_a_blocks(self, blocks: int):
        """Consecutive blocks per pass A task with the packed-table variants (0: library choice)."""
        _check(self._lib.sk_plan_set_pass_a_blocks(self.handle, int(blocks)))

    def set_pass_a_variant(self, variant: int, grid: int = 0):
        """Pass A variant (-1: library choice; 0 shared table, 1/2 packed lane
        table with 8/16 rows per load, 3 blocks side by side, 4 deferred stores)
        and workgroup count (0: one per task)."""
        _check(self._lib.sk_plan_set_pass_a_variant(self.handle, int(variant), int(grid)))

    def alloc_outputs(self, device, want: Sequence[str] = DEFAULT_OUTPUTS) -> Result:
        F, N, B = self.desc.n_channels, self.desc.n_inputs, self.n_blocks
        mk = {
            "s1": lambda: torch.empty((F, B, N), dtype=torch.int32, device=device),
            "s2": lambda: torch.empty((F, B, N), dtype=torch.int32, device=device),
            "r1": lambda: torch.empty((F, B), dtype=torch.int64, device=device),
            "r2": lambda: torch.empty((F, B), dtype=torch.int64, device=device),
            "v": lambda: torch.empty((F, B), dtype=torch.float32, device=device),
            "flags": lambda: torch.empty((F, B), dtype=torch.uint8, device=device),
            "n_eff": lambda: torch.empty((F, B), dtype=torch.int32, device=device),
            "sk_i": lambda: torch.empty((F, B, N), dtype=torch.float32, device=device),
            "significance": lambda: torch.empty((F, B), dtype=torch.float32, device=device),
        }
        return Result(**{k: (mk[k]() if k in want else None) for k in ALL_OUTPUTS})

    def compute_into(self, packed: torch.Tensor, out: Result, mask: Optional[torch.Tensor] = None,
                     stream: Optional[torch.cuda.Stream] = None) -> Result:
        T, F, N = self.desc.n_samples, self.desc.n_channels, self.desc.n_inputs
        dev = self.device_index
        _device_tensor(packed, "packed", torch.uint8, (T, F, N), dev)
        if mask is not None:
            _device_tensor(mask, "mask", torch.uint8, (F, N), dev)
        _check_outputs(out, F, self.n_blocks, N, dev)
        o = Outputs(*[_ptr(getattr(out, k)) for k in ALL_OUTPUTS])
        _check(self._lib.sk_compute(self.handle, _ptr(packed), _ptr(mask), ctypes.byref(o), _stream_handle(stream)))
        return out

    def compute(self, packed: torch.Tensor, mask: Optional[torch.Tensor] = None,
                want: Sequence[str] = DEFAULT_OUTPUTS, stream: Optional[torch.cuda.Stream] = None) -> Result:
        out = self.alloc_outputs(packed.device, want)
        return self.compute_into(packed, out, mask, stream)

    def flags(self, v: torch.Tensor, n_eff: torch.Tensor, stream: Optional[torch.cuda.Stream] = None) -> torch.Tensor:
        v = v.contiguous()
        n_eff = n_eff.contiguous()
        _device_tensor(v, "v", torch.float32, tuple(v.shape), self.device_index)
        _device_tensor(n_eff, "n_eff", torch.int32, tuple(v.shape), self.device_index)
        out = torch.empty(v.shape, dtype=torch.uint8, device=v.device)
        _check(self._lib.sk_flags(self.handle, _ptr(v), _ptr(n_eff), _ptr(out), v.numel(), _stream_handle(stream)))
        return out

    def reset(self):
        _check(self._lib.sk_state_reset(self.handle))

    def export_state(self, stream: Optional[torch.cuda.Stream] = None) -> bytes:
        n = ctypes.c_size_t()
        _check(self._lib.sk_state_size(self.handle, ctypes.byref(n)))
        buf = ctypes.create_string_buffer(n.value)
        _check(self._lib.sk_state_export(self.handle, buf, n.value, _stream_handle(stream)))
        return buf.raw

    def import_state(self, blob: bytes, stream: Optional[torch.cuda.Stream] = None):
        buf = ctypes.create_string_buffer(blob, len(blob))
        _check(self._lib.sk_state_import(self.handle, buf, len(blob), _stream_handle(stream)))


def compute_noalloc(packed: torch.Tensor, out: "Result", block_len: int, norm_window: int = 1,
                    estimator: int = EST_HAT, k_sigma: float = 5.0, expect_offset: float = 0.0,
                    sigma_override: float = 0.0, mask: Optional[torch.Tensor] = None,
                    stream: Optional[torch.cuda.Stream] = None) -> "Result":
    """One call of the whole path with a fresh normaliser and no plan, through
    the entry point that allocates nothing (sk_compute_noalloc): ``packed`` is
    [T][F][N] uint8 on the current device, ``out`` holds at least s1 and s2."""
    if not isinstance(packed, torch.Tensor) or packed.dim() != 3:
        raise ValueError("packed must be a [T][F][N] tensor")
    T, F, N = packed.shape
    dev = torch.cuda.current_device()
    _device_tensor(packed, "packed", torch.uint8, (T, F, N), dev)
    if out.s1 is None or out.s2 is None:
        raise ValueError("compute_noalloc needs the s1 and s2 outputs")
    if block_len < 1 or T % block_len:
        raise ValueError(f"T = {T} is not a multiple of block_len = {block_len}")
    if mask is not None:
        _device_tensor(mask, "mask", torch.uint8, (F, N), dev)
    _check_outputs(out, F, T // block_len, N, dev)
    d = PlanDesc(N, F, T, block_len, norm_window, estimator, k_sigma, expect_offset, sigma_override)
    o = Outputs(*[_ptr(getattr(out, k)) for k in ALL_OUTPUTS])
    _check(load_library().sk_compute_noalloc(ctypes.byref(d), _ptr(packed), _ptr(mask), ctypes.byref(o),
                                              _stream_handle(stream)))
    return out


def noalloc_scratch_bytes() -> int:
    return int(load_library().sk_noalloc_scratch_bytes())


class Batch:
    """Many independent problems in one graph launch per call (``sk_batch_t``).

    ``plans`` is a list of dicts with the Plan keyword arguments; ``inputs`` the
    device tensors [T][F][N]; the outputs named in ``want`` are allocated here
    (the others are not computed)."""

    def __init__(self, plans, inputs, autotune: bool = True, use_graph: bool = True,
                 tune_cache: Optional[str] = None, want: Sequence[str] = DEFAULT_OUTPUTS):
        self._lib = load_library()
        n = len(plans)
        if n < 1 or len(inputs) != n:
            raise ValueError("one input tensor per problem, at least one problem")
        self.device_index = torch.cuda.current_device()
        self.descs = (PlanDesc * n)()
        self.outputs = []
        outs = (Outputs * n)()
        for j, (kw, x) in enumerate(zip(plans, inputs)):
            d = PlanDesc(kw["n_inputs"], kw["n_channels"], kw["n_samples"], kw["block_len"],
                         kw.get("norm_window", 1), kw.get("estimator", EST_HAT), kw.get("k_sigma", 5.0),
                         kw.get("expect_offset", 0.0), kw.get("sigma_override", 0.0))
            self.descs[j] = d
            T, F, N, M = d.n_samples, d.n_channels, d.n_inputs, d.block_len
            _device_tensor(x, f"input {j}", torch.uint8, (T, F, N), self.device_index)
            B = T // M
            specs = _output_specs(F, B, N)
            r = Result(*[torch.empty(specs[k][0], dtype=specs[k][1], device=x.device) if k in want else None
                         for k in ALL_OUTPUTS])
            self.outputs.append(r)
            outs[j] = Outputs(*[_ptr(getattr(r, k)) for k in ALL_OUTPUTS])
        self._inputs = list(inputs)
        ptrs = (ctypes.c_void_p * n)(*[x.data_ptr() for x in inputs])
        opts = BatchOpts(int(autotune), int(use_graph), tune_cache.encode() if tune_cache else None)
        h = ctypes.c_void_p()
        _check(self._lib.sk_batch_create(self.descs, n, ctypes.byref(opts), ptrs, outs, ctypes.byref(h)))
        self.handle = h
        self.n = n

    def compute(self, inputs=None, stream: Optional[torch.cuda.Stream] = None):
        ptrs = None
        if inputs is not None:
            if len(inputs) != self.n:
                raise ValueError(f"expected {self.n} inputs, got {len(inputs)}")
            for j, x in enumerate(inputs):
                d = self.descs[j]
                _device_tensor(x, f"input {j}", torch.uint8, (d.n_samples, d.n_channels, d.n_inputs),
                               self.device_index)
            self._inputs = list(inputs)
            ptrs = (ctypes.c_void_p * self.n)(*[x.data_ptr() for x in inputs])
        _check(self._lib.sk_batch_compute(self.handle, ptrs, _stream_handle(stream)))
        return self.outputs

    def reset(self, stream: Optional[torch.cuda.Stream] = None):
        _check(self._lib.sk_batch_state_reset(self.handle, _stream_handle(stream)))

    def hist_len(self, j: int) -> int:
        h = ctypes.c_int32()
        _check(self._lib.sk_batch_get_state(self.handle, j, ctypes.byref(h)))
        return h.value

    def tiles(self, j: int):
        lpr, grid = ctypes.c_int32(), ctypes.c_int32()
        _check(self._lib.sk_batch_get_tiles(self.handle, j, ctypes.byref(lpr), ctypes.byref(grid)))
        return lpr.value, grid.value

    def tuning(self, j: int) -> dict:
        """Problem j's tile choices: pass A rows per load and blocks per task,
        pass B chunk length, and whether they came from the tuning cache."""
        v = [ctypes.c_int32() for _ in range(4)]
        _check(self._lib.sk_batch_get_tuning(self.handle, j, *[ctypes.byref(x) for x in v]))
        return dict(rows=v[0].value, blocks=v[1].value, chunk=v[2].value, from_cache=bool(v[3].value))

    def time_pass_a(self, stream=None) -> float:
        """Best of three runs of batched pass A alone, in milliseconds (profiling)."""
        import torch
        s = stream if stream is not None else torch.cuda.current_stream()
        ms = ctypes.c_float()
        _check(self._lib.sk_batch_time_pass_a(self.handle, ctypes.c_void_p(s.cuda_stream), ctypes.byref(ms)))
        return float(ms.value)

    def close(self):
        if getattr(self, "handle", None):
            _check(self._lib.sk_batch_destroy(self.handle))
            self.handle = None

    def __del__(self, _finalizing=sys.is_finalizing):
        if _finalizing():
            return
        try:
            self.close()
        except Exception:
            pass


class Server:
    """Continuous-batching server (``sk_server_t``): arrays submit frames as they arrive."""

    def __init__(self, hbm_budget_bytes: int, max_inflight: int = 8, n_streams: int = 4, queue_capacity: int = 1024):
        self._lib = load_library()
        self.device_index = torch.cuda.current_device()
        d = ServerDesc(int(hbm_budget_bytes), int(max_inflight), int(n_streams), int(queue_capacity))
        h = ctypes.c_void_p()
        _check(self._lib.sk_server_create(ctypes.byref(d), ctypes.byref(h)))
        self.handle = h
        self.arrays = []
        self._keep = {}

    def add_array(self, **kw) -> int:
        d = PlanDesc(kw["n_inputs"], kw["n_channels"], kw["n_samples"], kw["block_len"], kw.get("norm_window", 1),
                     kw.get("estimator", EST_HAT), kw.get("k_sigma", 5.0), kw.get("expect_offset", 0.0),
                     kw.get("sigma_override", 0.0))
        aid = ctypes.c_int32()
        _check(self._lib.sk_server_add_array(self.handle, ctypes.byref(d), ctypes.byref(aid)))
        self.arrays.append(d)
        return aid.value

    def alloc_outputs(self, array_id: int, device, want: Sequence[str] = DEFAULT_OUTPUTS) -> Result:
        d = self.arrays[array_id]
        F, N, B = d.n_channels, d.n_inputs, d.n_samples // d.block_len
        shapes = {"s1": ((F, B, N), torch.int32), "s2": ((F, B, N), torch.int32), "r1": ((F, B), torch.int64),
                  "r2": ((F, B), torch.int64), "v": ((F, B), torch.float32), "flags": ((F, B), torch.uint8),
                  "n_eff": ((F, B), torch.int32), "sk_i": ((F, B, N), torch.float32),
                  "significance": ((F, B), torch.float32)}
        return Result(**{k: (torch.empty(shapes[k][0], dtype=shapes[k][1], device=device) if k in want else None)
                         for k in ALL_OUTPUTS})

    def submit(self, array_id: int, frame: torch.Tensor, out: Result, tag: int = 0,
               stream: Optional[torch.cuda.Stream] = None) -> Optional[int]:
        """Returns the ticket, or None when the queue is full. The frame's work
        waits for what is already enqueued on ``stream`` (default: the current
        stream), so frames and output buffers written there need no sync."""
        if not 0 <= array_id < len(self.arrays):
            raise ValueError(f"unknown array {array_id}")
        d = self.arrays[array_id]
        T, F, N = d.n_samples, d.n_channels, d.n_inputs
        if frame.is_cuda:
            _device_tensor(frame, "frame", torch.uint8, (T, F, N), self.device_index)
        else:
            if frame.dtype != torch.uint8 or tuple(frame.shape) != (T, F, N) or not frame.is_contiguous():
                raise ValueError(f"host frame must be a contiguous uint8 tensor of shape {(T, F, N)}")
            if not frame.is_pinned():
                raise ValueError("host frames must be in pinned memory (asynchronous copy)")
        _check_outputs(out, F, d.n_samples // d.block_len, N, self.device_index)
        o = Outputs(*[_ptr(getattr(out, k)) for k in ALL_OUTPUTS])
        t = ctypes.c_uint64()
        rc = self._lib.sk_stream_submit(self.handle, array_id, ctypes.c_void_p(frame.data_ptr()),
                                        0 if frame.is_cuda else 1, ctypes.byref(o), tag,
                                        _stream_handle(stream), ctypes.byref(t))
        if rc == SK_ERR_AGAIN:
            return None
        _check(rc)
        self._keep[t.value] = (frame, out)
        return t.value

    def poll(self, ticket: int) -> Optional[ServerResult]:
        r = ServerResult()
        rc = self._lib.sk_stream_poll(self.handle, ticket, ctypes.byref(r))
        if rc == SK_ERR_AGAIN:
            return None
        _check(rc)
        self._keep.pop(ticket, None)
        return r

    def drain(self):
        _check(self._lib.sk_server_drain(self.handle))

    def stats(self) -> ServerStats:
        st = ServerStats()
        _check(self._lib.sk_server_get_stats(self.handle, ctypes.byref(st)))
        return st

    def now(self) -> float:
        return self._lib.sk_server_now()

    def close(self):
        if getattr(self, "handle", None):
            _check(self._lib.sk_server_destroy(self.handle))
            self.handle = None
            self._keep.clear()

    def __del__(self, _finalizing=sys.is_finalizing):
        if _finalizing():
            return
        try:
            self.close()
        except Exception:
            pass


def build(verbose: bool = False) -> str:
    from . import _build
    return _build.build_library(verbose=verbose)
