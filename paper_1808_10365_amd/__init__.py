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
                ("n_eff", ctypes.c_void_p)]


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
    lib.sk_state_reset.argtypes = [VP]
    lib.sk_state_size.argtypes = [VP, ctypes.POINTER(SZ)]
    lib.sk_state_export.argtypes = [VP, VP, SZ, VP]
    lib.sk_state_import.argtypes = [VP, VP, SZ, VP]
    lib.sk_digitised_expectation.argtypes = [VP, I32, I32, I32, ctypes.POINTER(F64), ctypes.POINTER(F64)]
    lib.sk_plan_set_pass_a_tile.argtypes = [VP, I32]
    lib.sk_plan_get_pass_a_tile.argtypes = [VP, VP, ctypes.POINTER(I32), ctypes.POINTER(I32), ctypes.POINTER(I64)]
    lib.sk_plan_set_pass_a_variant.argtypes = [VP, I32, I32]
    lib.sk_profile_enable.argtypes = [VP, I32]
    lib.sk_profile_read.argtypes = [VP, VP, VP, I32, ctypes.POINTER(I32)]
    for name in ("sk_plan_create", "sk_plan_destroy", "sk_plan_device_bytes", "sk_compute", "sk_flags",
                 "sk_state_reset", "sk_state_size", "sk_state_export", "sk_state_import",
                 "sk_digitised_expectation", "sk_plan_set_pass_a_tile", "sk_plan_get_pass_a_tile",
                 "sk_profile_enable", "sk_profile_read", "sk_plan_set_pass_a_variant"):
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


def digitised_expectation(sigma: Sequence[float], block_len: int, clip: int = 7):
    """App. B model: (delta, sigma_V) for inputs of per-component RMS ``sigma``."""
    import numpy as np
    s = np.ascontiguousarray(sigma, dtype=np.float64)
    d, sv = ctypes.c_double(), ctypes.c_double()
    _check(load_library().sk_digitised_expectation(s.ctypes.data, len(s), int(block_len), int(clip),
                                                   ctypes.byref(d), ctypes.byref(sv)))
    return d.value, sv.value


@dataclass
class Result:
    s1: Optional[torch.Tensor]
    s2: Optional[torch.Tensor]
    r1: Optional[torch.Tensor]
    r2: Optional[torch.Tensor]
    v: Optional[torch.Tensor]
    flags: Optional[torch.Tensor]
    n_eff: Optional[torch.Tensor]


ALL_OUTPUTS = ("s1", "s2", "r1", "r2", "v", "flags", "n_eff")


class Plan:
    """One stream of [T][F][N] frames with its own normaliser state (a ``sk_plan_t``)."""

    def __init__(self, n_inputs: int, n_channels: int, n_samples: int, block_len: int,
                 norm_window: int = 1, estimator: int = EST_HAT, k_sigma: float = 5.0,
                 expect_offset: float = 0.0, sigma_override: float = 0.0):
        self._lib = load_library()
        self.desc = PlanDesc(n_inputs, n_channels, n_samples, block_len, norm_window, estimator,
                             k_sigma, expect_offset, sigma_override)
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

    def __del__(self):
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

    def set_pass_a_variant(self, variant: int, grid: int = 0):
        """Row batching variant of pass A (0..3) and workgroup count (0: one per task)."""
        _check(self._lib.sk_plan_set_pass_a_variant(self.handle, int(variant), int(grid)))

    def alloc_outputs(self, device, want: Sequence[str] = ALL_OUTPUTS) -> Result:
        F, N, B = self.desc.n_channels, self.desc.n_inputs, self.n_blocks
        mk = {
            "s1": lambda: torch.empty((F, B, N), dtype=torch.int32, device=device),
            "s2": lambda: torch.empty((F, B, N), dtype=torch.int32, device=device),
            "r1": lambda: torch.empty((F, B), dtype=torch.int64, device=device),
            "r2": lambda: torch.empty((F, B), dtype=torch.int64, device=device),
            "v": lambda: torch.empty((F, B), dtype=torch.float32, device=device),
            "flags": lambda: torch.empty((F, B), dtype=torch.uint8, device=device),
            "n_eff": lambda: torch.empty((F, B), dtype=torch.int32, device=device),
        }
        return Result(**{k: (mk[k]() if k in want else None) for k in ALL_OUTPUTS})

    def compute_into(self, packed: torch.Tensor, out: Result, mask: Optional[torch.Tensor] = None,
                     stream: Optional[torch.cuda.Stream] = None) -> Result:
        T, F, N = self.desc.n_samples, self.desc.n_channels, self.desc.n_inputs
        if packed.dtype != torch.uint8 or tuple(packed.shape) != (T, F, N) or not packed.is_contiguous() or not packed.is_cuda:
            raise ValueError(f"packed must be a contiguous CUDA uint8 tensor of shape {(T, F, N)}")
        if mask is not None and (mask.dtype != torch.uint8 or tuple(mask.shape) != (F, N) or not mask.is_contiguous()):
            raise ValueError(f"mask must be a contiguous uint8 tensor of shape {(F, N)}")
        o = Outputs(*[_ptr(getattr(out, k)) for k in ALL_OUTPUTS])
        _check(self._lib.sk_compute(self.handle, _ptr(packed), _ptr(mask), ctypes.byref(o), _stream_handle(stream)))
        return out

    def compute(self, packed: torch.Tensor, mask: Optional[torch.Tensor] = None,
                want: Sequence[str] = ALL_OUTPUTS, stream: Optional[torch.cuda.Stream] = None) -> Result:
        out = self.alloc_outputs(packed.device, want)
        return self.compute_into(packed, out, mask, stream)

    def flags(self, v: torch.Tensor, n_eff: torch.Tensor, stream: Optional[torch.cuda.Stream] = None) -> torch.Tensor:
        assert v.dtype == torch.float32 and n_eff.dtype == torch.int32 and v.shape == n_eff.shape
        v = v.contiguous()
        n_eff = n_eff.contiguous()
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


def build(verbose: bool = False) -> str:
    from . import _build
    return _build.build_library(verbose=verbose)
