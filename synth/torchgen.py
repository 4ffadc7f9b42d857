"""torch implementation of selected ``synth`` generators, bit-identical to the numpy ones.

Used for large inputs (the many-matrix batch), where torch's multi-threaded host kernels
generate the arrays much faster.  Same SplitMix64 streams: int64 tensors hold the uint64
state (wrapping multiplication and addition give the same bits), and right shifts are made
logical by masking.
"""
from __future__ import annotations

import torch

import synth

_GOLDEN = 0x9E3779B97F4A7C15 - (1 << 64)
_M1 = 0xBF58476D1CE4E5B9 - (1 << 64)
_M2 = 0x94D049BB133111EB - (1 << 64)


def _srl(z: torch.Tensor, s: int) -> torch.Tensor:
    return (z >> s) & ((1 << (64 - s)) - 1)


def _mix(z: torch.Tensor) -> torch.Tensor:
    z = (z ^ _srl(z, 30)) * _M1
    z = (z ^ _srl(z, 27)) * _M2
    return z ^ _srl(z, 31)


def _signed(u: int) -> int:
    return u - (1 << 64) if u >= (1 << 63) else u


def stream_u64(seed: int, stream: int, n: int, start: int = 0, device="cpu") -> torch.Tensor:
    """Outputs start..start+n-1 of SplitMix64 stream (seed, stream) as int64 bit patterns."""
    key = _signed(int(synth._key(seed, stream)))
    k = torch.arange(start + 1, start + n + 1, dtype=torch.int64, device=device)
    return _mix(key + k * _GOLDEN)


def uniform01(seed: int, stream: int, n: int, device="cpu") -> torch.Tensor:
    return _srl(stream_u64(seed, stream, n, device=device), 11).to(torch.float64) * (1.0 / 9007199254740992.0)


def _uniform_int(seed, stream, n, lo, hi, device):
    z = _srl(stream_u64(seed, stream, n, device=device), 32)
    return lo + ((z * (hi - lo + 1)) >> 32)


def banded_stratified(n: int, seed: int, len_lo: int = 3, len_hi: int = 60, halo: int = 4096,
                      device="cpu"):
    """Same arrays as ``synth.banded_stratified`` (row_ptr, col int32, val f64) as tensors."""
    lens = _uniform_int(seed, 1, n, len_lo, len_hi, device)
    i = torch.arange(n, dtype=torch.int64, device=device)
    lo = torch.clamp(i - halo, min=0)
    width = torch.clamp(i + halo, max=n - 1) - lo + 1
    lens = torch.minimum(lens, width)
    row_ptr = torch.zeros(n + 1, dtype=torch.int64, device=device)
    row_ptr[1:] = torch.cumsum(lens, 0)
    nnz = int(row_ptr[-1])
    row = torch.repeat_interleave(i, lens)
    j = torch.arange(nnz, dtype=torch.int64, device=device) - row_ptr[row]
    L = lens[row]
    w = width[row]
    s0 = torch.div(j * w, L, rounding_mode="floor")
    s1 = torch.div((j + 1) * w, L, rounding_mode="floor")
    z = _srl(stream_u64(seed, 2, nnz, device=device), 32)
    off = (z * (s1 - s0)) >> 32
    col = (lo[row] + s0 + off).to(torch.int32)
    val = 2.0 * uniform01(seed, 3, nnz, device=device) - 1.0
    return row_ptr, col, val


def dense_x(n: int, seed: int = 1, device="cpu") -> torch.Tensor:
    """Same values as ``synth.dense_x(n, seed)``: uniform in [-1, 1)."""
    return 2.0 * uniform01(seed, 7, n, device=device) - 1.0
