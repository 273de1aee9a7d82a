"""Python entry points over libsten (argument marshalling only).

Every step of the computation runs in libsten's HIP kernels; torch provides
device memory and the current stream. Grids are 2-D tensors on the current
HIP device, row-major with unit column stride (row stride = tensor.stride(0)).
"""

from __future__ import annotations

import torch

from . import _lib


def _stream_ptr(stream=None) -> int:
    s = stream if stream is not None else torch.cuda.current_stream()
    return int(s.cuda_stream)


def _check_grid(t: torch.Tensor, dtype, name: str) -> None:
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name} must be a torch.Tensor")
    if t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}, got {t.dtype}")
    if t.dim() != 2:
        raise ValueError(f"{name} must be 2-D")
    if not t.is_cuda:
        raise ValueError(f"{name} must be on the GPU (libsten has no CPU path)")
    if t.numel() > 0 and t.stride(1) != 1:
        raise ValueError(f"{name} must have unit column stride")


def _ld(t: torch.Tensor) -> int:
    return int(t.stride(0)) if t.shape[0] > 1 else int(max(t.shape[1], 1))


def jacobi5(u0: torch.Tensor, T: int, c: float = 0.25, out: torch.Tensor | None = None,
            work: torch.Tensor | None = None, stream=None) -> torch.Tensor:
    """T five-point Jacobi sweeps of u0 (FP64 or FP32) on the GPU; returns the result grid.

    The method of the listing of the Laplace solver (Section III-A): the ring
    is kept, each interior point becomes c*(((N+S)+W)+E), buffers swap each
    sweep. `out` and `work` (same shape/stride as u0) are allocated when not given.
    """
    if u0.dtype == torch.float64:
        fn = "sten_jacobi5_f64"
    elif u0.dtype == torch.float32:
        fn = "sten_jacobi5_f32"
    else:
        raise TypeError("u0 must be float32 or float64")
    _check_grid(u0, u0.dtype, "u0")
    H, W = u0.shape
    if out is None:
        out = torch.empty_strided(u0.shape, u0.stride(), dtype=u0.dtype, device=u0.device)
    _check_grid(out, u0.dtype, "out")
    if out.shape != u0.shape or (H > 1 and out.stride() != u0.stride()):
        raise ValueError("out must match u0's shape and strides")
    need_work = T >= 2 and H >= 3 and W >= 3
    if work is None and need_work:
        work = torch.empty_strided(u0.shape, u0.stride(), dtype=u0.dtype, device=u0.device)
    if work is not None:
        _check_grid(work, u0.dtype, "work")
        if work.shape != u0.shape or (H > 1 and work.stride() != u0.stride()):
            raise ValueError("work must match u0's shape and strides")
    _lib.call(fn, u0.data_ptr(), out.data_ptr(), work.data_ptr() if work is not None else None,
              H, W, _ld(u0), int(T), float(c), _stream_ptr(stream))
    return out


def sweep(src: torch.Tensor, dst: torch.Tensor, c: float = 0.25, stream=None) -> torch.Tensor:
    """One sweep: dst's interior from src (dst's ring untouched); returns dst."""
    fn = {torch.float64: "sten_sweep_f64", torch.float32: "sten_sweep_f32"}.get(src.dtype)
    if fn is None:
        raise TypeError("src must be float32 or float64")
    _check_grid(src, src.dtype, "src")
    _check_grid(dst, src.dtype, "dst")
    if dst.shape != src.shape or (src.shape[0] > 1 and dst.stride() != src.stride()):
        raise ValueError("dst must match src's shape and strides")
    H, W = src.shape
    _lib.call(fn, src.data_ptr(), dst.data_ptr(), H, W, _ld(src), float(c), _stream_ptr(stream))
    return dst


def set_sweep_rows(rows: int) -> None:
    """Tuning hook: rows per tile of the sweep kernels (4, 8, 16; 0 = built-in)."""
    _lib.call("sten_tune_sweep_rows", int(rows))
