"""Seeded synthetic inputs for the five-point Jacobi sweep workloads.

This module only draws random numbers and builds shapes. It holds none of the
method's arithmetic, so the CPU oracle (``oracle/``), the tests and the
benchmark can all share it without sharing any part of the computation.

Every generator uses ``numpy.random.default_rng(seed)`` (PCG64) and draws in a
fixed order, so a given (recipe, seed) always yields the same arrays. FP32
inputs are drawn in FP64 and then cast; the FP64 oracle consumes the cast
values, so FP32 and FP64 runs start from the same numbers.

Workload recipes (sizes follow the paper's Laplace benchmark, Section V, and
the listing of the Laplace solver in Section III-A):

* ``small_f64``    one 64x64 FP64 grid, N(0,1)
* ``large_f64``    one 4096x4096 FP64 grid, N(0,1)
* ``mixed_f64``    one 4096x4096 FP64 grid, N(0,1) times 10**U(-3,3) per element
* ``batch_f32``    1024 FP32 grids, point counts log-uniform in [2^8, 2^16]
* ``adjoint_f32``  one 1024x1024 FP32 grid, N(0,1), a weight grid w ~ N(0,1)
                   and 64 distinct flat coordinates for finite differences
* ``paper_grid``   the listing's initial state: unit boundary ring, zero
                   interior (16384x16384 per GPU in the paper's runs)
* ``hashed_grid``  values from an integer hash of (seed, row, column), uniform
                   in [-1, 1): a grid too large to draw on the host (past 2^31
                   points) is filled on the device row block by row block with
                   ``hashed_rows_torch``, and any window of it is rebuilt on the
                   host with ``hashed_grid``, bit for bit
"""

from __future__ import annotations

import numpy as np

__all__ = [
    "normal_grid",
    "small_f64",
    "large_f64",
    "mixed_f64",
    "batch_shapes",
    "batch_f32",
    "adjoint_f32",
    "unit_ring_grid",
    "hashed_grid",
    "hashed_rows_torch",
    "BATCH_COUNT",
]

BATCH_COUNT = 1024


def normal_grid(H: int, W: int, seed: int = 0, dtype=np.float64) -> np.ndarray:
    """An HxW grid of i.i.d. N(0,1) values drawn in FP64, then cast to dtype."""
    rng = np.random.default_rng(seed)
    return rng.standard_normal((H, W)).astype(dtype, copy=False)


def small_f64(seed: int = 0) -> np.ndarray:
    """64x64 FP64 grid, N(0,1): the smallest instance of the Laplace problem."""
    return normal_grid(64, 64, seed)


def large_f64(seed: int = 0, n: int = 4096) -> np.ndarray:
    """n x n FP64 grid, N(0,1) (4096x4096 = 2^24 points by default)."""
    return normal_grid(n, n, seed)


def mixed_f64(seed: int = 0, n: int = 4096) -> np.ndarray:
    """n x n FP64 grid z*s with z ~ N(0,1) and s = 10**U(-3,3) drawn per element.

    The per-element log-uniform factor spreads magnitudes over six decades, which
    stresses any reduced-precision representation of the grid.
    """
    rng = np.random.default_rng(seed)
    z = rng.standard_normal((n, n))
    s = 10.0 ** rng.uniform(-3.0, 3.0, (n, n))
    return z * s


def batch_shapes(seed: int = 0, count: int = BATCH_COUNT) -> list[tuple[int, int]]:
    """Shapes of `count` near-square grids with point counts log-uniform in [2^8, 2^16].

    n = rint(2**U(8,16)); H = max(3, rint(sqrt(n))); W = max(3, rint(n / H)).
    """
    rng = np.random.default_rng(seed)
    lg = rng.uniform(8.0, 16.0, count)
    shapes = []
    for v in lg:
        n = int(np.rint(2.0 ** v))
        H = max(3, int(np.rint(np.sqrt(n))))
        W = max(3, int(np.rint(n / H)))
        shapes.append((H, W))
    return shapes


def batch_f32(seed: int = 0, count: int = BATCH_COUNT) -> list[np.ndarray]:
    """`count` FP32 grids of the shapes from `batch_shapes`, each N(0,1).

    The shapes are drawn first; the grids follow from the same generator, in order.
    """
    rng = np.random.default_rng(seed)
    lg = rng.uniform(8.0, 16.0, count)
    shapes = []
    for v in lg:
        n = int(np.rint(2.0 ** v))
        H = max(3, int(np.rint(np.sqrt(n))))
        W = max(3, int(np.rint(n / H)))
        shapes.append((H, W))
    return [rng.standard_normal(s).astype(np.float32) for s in shapes]


def adjoint_f32(seed: int = 0, n: int = 1024, n_coords: int = 64):
    """(u0, w, coords): u0 FP32 n x n N(0,1); w FP64 n x n N(0,1); distinct flat coords."""
    rng = np.random.default_rng(seed)
    u0 = rng.standard_normal((n, n)).astype(np.float32)
    w = rng.standard_normal((n, n))
    coords = rng.choice(n * n, n_coords, replace=False)
    return u0, w, coords


def unit_ring_grid(H: int, W: int, dtype=np.float64) -> np.ndarray:
    """The listing's initial state: boundary ring set to 1, interior 0."""
    u = np.zeros((H, W), dtype=dtype)
    u[0, :] = 1
    u[-1, :] = 1
    u[:, 0] = 1
    u[:, -1] = 1
    return u


# Integer hash of (seed, i, j) into [0, 2^32): two odd multipliers and xor-shifts,
# all in 64-bit integers without overflow (i, j < 2^31, products < 2^63).
_HM1, _HM2, _HM3, _HS = 0x9E3779B1, 0x85EBCA77, 0x2C1B3C6D, 0x27D4EB2F
_M32 = 0xFFFFFFFF


def _hash_to_unit(h):
    # h in [0, 2^32) -> h / 2^31 - 1, exact in FP64
    return h * (1.0 / 2147483648.0) - 1.0


def hashed_grid(r0: int, r1: int, c0: int, c1: int, seed: int = 0) -> np.ndarray:
    """Rows [r0, r1) and columns [c0, c1) of the hashed grid, FP64 in [-1, 1)."""
    i = np.arange(r0, r1, dtype=np.int64)[:, None]
    j = np.arange(c0, c1, dtype=np.int64)[None, :]
    h = ((i * _HM1) ^ (j * _HM2) ^ (seed * _HS)) & _M32
    h = h ^ (h >> 15)
    h = (h * _HM3) & _M32
    h = h ^ (h >> 12)
    return _hash_to_unit(h.astype(np.float64))


def hashed_rows_torch(r0: int, r1: int, W: int, device, seed: int = 0):
    """Rows [r0, r1) (all W columns) of the hashed grid as an FP64 torch tensor on `device`."""
    import torch

    i = torch.arange(r0, r1, dtype=torch.int64, device=device)[:, None]
    j = torch.arange(0, W, dtype=torch.int64, device=device)[None, :]
    h = ((i * _HM1) ^ (j * _HM2) ^ (seed * _HS)) & _M32
    h = h ^ (h >> 15)
    h = (h * _HM3) & _M32
    h = h ^ (h >> 12)
    return _hash_to_unit(h.to(torch.float64))
