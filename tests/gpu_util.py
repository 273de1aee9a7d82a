"""Helpers shared by the GPU parity tests (no method arithmetic here)."""

from __future__ import annotations

import sys

import numpy as np


def device():
    import torch

    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    return torch.device("cuda:0")


def to_dev(a: np.ndarray):
    import torch

    return torch.from_numpy(np.ascontiguousarray(a)).to(device())


def to_host(t) -> np.ndarray:
    import torch

    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


def say(msg: str) -> None:
    """Name the case before each GPU step, flushed, so a crash log shows it."""
    print(msg, flush=True)
    sys.stdout.flush()


def cone_window(H: int, W: int, i: int, j: int, T: int):
    """Rows/cols of the sub-grid whose T-sweep result at (i, j) equals the full grid's.

    A point's value after T sweeps depends only on points within Manhattan
    distance T; the sub-grid's own (fixed) ring sits at distance T + 1, so its
    influence cannot reach (i, j) within T sweeps. Where the window meets the
    real boundary, the real ring is part of it.
    """
    r0, r1 = max(0, i - T - 1), min(H - 1, i + T + 1)
    c0, c1 = max(0, j - T - 1), min(W - 1, j + T + 1)
    return r0, r1, c0, c1


def stream_edges(H: int, W: int, V: int = 2, TL: int = 11, bands=(54, 22)):
    """Store boundaries of the streaming blocked kernel: the first stored column of each strip (and the
    column before it) in the right-aligned layout used when W is a multiple of V and at least 64*V
    (strip k >= 1 stores from k*OW + HALO, the last strip from W - 64*V + HALO), and the first row of
    each band (and the row before it) for the given band heights. Grid geometry only."""
    halo = -(-TL // V) * V
    ow = 64 * V - 2 * halo
    cols = set()
    if W % V == 0 and W >= 64 * V:
        strips = -(-(W - 64 * V) // ow) + 1
        starts = [k * ow + halo for k in range(1, strips - 1)] + [W - 64 * V + halo]
    else:
        starts = [k * ow for k in range(1, -(-(W - 1) // ow))]
    for c0 in starts:
        cols.update((c0 - 1, c0))
    rows = set()
    for band in bands:
        for rb in range(1 + band, H - 1, band):
            rows.update((rb - 1, rb))
    return sorted(rows), sorted(cols)


def sample_points(H: int, W: int, n: int, seed: int = 0, stream=None):
    """Corners, ring points, tile-edge points and random interior points. With stream = (V, TL), also
    points where band-edge rows meet strip-edge columns of the streaming kernel of that geometry."""
    rng = np.random.default_rng(seed)
    pts = {(0, 0), (H - 1, W - 1), (1, 1), (H - 2, W - 2), (1, W - 2), (H - 2, 1), (0, W // 2)}
    for r in (7, 8, 9, 15, 16, 17):
        for cc in (255, 256, 511, 512, 513):
            if 0 < r < H - 1 and 0 < cc < W - 1:
                pts.add((r, cc))
    if stream is not None:
        rows, cols = stream_edges(H, W, *stream)
        picks = rng.permutation(len(rows) * len(cols))[: max(8, n // 2)]
        for k in picks:
            r, cc = rows[k // len(cols)], cols[k % len(cols)]
            if 0 < r < H - 1 and 0 < cc < W - 1:
                pts.add((int(r), int(cc)))
    while len(pts) < n:
        pts.add((int(rng.integers(0, H)), int(rng.integers(0, W))))
    return sorted(pts)
