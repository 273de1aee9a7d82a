"""The allocation-free adjoint segment call against the call it replaces, through the C ABI.

sten_jacobi5_adjoint_f32_seg_noalloc keeps the FP64 partial sums of dL/dc in
a per-device static buffer and reduces them into a device double; it must
give the bits of sten_jacobi5_adjoint_f32_seg (caller-provided partials)
followed by sten_reduce_f64, on consecutive calls of different sizes.
"""

import numpy as np
import pytest

from tests.gpu_util import device, say, to_dev, to_host
from workloads import normal_grid

pytestmark = pytest.mark.gpu


def _stream():
    import torch

    return torch.cuda.current_stream().cuda_stream


def _states(lib, u0, T, c):
    import torch

    H, W = u0.shape
    st = torch.empty((T + 1, H, W), dtype=torch.float32, device=u0.device)
    assert lib.sten_jacobi5_f32_states(u0.data_ptr(), st.data_ptr(), H, W, W, T, c, _stream()) == 0
    return st


def _reference(lib, lam, states, nsteps, reset, partials, H, W, c):
    """The existing pair: the segment call with caller-owned partials, then the fixed-order reduction."""
    import torch

    out = torch.empty_like(lam)
    work = torch.empty_like(lam)
    sp = states.data_ptr() if states is not None else None
    assert lib.sten_jacobi5_adjoint_f32_seg(lam.data_ptr(), sp, nsteps, out.data_ptr(), work.data_ptr(),
                                            partials.data_ptr(), reset, H, W, W, c, _stream()) == 0
    dc = torch.empty(1, dtype=torch.float64, device=lam.device)
    assert lib.sten_reduce_f64(partials.data_ptr(), partials.numel(), dc.data_ptr(), _stream()) == 0
    return to_host(out), to_host(dc)[0]


def _noalloc(lib, lam, states, nsteps, reset, H, W, c):
    import torch

    out = torch.empty_like(lam)
    work = torch.empty_like(lam)
    dc = torch.full((1,), float("nan"), dtype=torch.float64, device=lam.device)
    sp = states.data_ptr() if states is not None else None
    assert lib.sten_jacobi5_adjoint_f32_seg_noalloc(lam.data_ptr(), sp, nsteps, out.data_ptr(), work.data_ptr(),
                                                    reset, dc.data_ptr(), H, W, W, c, _stream()) == 0
    return to_host(out), to_host(dc)[0]


@pytest.fixture(scope="module")
def lib():
    device()
    from paper_2512_19851_amd import _lib

    return _lib.load()


def test_noalloc_matches_seg_and_reduce_twice(lib):
    """Two calls in a row, the second on a smaller grid: lambda and dL/dc bit-identical."""
    import torch

    c = 0.25
    for (H, W, T, seed) in [(257, 1031, 6, 1), (40, 70, 3, 2)]:
        say(f"noalloc adjoint {H}x{W} T={T}")
        u0 = to_dev(normal_grid(H, W, seed=seed, dtype=np.float32))
        lam = to_dev(normal_grid(H, W, seed=seed + 100, dtype=np.float32))
        st = _states(lib, u0, T, c)
        parts = torch.empty(int(lib.sten_adjoint_partials_len(H, W)), dtype=torch.float64, device=u0.device)
        want_lam, want_dc = _reference(lib, lam, st, T, 1, parts, H, W, c)
        got_lam, got_dc = _noalloc(lib, lam, st, T, 1, H, W, c)
        assert np.array_equal(got_lam, want_lam)
        assert got_dc == want_dc and np.isfinite(got_dc)


def test_noalloc_segments_accumulate(lib):
    """A checkpointed reverse pass: the second segment (reset = 0) adds to the first's sums."""
    import torch

    H, W, c = 130, 300, 0.25
    u0 = to_dev(normal_grid(H, W, seed=7, dtype=np.float32))
    w = to_dev(normal_grid(H, W, seed=8, dtype=np.float32))
    st = _states(lib, u0, 7, c)
    parts = torch.empty(int(lib.sten_adjoint_partials_len(H, W)), dtype=torch.float64, device=u0.device)
    say("noalloc adjoint segments")
    # segment 1: states 3..6 (lambda_7 -> lambda_3); segment 2: states 0..2 (lambda_3 -> lambda_0)
    ref1, dc1 = _reference(lib, w, st[3:], 4, 1, parts, H, W, c)
    ref2, dc2 = _reference(lib, to_dev(ref1), st[:3], 3, 0, parts, H, W, c)
    got1, g1 = _noalloc(lib, w, st[3:], 4, 1, H, W, c)
    got2, g2 = _noalloc(lib, to_dev(got1), st[:3], 3, 0, H, W, c)
    assert np.array_equal(got1, ref1) and np.array_equal(got2, ref2)
    assert g1 == dc1 and g2 == dc2 and g1 != g2


def test_noalloc_rejects_oversize_and_bad_args(lib):
    # more workgroups than the static buffer holds: rejected before any pointer is used
    assert lib.sten_jacobi5_adjoint_f32_seg_noalloc(None, None, 1, None, None, 1, None, 8 * (2**20 + 1), 256, 256,
                                                    0.25, None) == -4
    assert lib.sten_jacobi5_adjoint_f32_seg_noalloc(None, None, 1, None, None, 1, None, -1, 8, 8, 0.25, None) == -1
    assert lib.sten_jacobi5_adjoint_f32_seg_noalloc(None, None, 1, None, None, 1, None, 8, 8, 8, 0.25, None) == -3
    assert lib.sten_jacobi5_adjoint_f32_seg_noalloc(None, None, 1, None, None, 1, None, 0, 8, 8, 0.25, None) == 0
