"""GPU parity of the hi/lo reduced-precision form, via the C ABI.

Encode and decode are integer/bit work: bit-exact against the oracle's FP64
definitions. The encoded sweep is bit-exact against the oracle's step-by-step
FP32 model, and its decoded result stays within the analytic bound of the
FP64 method (target: componentwise error <= 1e-10 at T = 100).
"""

import numpy as np
import pytest

import oracle
from tests.gpu_util import cone_window, device, sample_points, say, to_dev, to_host
from workloads import mixed_f64, normal_grid

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ops():
    device()
    from paper_2512_19851_amd import ops

    return ops


def _crafted(n=64, seed=0):
    """Mixed-magnitude grid plus values that hit the renormalisation and tie cases."""
    u = mixed_f64(seed=seed, n=n)
    special = [1.0 + 2.0 ** -24, 2.0 - 2.0 ** -24 - 2.0 ** -41, -(1.0 + 2.0 ** -24), 1.0 + 2.0 ** -40,
               1.0 + 3 * 2.0 ** -40, 0.0, -0.0, 1e-40, -3e-42, 2.0 ** -126, 3.0e38, -1.0 / 3.0]
    k = min(len(special), u.size)
    u.flat[:k] = special[:k]
    return u


@pytest.mark.parametrize("shape", [(1, 1), (3, 3), (64, 64), (37, 129), (130, 1030), (36, 1028), (9, 4100)],
                         ids=str)
def test_encode_decode_bit_exact(ops, shape):
    u = _crafted(max(shape), seed=shape[1])[: shape[0], : shape[1]].copy()
    say(f"encode {shape}")
    g = ops.hilo_encode(to_dev(u))
    hi_want, q_want = oracle.hilo_encode(u)
    assert np.array_equal(to_host(g.hi()).view(np.uint32), hi_want.view(np.uint32))
    assert np.array_equal(to_host(g.q()), q_want)
    say(f"decode {shape}")
    assert np.array_equal(to_host(ops.hilo_decode(g)), oracle.hilo_decode(hi_want, q_want))


def test_encode_decode_strided_vector_rows(ops):
    """Row stride a multiple of 4 with widths that are not (the vector kernels' ragged last lanes), and a
    stride that is not (the element-wise kernels), each bit-exact with the oracle's encoding."""
    import torch

    for (H, W, ld) in [(7, 1027, 1028), (5, 2050, 2052), (6, 1021, 1023)]:
        u = _crafted(max(H, W), seed=W)[:H, :W].copy()
        x = torch.zeros((H, ld), dtype=torch.float64, device=device())[:, :W]
        x.copy_(to_dev(u))
        say(f"encode strided {H}x{W} ld={ld}")
        g = ops.hilo_encode(x)
        hi_want, q_want = oracle.hilo_encode(u)
        assert np.array_equal(to_host(g.hi())[:, :W].view(np.uint32), hi_want.view(np.uint32))
        assert np.array_equal(to_host(g.q())[:, :W], q_want)
        out = torch.zeros((H, ld), dtype=torch.float64, device=device())[:, :W]
        assert np.array_equal(to_host(ops.hilo_decode(g, out=out)), oracle.hilo_decode(hi_want, q_want))


SHAPES = [(3, 3), (5, 7), (64, 64), (63, 65), (257, 1031), (600, 3), (3, 600), (130, 2049)]


@pytest.mark.parametrize("shape", SHAPES, ids=lambda s: f"{s[0]}x{s[1]}")
def test_hilo_sweeps_bit_exact_with_model(ops, shape):
    u0 = mixed_f64(seed=sum(shape), n=max(shape))[: shape[0], : shape[1]].copy()
    d = to_dev(u0)
    for T in (0, 1, 2, 3, 10):
        say(f"hilo {shape} T={T}")
        got = to_host(ops.jacobi5_hilo(d, T))
        want = oracle.jacobi5_hilo_model(u0, T)
        assert np.array_equal(got, want), f"{shape} T={T}"
        assert np.all(np.abs(got - oracle.jacobi5(u0, T)) <= oracle.bound_hilo(u0, T))


@pytest.mark.parametrize("c", [0.3, -0.5, 1.0 / 3.0])
def test_hilo_general_coefficient(ops, c):
    u0 = mixed_f64(seed=7, n=200)[:150, :]
    say(f"hilo c={c}")
    got = to_host(ops.jacobi5_hilo(to_dev(u0), 4, c))
    assert np.array_equal(got, oracle.jacobi5_hilo_model(u0, 4, c))
    assert np.all(np.abs(got - oracle.jacobi5(u0, 4, c)) <= oracle.bound_hilo(u0, 4, c))


def test_hilo_encoded_state_between_calls(ops):
    """Sweeps on encoded grids: 3 calls of 2 sweeps equal one call of 6."""
    u0 = mixed_f64(seed=8, n=300)
    say("hilo encoded chain")
    g = ops.hilo_encode(to_dev(u0))
    cur = g
    for _ in range(3):
        cur = ops.jacobi5_hilo_encoded(cur, 2)
    chained = to_host(ops.hilo_decode(cur))
    one = to_host(ops.hilo_decode(ops.jacobi5_hilo_encoded(g, 6)))
    assert np.array_equal(chained, one)
    hi, q = oracle.hilo_encode(u0)
    for _ in range(6):
        hi, q = oracle.hilo_sweep_model(hi, q)
    assert np.array_equal(one, oracle.hilo_decode(hi, q))


@pytest.mark.parametrize("variant", [1, 2, 3, 4, 5, 6, 7, 8, 9, 10])
def test_hilo_kernel_variants(ops, variant):
    """Every kernel variant gives the model's bits, on full and ragged tiles."""
    ops.set_hilo_variant(variant)
    try:
        for shape in [(260, 260), (131, 1029), (70, 2048)]:
            u0 = mixed_f64(seed=variant, n=max(shape))[: shape[0], : shape[1]].copy()
            say(f"hilo variant={variant} {shape}")
            assert np.array_equal(to_host(ops.jacobi5_hilo(to_dev(u0), 3)), oracle.jacobi5_hilo_model(u0, 3))
    finally:
        ops.set_hilo_variant(0)


def test_hilo_odd_stride(ops):
    import torch

    u0 = mixed_f64(seed=10, n=101)[:50, :99].copy()
    t = torch.empty((50, 101), dtype=torch.float64, device=device())[:, :99]
    t.copy_(to_dev(u0))
    say("hilo odd ld")
    assert np.array_equal(to_host(ops.jacobi5_hilo(t, 3)), oracle.jacobi5_hilo_model(u0, 3))


def test_hilo_full_size_T10(ops):
    """4096x4096 mixed-magnitude workload, T = 10: whole grid bit-exact with the model."""
    u0 = mixed_f64(0)
    say("hilo 4096 T=10")
    got = to_host(ops.jacobi5_hilo(to_dev(u0), 10))
    assert np.array_equal(got, oracle.jacobi5_hilo_model(u0, 10))
    ref = oracle.jacobi5(u0, 10)
    rep = oracle.error_report(got, ref, oracle.abs_reference(u0, 10))
    say(f"hilo 4096 T=10 errors {rep}")
    assert rep["componentwise"] <= 1e-10 and rep["normwise"] <= 1e-10


def test_hilo_full_size_T100_sampled(ops):
    """4096x4096 at T = 100 (the benchmarked call): sampled outputs bit-exact with the
    model on their dependence cones, and within 1e-10 componentwise of FP64."""
    u0 = mixed_f64(0)
    T = 100
    say("hilo 4096 T=100")
    got = to_host(ops.jacobi5_hilo(to_dev(u0), T))
    H, W = u0.shape
    worst = 0.0
    for (i, j) in sample_points(H, W, 32, seed=2):
        r0, r1, c0, c1 = cone_window(H, W, i, j, T)
        sub = u0[r0:r1 + 1, c0:c1 + 1]
        m = oracle.jacobi5_hilo_model(sub, T)
        assert got[i, j] == m[i - r0, j - c0], f"point {(i, j)}"
        ref = oracle.jacobi5(sub, T)[i - r0, j - c0]
        scale = oracle.abs_reference(sub, T)[i - r0, j - c0]
        if scale > 0:
            worst = max(worst, abs(got[i, j] - ref) / scale)
    say(f"hilo T=100 sampled componentwise {worst:.3e}")
    assert worst <= 1e-10


def test_hilo_beyond_int32_points(ops):
    """46400 x 46400 (2.15e9 points, past 2^31): encode, 5 encoded sweeps and decode, sampled outputs
    bit-exact with the model on their dependence cones."""
    import torch

    from workloads import hashed_grid, hashed_rows_torch

    n, T = 46400, 5
    dev = device()
    say(f"hilo beyond int32: fill {n}x{n}")
    u0 = torch.empty((n, n), dtype=torch.float64, device=dev)
    for r0 in range(0, n, 2048):
        u0[r0:min(n, r0 + 2048)] = hashed_rows_torch(r0, min(n, r0 + 2048), n, dev, seed=31)
    say(f"hilo beyond int32: T={T}")
    got = ops.jacobi5_hilo(u0, T)
    pts = sample_points(n, n, 24, seed=4) + [(n - 2, n // 2), (n // 2, n - 2), (46341, 46341)]
    flat = torch.tensor([i * n + j for i, j in pts], dtype=torch.int64, device=dev)
    vals = to_host(got.view(-1)[flat])
    del got, u0
    torch.cuda.empty_cache()
    for k, (i, j) in enumerate(pts):
        r0, r1, c0, c1 = cone_window(n, n, i, j, T)
        m = oracle.jacobi5_hilo_model(hashed_grid(r0, r1 + 1, c0, c1 + 1, seed=31), T)
        assert vals[k] == m[i - r0, j - c0], f"point {(i, j)}"


def test_hilo_errors(ops):
    import torch

    from paper_2512_19851_amd import _lib

    lib = _lib.load()
    stream = torch.cuda.current_stream().cuda_stream
    u0 = to_dev(normal_grid(8, 8))
    out = torch.empty_like(u0)
    need = ops.hilo_work_bytes(8, 8)
    work = torch.empty(need, dtype=torch.uint8, device=u0.device)
    say("hilo error paths")
    assert lib.sten_jacobi5_f64_hilo(u0.data_ptr(), out.data_ptr(), work.data_ptr(), need - 1, 8, 8, 8, 2,
                                     0.25, stream) == -4
    assert lib.sten_jacobi5_f64_hilo(u0.data_ptr(), out.data_ptr(), work.data_ptr() + 8, need, 8, 8, 8, 2,
                                     0.25, stream) == -1
    assert lib.sten_jacobi5_f64_hilo(u0.data_ptr(), u0.data_ptr(), work.data_ptr(), need, 8, 8, 8, 2,
                                     0.25, stream) == -2
    torch.cuda.synchronize()
