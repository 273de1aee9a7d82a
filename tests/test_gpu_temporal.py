"""Temporal blocking (several sweeps per HBM pass) is bit-identical to the oracle, via the C ABI.

Both blocked kernels run: the register tile (levels 1..6) and the streaming
kernel (levels 1..12, several band heights, both strip layouts).
"""

import numpy as np
import pytest

import oracle
from tests.gpu_util import cone_window, device, sample_points, say, to_dev, to_host
from workloads import large_f64, normal_grid

pytestmark = pytest.mark.gpu

BLOCK, STREAM = 1, 2
VARIANTS = [("block", BLOCK, range(1, 7)), ("stream", STREAM, range(1, 13))]


@pytest.fixture(scope="module")
def ops():
    device()
    from paper_2512_19851_amd import ops

    yield ops
    ops.set_tb(0, 0, 0)


SHAPES = [(3, 3), (5, 7), (9, 130), (64, 64), (63, 65), (257, 1031), (130, 2049), (600, 3), (3, 600), (17, 250),
          (41, 512), (12, 260)]
TS = (1, 2, 3, 5, 10, 17)


@pytest.mark.parametrize("dtype", [np.float64, np.float32], ids=["f64", "f32"])
@pytest.mark.parametrize("shape", SHAPES, ids=lambda s: f"{s[0]}x{s[1]}")
def test_tb_bit_exact(ops, shape, dtype):
    u0 = normal_grid(*shape, seed=sum(shape), dtype=dtype)
    d = to_dev(u0)
    want = {T: oracle.jacobi5(u0, T, dtype=dtype) for T in TS}
    try:
        for name, variant, levels_range in VARIANTS:
            ops.set_tb(variant, 0, 0)
            if dtype == np.float64:  # FP64 launches of 13 and 14 sweeps (2 waves per SIMD), either variant
                levels_range = list(levels_range) + [13, 14]
            for levels in levels_range:
                for T in TS:
                    say(f"tb {name} {dtype.__name__} {shape} levels={levels} T={T}")
                    got = to_host(ops.jacobi5_tb(d, T, levels=levels))
                    assert np.array_equal(got, want[T]), f"{name} {shape} L={levels} T={T}"
    finally:
        ops.set_tb(0, 0, 0)


@pytest.mark.parametrize("variant", [STREAM], ids=["stream"])
@pytest.mark.parametrize("depth", [0, 4])
@pytest.mark.parametrize("band", [1, 2, 7, 32, 1000])
def test_tb_stream_band_and_depth(ops, band, depth, variant):
    """Band heights that leave a ragged last band, a band of one row, and one band for the whole grid;
    widths that give the right-aligned strip layout (multiple of the vector width, >= 64 vectors) and
    widths that do not."""
    cases = [((131, 300), np.float64), ((67, 1030), np.float32), ((40, 2049), np.float64),
             ((29, 1032), np.float32), ((33, 128), np.float64), ((30, 256), np.float32), ((45, 258), np.float64),
             ((37, 1030), np.float64), ((21, 257), np.float64)]
    try:
        ops.set_tb(variant, band, depth)
        for shape, dtype in cases:
            u0 = normal_grid(*shape, seed=band + depth + shape[0], dtype=dtype)
            d = to_dev(u0)
            for levels in (1, 3, 5, 8, 10, 12):
                T = 11
                say(f"tb variant={variant} band={band} depth={depth} {shape} {dtype.__name__} levels={levels}")
                got = to_host(ops.jacobi5_tb(d, T, levels=levels))
                assert np.array_equal(got, oracle.jacobi5(u0, T, dtype=dtype)), f"{shape} L={levels}"
    finally:
        ops.set_tb(0, 0, 0)


def test_tb_general_coefficient(ops):
    u0 = normal_grid(70, 300, seed=2)
    want = oracle.jacobi5(u0, 7, 0.3)
    try:
        for name, variant, _ in VARIANTS:
            ops.set_tb(variant, 0, 0)
            say(f"tb {name} c=0.3")
            assert np.array_equal(to_host(ops.jacobi5_tb(to_dev(u0), 7, 0.3, levels=3)), want)
    finally:
        ops.set_tb(0, 0, 0)


def test_tb_levels_out_of_range(ops):
    """FP64 1..14 and FP32 1..12 levels under either variant (the register tile hands launches of more
    than 6 sweeps to the streaming kernel); 0, 15 (FP64) and 13 (FP32) are rejected."""
    u = normal_grid(20, 20, seed=1)
    u0 = to_dev(u)
    u32 = normal_grid(20, 24, seed=2, dtype=np.float32)
    d32 = to_dev(u32)
    try:
        for variant in (BLOCK, STREAM):
            ops.set_tb(variant, 0, 0)
            assert np.array_equal(to_host(ops.jacobi5_tb(u0, 10, levels=7)), oracle.jacobi5(u, 10))
            assert np.array_equal(to_host(ops.jacobi5_tb(u0, 28, levels=14)), oracle.jacobi5(u, 28))
            assert np.array_equal(to_host(ops.jacobi5_tb(d32, 12, levels=12)),
                                  oracle.jacobi5(u32, 12, dtype=np.float32))
            for bad in (0, 15):
                with pytest.raises(ops._lib.StenError):
                    ops.jacobi5_tb(u0, 10, levels=bad)
            with pytest.raises(ops._lib.StenError):
                ops.jacobi5_tb(d32, 10, levels=13)
    finally:
        ops.set_tb(0, 0, 0)


def test_tb_full_size(ops):
    """4096 x 4096 FP64, the benchmark's launch configuration among others, against the oracle."""
    u0 = large_f64(0)
    d = to_dev(u0)
    want = oracle.jacobi5(u0, 10)
    try:
        for name, variant, levels_list in [("block", BLOCK, (2, 4, 5)), ("stream", STREAM, (2, 5, 8, 10, 12))]:
            ops.set_tb(variant, 0, 0)
            for levels in levels_list:
                say(f"tb {name} 4096 levels={levels} T=10")
                assert np.array_equal(to_host(ops.jacobi5_tb(d, 10, levels=levels)), want)
    finally:
        ops.set_tb(0, 0, 0)


def test_tb_full_size_T100_sampled(ops):
    """The benchmark's step (built-in schedule, T = 100) on sampled points, each from its dependence cone."""
    u0 = large_f64(0)
    T = 100
    say("tb 4096 T=100 sampled (built-in)")
    got = to_host(ops.jacobi5(to_dev(u0), T))
    H, W = u0.shape
    for (i, j) in sample_points(H, W, 32, seed=3, stream=(2, 11)):
        r0, r1, c0, c1 = cone_window(H, W, i, j, T)
        sub = oracle.jacobi5(u0[r0:r1 + 1, c0:c1 + 1], T)
        assert got[i, j] == sub[i - r0, j - c0], f"point {(i, j)}"


@pytest.mark.parametrize("T", [28, 100])
def test_f64_deep_schedule_sampled(ops, T):
    """FP64 through the plain call at 8192^2, where one buffer is past half the MALL and the built-in
    schedule takes 14 sweeps per launch (2 waves per SIMD): T = 28 is two launches of 14, T = 100 four of
    13 and four of 12; sampled points, each from its dependence cone, with the deep kernel's band edges
    (342-row bands) among them."""
    n = 8192
    u0 = large_f64(0, n)
    say(f"f64 {n} T={T} sampled (built-in, deep launches)")
    got = to_host(ops.jacobi5(to_dev(u0), T))
    for (i, j) in sample_points(n, n, 24, seed=T, stream=(2, 14, (342, 171))):
        r0, r1, c0, c1 = cone_window(n, n, i, j, T)
        sub = oracle.jacobi5(u0[r0:r1 + 1, c0:c1 + 1], T)
        assert got[i, j] == sub[i - r0, j - c0], f"point {(i, j)}"


def test_tb_unsupported_falls_back(ops):
    import torch

    u0 = normal_grid(40, 99, seed=4)
    t = torch.empty((40, 101), dtype=torch.float64, device=device())[:, :99]
    t.copy_(to_dev(u0))
    say("tb odd ld fallback")
    assert np.array_equal(to_host(ops.jacobi5_tb(t, 5, levels=2)), oracle.jacobi5(u0, 5))


def test_f32_full_size_default_schedule(ops):
    """4096 x 4096 FP32 through the plain call (built-in schedule: 8 sweeps per launch) vs the FP32 oracle."""
    u0 = large_f64(0).astype(np.float32)
    say("f32 4096 T=10 built-in schedule")
    got = to_host(ops.jacobi5(to_dev(u0), 10))
    assert np.array_equal(got, oracle.jacobi5(u0, 10, dtype=np.float32))


@pytest.mark.parametrize("n,T", [(4096, 100), (8192, 25)], ids=["4096-T100", "8192-T25"])
def test_f32_default_schedule_sampled(ops, n, T):
    """FP32 through the plain call on sampled points, each from its dependence cone: 4096^2 at T = 100
    (8 sweeps per launch: 100 sweeps split over 13 launches) and 8192^2 at T = 25 (one buffer past half
    the MALL: 12 sweeps per launch, 25 split over 3 launches)."""
    u0 = large_f64(0, n).astype(np.float32)
    say(f"f32 {n} T={T} sampled (built-in)")
    got = to_host(ops.jacobi5(to_dev(u0), T))
    for (i, j) in sample_points(n, n, 24, seed=T, stream=(4, 8 if n == 4096 else 12)):
        r0, r1, c0, c1 = cone_window(n, n, i, j, T)
        sub = oracle.jacobi5(u0[r0:r1 + 1, c0:c1 + 1], T, dtype=np.float32)
        assert got[i, j] == sub[i - r0, j - c0], f"point {(i, j)}"


def test_register_variant_keeps_other_calls_whole(ops):
    """With the register-tile variant selected (it has launches of 1..6 sweeps), the plain calls'
    built-in schedule (up to 12 sweeps per launch) and the listing's chain of sweeps on two arrays
    still apply every sweep: launches of more than 6 sweeps take the streaming kernel."""
    import torch

    from paper_2512_19851_amd import _lib

    u0 = normal_grid(70, 300, seed=3)
    f32 = u0.astype(np.float32)
    try:
        ops.set_tb(BLOCK, 0, 0)
        for T in (6, 7, 12, 25, 100):
            say(f"register variant: jacobi5 default schedule T={T}")
            assert np.array_equal(to_host(ops.jacobi5(to_dev(u0), T)), oracle.jacobi5(u0, T)), f"f64 T={T}"
            assert np.array_equal(to_host(ops.jacobi5(to_dev(f32), T)), oracle.jacobi5(f32, T, dtype=np.float32))
        for m in (2, 8, 14, 27):
            a, b = to_dev(u0), to_dev(u0)  # equal rings, as the chain requires
            say(f"register variant: sweep chain m={m}")
            _lib.call("sten_sweep_chain_f64", a.data_ptr(), b.data_ptr(), 70, 300, 300, m, 0.25,
                      torch.cuda.current_stream().cuda_stream)
            last, prev = (b, a) if m % 2 else (a, b)
            assert np.array_equal(to_host(last), oracle.jacobi5(u0, m)), f"chain m={m}"
            assert np.array_equal(to_host(prev), oracle.jacobi5(u0, m - 1)), f"chain m={m} previous iterate"
    finally:
        ops.set_tb(0, 0, 0)
