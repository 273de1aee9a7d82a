"""GPU parity of the plain method (FP64 and FP32) against the CPU oracle, via the C ABI."""

import ctypes

import numpy as np
import pytest

import oracle
from tests.gpu_util import cone_window, device, sample_points, say, to_dev, to_host
from workloads import large_f64, normal_grid, small_f64, unit_ring_grid

pytestmark = pytest.mark.gpu

SHAPES = [(1, 1), (2, 9), (9, 2), (3, 3), (4, 4), (5, 7), (63, 65), (64, 64), (3, 600), (600, 3),
          (257, 1031), (1000, 513), (130, 2049)]
TS = [0, 1, 2, 3, 10]


@pytest.fixture(scope="module", params=["auto", "single"])
def ops(request):
    """Every plain-path test runs under the built-in schedule and one sweep per launch."""
    device()
    from paper_2512_19851_amd import ops

    ops.set_schedule(0 if request.param == "auto" else 1)
    yield ops
    ops.set_schedule(0)


@pytest.mark.parametrize("shape", SHAPES, ids=lambda s: f"{s[0]}x{s[1]}")
def test_f64_bit_exact(ops, shape):
    u0 = normal_grid(*shape, seed=sum(shape))
    d = to_dev(u0)
    for T in TS:
        say(f"f64 {shape} T={T}")
        got = to_host(ops.jacobi5(d, T))
        want = oracle.jacobi5(u0, T)
        assert np.array_equal(got, want), f"{shape} T={T}: max diff {np.max(np.abs(got - want))}"


@pytest.mark.parametrize("shape", SHAPES, ids=lambda s: f"{s[0]}x{s[1]}")
def test_f32_bit_exact(ops, shape):
    u0 = normal_grid(*shape, seed=sum(shape) + 1, dtype=np.float32)
    d = to_dev(u0)
    for T in TS:
        say(f"f32 {shape} T={T}")
        got = to_host(ops.jacobi5(d, T))
        want = oracle.jacobi5(u0, T, dtype=np.float32)
        assert got.dtype == np.float32
        assert np.array_equal(got, want), f"{shape} T={T}"
        if T > 0:
            err = np.abs(got.astype(np.float64) - oracle.jacobi5(u0.astype(np.float64), T))
            assert np.all(err <= oracle.bound_fp32(u0, T))


def test_small_config_paper_shape(ops):
    """64x64 FP64, N(0,1), seed 0: the small workload, all parity T values and T = 100."""
    u0 = small_f64(0)
    d = to_dev(u0)
    for T in TS + [100]:
        say(f"small T={T}")
        assert np.array_equal(to_host(ops.jacobi5(d, T)), oracle.jacobi5(u0, T))


def test_general_coefficient(ops):
    u0 = normal_grid(77, 301, seed=9)
    for c in (0.3, -1.5, 1.0 / 3.0):
        say(f"c={c}")
        assert np.array_equal(to_host(ops.jacobi5(to_dev(u0), 5, c)), oracle.jacobi5(u0, 5, c))


def test_unit_ring_listing_state(ops):
    u0 = unit_ring_grid(300, 517)
    say("unit ring")
    got = to_host(ops.jacobi5(to_dev(u0), 37))
    assert np.array_equal(got, oracle.jacobi5(u0, 37))


@pytest.mark.parametrize("rows", [4, 8, 16])
def test_rows_per_tile_variants(ops, rows):
    u0 = normal_grid(203, 777, seed=rows)
    ops.set_sweep_rows(rows)
    try:
        for T in (1, 4):
            say(f"rows={rows} T={T}")
            assert np.array_equal(to_host(ops.jacobi5(to_dev(u0), T)), oracle.jacobi5(u0, T))
    finally:
        ops.set_sweep_rows(0)


@pytest.mark.parametrize("dtype", [np.float64, np.float32])
def test_strided_and_misaligned_views(ops, dtype):
    """Row stride ld > W, odd ld, and a base pointer off 16-byte alignment (scalar path)."""
    import torch

    rng_grid = normal_grid(70, 140, seed=3, dtype=dtype)
    big = to_dev(rng_grid)
    for (c0, W) in [(0, 100), (1, 100), (3, 97), (0, 139)]:
        view = big[:, c0:c0 + W]
        assert view.stride(0) == 140
        u0 = rng_grid[:, c0:c0 + W]
        for T in (1, 2, 7):
            say(f"view {dtype.__name__} c0={c0} W={W} T={T}")
            got = ops.jacobi5(view, T)
            assert got.stride(0) == 140
            want = oracle.jacobi5(u0, T, dtype=dtype)
            assert np.array_equal(to_host(got), want)
    # odd row stride
    odd = torch.empty((50, 101), dtype=big.dtype, device=big.device)[:, :99]
    u0 = normal_grid(50, 99, seed=4, dtype=dtype)
    odd.copy_(to_dev(u0))
    say("odd ld")
    assert np.array_equal(to_host(ops.jacobi5(odd, 5)), oracle.jacobi5(u0, 5, dtype=dtype))


@pytest.mark.parametrize("dtype", [np.float64, np.float32])
def test_strided_view_wide(ops, dtype):
    """ld > W with W a multiple of the vector width and >= 64 vectors (the strip layout aligned with the
    grid's sides), and with W just above it."""
    rng_grid = normal_grid(70, 300, seed=6, dtype=dtype)
    big = to_dev(rng_grid)
    for W in (256, 260, 296):
        view = big[:, :W]
        u0 = rng_grid[:, :W]
        for T in (1, 3, 11):
            say(f"wide view {dtype.__name__} W={W} T={T}")
            assert np.array_equal(to_host(ops.jacobi5(view, T)), oracle.jacobi5(u0, T, dtype=dtype))


def test_odd_large_shape(ops):
    """4097 x 4095 FP64 (odd sizes, past 2^24 points): whole-grid bit-exact for odd and even T."""
    u0 = normal_grid(4097, 4095, seed=7)
    d = to_dev(u0)
    for T in (1, 2, 3, 10):
        say(f"4097x4095 T={T}")
        assert np.array_equal(to_host(ops.jacobi5(d, T)), oracle.jacobi5(u0, T)), f"T={T}"


def test_single_sweep_entry_keeps_ring(ops):
    import torch

    u0 = normal_grid(33, 515, seed=5)
    src = to_dev(u0)
    dst = torch.full_like(src, float("nan"))
    say("single sweep")
    ops.sweep(src, dst)
    got = to_host(dst)
    want = oracle.jacobi5(u0, 1)
    assert np.array_equal(got[1:-1, 1:-1], want[1:-1, 1:-1])
    assert np.all(np.isnan(got[0, :])) and np.all(np.isnan(got[:, 0]))
    assert np.all(np.isnan(got[-1, :])) and np.all(np.isnan(got[:, -1]))


def test_large_f64_full_compare(ops):
    """4096x4096 FP64 (2^24 points), seed 0: whole-grid bit-exact at T = 1, 2, 10."""
    u0 = large_f64(0)
    d = to_dev(u0)
    for T in (1, 2, 10):
        say(f"large T={T}")
        got = to_host(ops.jacobi5(d, T))
        assert np.array_equal(got, oracle.jacobi5(u0, T)), f"T={T}"


def test_large_f64_sampled_bench_config(ops):
    """4096x4096 FP64 at T = 100 (the benchmarked call): bit-exact on sampled points.

    Each sampled point is recomputed by the oracle on its dependence cone.
    """
    u0 = large_f64(0)
    T = 100
    say("large sampled T=100")
    got = to_host(ops.jacobi5(to_dev(u0), T))
    H, W = u0.shape
    for (i, j) in sample_points(H, W, 48, seed=1, stream=(2, 11)):
        r0, r1, c0, c1 = cone_window(H, W, i, j, T)
        sub = oracle.jacobi5(u0[r0:r1 + 1, c0:c1 + 1], T)
        assert got[i, j] == sub[i - r0, j - c0], f"point {(i, j)}"
    # properties that hold at any size: ring unchanged, maximum principle
    assert np.array_equal(got[0, :], u0[0, :]) and np.array_equal(got[:, -1], u0[:, -1])
    assert got.min() >= u0.min() and got.max() <= u0.max()


@pytest.mark.parametrize("dtype", [np.float64, np.float32], ids=["f64", "f32"])
def test_beyond_int32_points(ops, dtype):
    """46400 x 46400: 2.15e9 points, past 2^31 (17.2 GB per FP64 buffer). Sampled outputs bit-exact
    with the oracle on their dependence cones after one launch (T = 12) and two (T = 23); row
    offsets beyond 32 bits on every kernel of the path (ring copy, sweeps, stores)."""
    import torch

    from workloads import hashed_grid, hashed_rows_torch

    n = 46400
    dev = device()
    tdt = torch.float64 if dtype == np.float64 else torch.float32
    say(f"beyond int32 {dtype.__name__}: fill {n}x{n}")
    u0 = torch.empty((n, n), dtype=tdt, device=dev)
    for r0 in range(0, n, 2048):
        u0[r0:min(n, r0 + 2048)] = hashed_rows_torch(r0, min(n, r0 + 2048), n, dev, seed=11).to(tdt)
    for T in (12, 23):
        say(f"beyond int32 {dtype.__name__}: T={T}")
        got = ops.jacobi5(u0, T)
        pts = sample_points(n, n, 24, seed=T, stream=(2, 12)) + [(n - 2, n // 2), (n // 2, n - 2), (46341, 46341)]
        flat = torch.tensor([i * n + j for i, j in pts], dtype=torch.int64, device=dev)
        vals = to_host(got.view(-1)[flat])
        del got
        torch.cuda.empty_cache()
        for k, (i, j) in enumerate(pts):
            r0, r1, c0, c1 = cone_window(n, n, i, j, T)
            win = hashed_grid(r0, r1 + 1, c0, c1 + 1, seed=11).astype(dtype)
            sub = oracle.jacobi5(win, T, dtype=dtype)
            assert vals[k] == sub[i - r0, j - c0], f"T={T} point {(i, j)}"
    del u0
    torch.cuda.empty_cache()  # hand the 2^31-point buffers back before the next test


def test_errors_reported(ops):
    import torch

    from paper_2512_19851_amd import StenError, _lib

    lib = _lib.load()
    d = to_dev(normal_grid(8, 8, seed=0))
    out = torch.empty_like(d)
    work = torch.empty_like(d)
    stream = torch.cuda.current_stream().cuda_stream
    say("error paths")
    # output aliasing the input: the listing's in-place rule
    assert lib.sten_jacobi5_f64(d.data_ptr(), d.data_ptr(), work.data_ptr(), 8, 8, 8, 2, 0.25, stream) == -2
    # host memory is not device memory
    host = np.zeros((8, 8))
    hp = host.ctypes.data_as(ctypes.c_void_p).value
    assert lib.sten_jacobi5_f64(d.data_ptr(), hp, work.data_ptr(), 8, 8, 8, 2, 0.25, stream) == -3
    # missing work buffer when two or more sweeps are asked for
    assert lib.sten_jacobi5_f64(d.data_ptr(), out.data_ptr(), None, 8, 8, 8, 2, 0.25, stream) == -3
    # T = 1 needs no work buffer
    assert lib.sten_jacobi5_f64(d.data_ptr(), out.data_ptr(), None, 8, 8, 8, 1, 0.25, stream) == 0
    with pytest.raises(StenError):
        ops.jacobi5(d, 2, out=d)
    # nothing sticky is left behind for torch
    torch.cuda.synchronize()
    assert torch.zeros(3, device=d.device).sum().item() == 0.0


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_plain_call_graph_replays(ops, dtype):
    """The plain call (ring copy + blocked launches, no allocation, no memset) captured in a HIP graph:
    every replay, with eager work on the output between replays, gives the eager call's bits."""
    import torch

    H, W, T = 600, 1024, 25
    u0 = large_f64(0, 1024)[:H, :W].copy()
    if dtype == "f32":
        u0 = u0.astype(np.float32)
    d = to_dev(u0)
    work = torch.empty_like(d)
    ref = ops.jacobi5(d, T, work=work)
    want = to_host(ref)
    assert np.array_equal(want, oracle.jacobi5(u0, T, dtype=u0.dtype.type))
    out = torch.empty_like(d)
    g = torch.cuda.CUDAGraph()
    s = torch.cuda.Stream()
    say(f"graph capture of the plain {dtype} call {H}x{W} T={T}")
    with torch.cuda.graph(g, stream=s):
        ops.jacobi5(d, T, out=out, work=work)
    for r in range(4):
        out.fill_(float("nan"))
        work.zero_()
        g.replay()
        got = to_host(out)
        assert np.array_equal(got, want), r
