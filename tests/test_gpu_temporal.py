"""Temporal blocking (several sweeps per HBM pass) is bit-identical to the oracle, via the C ABI."""

import numpy as np
import pytest

import oracle
from tests.gpu_util import cone_window, device, sample_points, say, to_dev, to_host
from workloads import large_f64, normal_grid

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ops():
    device()
    from paper_2512_19851_amd import ops

    return ops


SHAPES = [(3, 3), (5, 7), (9, 130), (64, 64), (63, 65), (257, 1031), (130, 2049), (600, 3), (3, 600), (17, 250)]


@pytest.mark.parametrize("dtype", [np.float64, np.float32], ids=["f64", "f32"])
@pytest.mark.parametrize("shape", SHAPES, ids=lambda s: f"{s[0]}x{s[1]}")
def test_tb_bit_exact(ops, shape, dtype):
    u0 = normal_grid(*shape, seed=sum(shape), dtype=dtype)
    d = to_dev(u0)
    for levels in (1, 2, 3, 4):
        for T in (1, 2, 3, 5, 10):
            say(f"tb {dtype.__name__} {shape} levels={levels} T={T}")
            got = to_host(ops.jacobi5_tb(d, T, levels=levels))
            assert np.array_equal(got, oracle.jacobi5(u0, T, dtype=dtype)), f"{shape} L={levels} T={T}"


def test_tb_general_coefficient(ops):
    u0 = normal_grid(70, 300, seed=2)
    say("tb c=0.3")
    assert np.array_equal(to_host(ops.jacobi5_tb(to_dev(u0), 7, 0.3, levels=3)), oracle.jacobi5(u0, 7, 0.3))


def test_tb_full_size(ops):
    u0 = large_f64(0)
    d = to_dev(u0)
    want = oracle.jacobi5(u0, 10)
    for levels in (2, 4):
        say(f"tb 4096 levels={levels} T=10")
        assert np.array_equal(to_host(ops.jacobi5_tb(d, 10, levels=levels)), want)


def test_tb_full_size_T100_sampled(ops):
    u0 = large_f64(0)
    T = 100
    say("tb 4096 T=100 sampled")
    got = to_host(ops.jacobi5_tb(to_dev(u0), T, levels=4))
    H, W = u0.shape
    for (i, j) in sample_points(H, W, 32, seed=3):
        r0, r1, c0, c1 = cone_window(H, W, i, j, T)
        sub = oracle.jacobi5(u0[r0:r1 + 1, c0:c1 + 1], T)
        assert got[i, j] == sub[i - r0, j - c0], f"point {(i, j)}"


def test_tb_unsupported_falls_back(ops):
    import torch

    u0 = normal_grid(40, 99, seed=4)
    t = torch.empty((40, 101), dtype=torch.float64, device=device())[:, :99]
    t.copy_(to_dev(u0))
    say("tb odd ld fallback")
    assert np.array_equal(to_host(ops.jacobi5_tb(t, 5, levels=2)), oracle.jacobi5(u0, 5))
