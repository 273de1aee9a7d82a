"""Tiled execution on one GPU (chares with depth-1 ghosts) against the oracle, via the C ABI.

Any tiling must give the single-grid result bit for bit; re-tiling a running
computation (a one-GPU stand-in for shrink/expand) must not change it either.
"""

import numpy as np
import pytest

import oracle
from tests.gpu_util import device, say, to_dev, to_host
from workloads import large_f64, normal_grid, unit_ring_grid

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ops():
    device()
    from paper_2512_19851_amd import ops

    return ops


CASES = [((5, 7), (1, 1)), ((5, 7), (2, 3)), ((5, 7), (5, 7)), ((64, 64), (2, 2)), ((64, 64), (4, 4)),
         ((130, 513), (3, 5)), ((257, 1031), (2, 3)), ((257, 1031), (7, 1)), ((100, 300), (1, 6)),
         ((3, 600), (3, 4)), ((600, 3), (5, 3))]


@pytest.mark.parametrize("shape,tiling", CASES, ids=lambda v: f"{v[0]}x{v[1]}")
def test_tiled_bit_exact(ops, shape, tiling):
    u0 = normal_grid(*shape, seed=sum(shape) + sum(tiling))
    d = to_dev(u0)
    for T in (0, 1, 2, 3, 10):
        say(f"tiled {shape} {tiling} T={T}")
        t = ops.TiledGrid(*shape, *tiling)
        t.scatter(d)
        t.run(T)
        got = to_host(t.gather())
        assert np.array_equal(got, oracle.jacobi5(u0, T)), f"{shape} {tiling} T={T}"
        st = t.stats()
        assert st["tiles"] == tiling[0] * tiling[1]
        if tiling != (1, 1):
            assert st["exchanges"] == T


def test_separate_comm_stream(ops):
    import torch

    u0 = unit_ring_grid(200, 333)
    s = torch.cuda.Stream()
    say("tiled comm stream")
    t = ops.TiledGrid(200, 333, 3, 4, comm_stream=s)
    t.scatter(to_dev(u0))
    t.run(25)
    assert np.array_equal(to_host(t.gather()), oracle.jacobi5(u0, 25))


def test_epochs_skip_redundant_exchange(ops):
    u0 = normal_grid(40, 60, seed=3)
    t = ops.TiledGrid(40, 60, 2, 2)
    t.scatter(to_dev(u0))
    say("tiled epochs")
    t.exchange()
    t.exchange()  # nothing was written since: skipped
    st = t.stats()
    assert st["exchanges"] == 1 and st["skipped"] == 1
    t.run(3)  # the first sweep reads the array just exchanged: skipped again
    st = t.stats()
    assert st["exchanges"] == 3 and st["skipped"] == 2
    assert np.array_equal(to_host(t.gather()), oracle.jacobi5(u0, 3))


@pytest.mark.parametrize("plan", [[(2, 2, 4), (4, 1, 5), (1, 3, 6)], [(1, 1, 7), (3, 3, 7)], [(5, 2, 1), (2, 5, 9)]])
def test_retiling_mid_run_keeps_result(ops, plan):
    """Checkpoint the grid, restore it under another tiling, continue: same bits as no re-tiling."""
    u0 = normal_grid(97, 143, seed=11)
    cur = to_dev(u0)
    total = 0
    for pr, pc, T in plan:
        say(f"retile {pr}x{pc} T={T}")
        t = ops.TiledGrid(97, 143, pr, pc)
        t.scatter(cur)
        t.run(T)
        cur = t.gather()
        total += T
    assert np.array_equal(to_host(cur), oracle.jacobi5(u0, total))


def test_full_size_tiled(ops):
    u0 = large_f64(0)
    say("tiled 4096 2x2 T=10")
    t = ops.TiledGrid(4096, 4096, 2, 2)
    t.scatter(to_dev(u0))
    t.run(10)
    assert np.array_equal(to_host(t.gather()), oracle.jacobi5(u0, 10))


def test_invalid_tiling(ops):
    with pytest.raises(ValueError):
        ops.TiledGrid(4, 4, 5, 1)
