"""Tiled execution on one GPU (chares with ghost frames) against the oracle, via the C ABI.

Any tiling and any ghost depth must give the single-grid result bit for bit;
re-tiling a running computation (a one-GPU stand-in for shrink/expand) must
not change it either.
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


@pytest.mark.parametrize("exchange", ["packed", "direct"])
@pytest.mark.parametrize("shape,tiling", CASES, ids=lambda v: f"{v[0]}x{v[1]}")
def test_tiled_bit_exact(ops, shape, tiling, exchange):
    u0 = normal_grid(*shape, seed=sum(shape) + sum(tiling))
    d = to_dev(u0)
    for T in (0, 1, 2, 3, 10):
        say(f"tiled {exchange} {shape} {tiling} T={T}")
        t = ops.TiledGrid(*shape, *tiling, exchange=exchange)
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


GHOST_CASES = [((64, 64), (2, 2), 2), ((64, 64), (4, 4), 12), ((130, 513), (3, 5), 3), ((257, 1031), (2, 3), 10),
               ((257, 1031), (7, 1), 12), ((100, 300), (1, 6), 5), ((3, 600), (1, 4), 12), ((600, 3), (5, 1), 12),
               ((41, 512), (2, 2), 7), ((97, 143), (6, 7), 4), ((300, 260), (3, 2), 12), ((40, 40), (8, 8), 5)]


@pytest.mark.parametrize("exchange", ["packed", "direct"])
@pytest.mark.parametrize("shape,tiling,g", GHOST_CASES, ids=lambda v: str(v))
def test_tiled_deep_ghosts_bit_exact(ops, shape, tiling, g, exchange):
    """Up to g sweeps per exchange (blocked kernel over all tile views, corners exchanged) give the same bits."""
    u0 = normal_grid(*shape, seed=7 * sum(shape) + g)
    d = to_dev(u0)
    for T in (0, 1, 2, 3, g, g + 1, 2 * g + 3, 25):
        say(f"tiled ghost {exchange} {shape} {tiling} g={g} T={T}")
        t = ops.TiledGrid(*shape, *tiling, ghost=g, exchange=exchange)
        t.scatter(d)
        t.run(T)
        got = to_host(t.gather())
        assert np.array_equal(got, oracle.jacobi5(u0, T)), f"{shape} {tiling} g={g} T={T}"
        st = t.stats()
        assert st["ghost"] == g and st["mode"] == ops.TiledGrid.MODES[exchange]
        if tiling != (1, 1):
            assert st["exchanges"] == -(-T // g)


@pytest.mark.parametrize("exchange", ["packed", "direct"])
def test_tiled_deep_ghosts_many_tiles(ops, exchange):
    """More tiles than one blocked launch takes (32): the chunk spans two launches."""
    u0 = normal_grid(120, 150, seed=5)
    say(f"tiled ghost {exchange} 6x7 tiles g=3")
    t = ops.TiledGrid(120, 150, 6, 7, ghost=3, exchange=exchange)
    t.scatter(to_dev(u0))
    t.run(14)
    assert np.array_equal(to_host(t.gather()), oracle.jacobi5(u0, 14))
    st = t.stats()
    assert st["tiles"] == 42 and st["exchanges"] == 5
    # chunks 3,3,3,3,2: two launches per chunk
    assert st["sweep_launches"] == 10


@pytest.mark.parametrize("exchange", ["packed", "direct"])
def test_tiled_deep_ghosts_comm_stream_and_epochs(ops, exchange):
    import torch

    u0 = unit_ring_grid(200, 333)
    s = torch.cuda.Stream()
    say(f"tiled ghost {exchange} comm stream")
    t = ops.TiledGrid(200, 333, 3, 4, comm_stream=s, ghost=6, exchange=exchange)
    t.scatter(to_dev(u0))
    t.exchange()
    t.exchange()
    t.run(25)  # chunks 5 x 5 sweeps; the first exchange is skipped
    st = t.stats()
    assert st["exchanges"] == 5 and st["skipped"] == 2
    assert np.array_equal(to_host(t.gather()), oracle.jacobi5(u0, 25))


@pytest.mark.parametrize("plan", [[(2, 2, 4, 9, "packed"), (4, 1, 1, 5, "direct"), (1, 3, 12, 26, "packed")],
                                  [(3, 3, 7, 7, "direct"), (2, 5, 2, 3, "packed")]])
def test_retiling_with_ghost_depths(ops, plan):
    u0 = normal_grid(97, 143, seed=13)
    cur = to_dev(u0)
    total = 0
    for pr, pc, g, T, mode in plan:
        say(f"retile {pr}x{pc} g={g} {mode} T={T}")
        t = ops.TiledGrid(97, 143, pr, pc, ghost=g, exchange=mode)
        t.scatter(cur)
        t.run(T)
        cur = t.gather()
        total += T
    assert np.array_equal(to_host(cur), oracle.jacobi5(u0, total))


def test_full_size_tiled_deep_ghosts(ops):
    u0 = large_f64(1)
    d = to_dev(u0)
    want = oracle.jacobi5(u0, 23)
    for mode, (pr, pc) in (("packed", (2, 2)), ("direct", (3, 3))):
        say(f"tiled 4096 {pr}x{pc} g=10 {mode} T=23")
        t = ops.TiledGrid(4096, 4096, pr, pc, ghost=10, exchange=mode)
        t.scatter(d)
        t.run(23)
        assert np.array_equal(to_host(t.gather()), want), mode


def test_invalid_ghost_depth(ops):
    for g in (0, 13):
        with pytest.raises(ValueError):
            ops.TiledGrid(64, 64, 2, 2, ghost=g)
    with pytest.raises(ValueError):
        ops.TiledGrid(20, 64, 4, 1, ghost=6)
    with pytest.raises(ValueError):
        ops.TiledGrid(64, 64, 2, 2, exchange="mail")


def test_invalid_tiling(ops):
    with pytest.raises(ValueError):
        ops.TiledGrid(4, 4, 5, 1)


@pytest.mark.parametrize("exchange", ["packed", "direct"])
def test_tiled_depth1_one_launch_per_sweep(ops, exchange):
    """Depth-1 ghosts: each sweep is one launch of the single-sweep kernel over all tiles (per 32 tiles),
    bit-identical to the single grid; 42 tiles take two launches per sweep, 4 x 4 tiles one."""
    for (pr, pc, launches) in [(6, 7, 2), (4, 4, 1)]:
        u0 = normal_grid(200, 301, seed=pr * pc)
        say(f"tiled depth 1 {exchange} {pr}x{pc}")
        t = ops.TiledGrid(200, 301, pr, pc, ghost=1, exchange=exchange)
        t.scatter(to_dev(u0))
        t.run(5)
        assert np.array_equal(to_host(t.gather()), oracle.jacobi5(u0, 5))
        st = t.stats()
        assert st["sweep_launches"] == 5 * launches


def test_depth1_direct_exchange_in_the_sweep(ops):
    """Direct mode at depth 1: every sweep but a run's last also stores the tiles' edge rows and columns into
    their neighbours' ghost cells (the exchange done inside the sweep). Runs continue bit-exact across calls
    and with a separate exchange in between, and the exchanges still number one per sweep; a tiling with
    tiles too small to sweep (1-row tiles) falls back to separate exchanges."""
    u0 = normal_grid(130, 517, seed=21)
    t = ops.TiledGrid(130, 517, 3, 4, ghost=1, exchange="direct")
    t.scatter(to_dev(u0))
    say("tiled depth 1 direct fused: 4 + 3 sweeps, exchange, 2 sweeps")
    t.run(4)
    t.run(3)
    assert np.array_equal(to_host(t.gather()), oracle.jacobi5(u0, 7))
    st = t.stats()
    assert st["exchanges"] == 7 and st["skipped"] == 0 and st["sweep_launches"] == 7
    t.exchange()
    t.run(2)
    assert np.array_equal(to_host(t.gather()), oracle.jacobi5(u0, 9))
    st = t.stats()  # the run's first exchange finds the ghosts fresh and is skipped
    assert st["exchanges"] == 9 and st["skipped"] == 1
    u1 = normal_grid(12, 40, seed=2)
    t2 = ops.TiledGrid(12, 40, 12, 2, ghost=1, exchange="direct")
    t2.scatter(to_dev(u1))
    say("tiled depth 1 direct, 1-row tiles")
    t2.run(6)
    assert np.array_equal(to_host(t2.gather()), oracle.jacobi5(u1, 6))
    assert t2.stats()["exchanges"] == 6


@pytest.mark.parametrize("exchange", ["packed", "direct"])
def test_depth1_views_past_whole_blocks(ops, exchange):
    """Tile views 513, 514, 515 and 1026 columns wide: the one-sweep launch over all tiles covers 512 columns
    per block and leaves the last 0 to 2 interior columns of a row to one thread; bit-exact for T = 1..4."""
    for (H, W, pr, pc) in [(40, 1024, 1, 2), (40, 1026, 1, 2), (40, 1028, 1, 2), (30, 1536, 2, 3), (20, 4096, 2, 4)]:
        u0 = normal_grid(H, W, seed=W + pr)
        for T in (1, 2, 4):
            say(f"tiled depth 1 {exchange} {H}x{W} {pr}x{pc} T={T}")
            t = ops.TiledGrid(H, W, pr, pc, ghost=1, exchange=exchange)
            t.scatter(to_dev(u0))
            t.run(T)
            assert np.array_equal(to_host(t.gather()), oracle.jacobi5(u0, T)), f"{H}x{W} {pr}x{pc} T={T}"
