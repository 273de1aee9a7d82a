"""Blocked pressure iterations of the cavity flow against the oracle, via the C ABI.

Several pressure iterations per pass over HBM (the walls applied at every
level inside the kernel) must give the bits of the oracle's one-at-a-time
iteration, for every level count, band height, ragged shape and both walk
directions of the bands.
"""

import numpy as np
import pytest

from oracle import cavity as oc
from tests.gpu_util import device, say, to_dev, to_host
from workloads import normal_grid

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ops():
    device()
    from paper_2512_19851_amd import ops

    yield ops
    ops.set_pressure_band(0)


def _want(p0, b, prm, nit):
    p = p0.copy()
    for _ in range(nit):
        p = oc.pressure_iteration(p, b, prm)
    return p


def _inputs(H, W, seed):
    # unequal spacings, so that the two neighbour weights differ
    prm = oc.CavityParams(H, W, lx=2.0, ly=1.3)
    return normal_grid(H, W, seed=seed), normal_grid(H, W, seed=seed + 1), prm


SHAPES = [(3, 128), (4, 130), (5, 256), (64, 128), (67, 258), (130, 300), (257, 1030), (40, 2050), (600, 128)]


@pytest.mark.parametrize("shape", SHAPES, ids=lambda s: f"{s[0]}x{s[1]}")
def test_pressure_bit_exact_every_level(ops, shape):
    H, W = shape
    p0, b, prm = _inputs(H, W, seed=H + W)
    dp, db = to_dev(p0), to_dev(b)
    for nit in (0, 1, 2, 3, 8, 9, 12, 13, 17, 25):
        want = _want(p0, b, prm, nit)
        for levels in range(0, 13):
            say(f"pressure {shape} nit={nit} levels={levels}")
            got = to_host(ops.cavity_pressure(dp, db, nit, prm.cw, prm.cn, prm.cb, levels=levels))
            assert np.array_equal(got, want), f"{shape} nit={nit} levels={levels}"


@pytest.mark.parametrize("band", [1, 2, 5, 16, 1000])
def test_pressure_band_heights(ops, band):
    """Bands of one row (every band's warm-up passes the bottom wall or the lid), ragged last bands, one band
    for the whole grid; odd bands walk upward."""
    try:
        ops.set_pressure_band(band)
        for H, W in ((37, 128), (130, 260), (11, 512)):
            p0, b, prm = _inputs(H, W, seed=3 * H + band)
            dp, db = to_dev(p0), to_dev(b)
            for nit, levels in ((5, 5), (16, 8), (7, 3), (1, 1), (12, 12), (20, 10), (9, 9), (22, 11)):
                say(f"pressure band={band} {H}x{W} nit={nit} levels={levels}")
                got = to_host(ops.cavity_pressure(dp, db, nit, prm.cw, prm.cn, prm.cb, levels=levels))
                assert np.array_equal(got, _want(p0, b, prm, nit)), (band, H, W, nit, levels)
    finally:
        ops.set_pressure_band(0)


def test_pressure_fifty_iterations(ops):
    """The cavity flow's 50 iterations per time step, on a 1024 x 1024 grid."""
    H = W = 1024
    p0, b, prm = _inputs(H, W, seed=9)
    say("pressure 1024x1024 nit=50")
    got = to_host(ops.cavity_pressure(to_dev(p0), to_dev(b), 50, prm.cw, prm.cn, prm.cb))
    assert np.array_equal(got, _want(p0, b, prm, 50))


def test_pressure_full_size(ops):
    H = W = 4096
    p0, b, prm = _inputs(H, W, seed=21)
    say("pressure 4096x4096 nit=9")
    got = to_host(ops.cavity_pressure(to_dev(p0), to_dev(b), 9, prm.cw, prm.cn, prm.cb))
    assert np.array_equal(got, _want(p0, b, prm, 9))


def test_pressure_strided_view(ops):
    """Views with a row stride wider than the grid (the padding is neither read nor written)."""
    import torch

    H, W = 70, 256
    p0, b, prm = _inputs(H, W, seed=4)
    big_p = torch.full((H, W + 64), float("nan"), dtype=torch.float64, device="cuda")
    big_b = torch.full((H, W + 64), float("nan"), dtype=torch.float64, device="cuda")
    big_o = torch.full((H, W + 64), 7.0, dtype=torch.float64, device="cuda")
    big_w = torch.full((H, W + 64), 7.0, dtype=torch.float64, device="cuda")
    big_p[:, 32:32 + W] = to_dev(p0)
    big_b[:, 32:32 + W] = to_dev(b)
    say("pressure strided view")
    ops.cavity_pressure(big_p[:, 32:32 + W], big_b[:, 32:32 + W], 12, prm.cw, prm.cn, prm.cb, levels=5,
                        out=big_o[:, 32:32 + W], work=big_w[:, 32:32 + W])
    got = to_host(big_o)
    assert np.array_equal(got[:, 32:32 + W], _want(p0, b, prm, 12))
    assert (got[:, :32] == 7.0).all() and (got[:, 32 + W:] == 7.0).all()


def test_pressure_unsupported_layouts(ops):
    from paper_2512_19851_amd import _lib

    for H, W in ((2, 128), (10, 127), (10, 100)):
        d = to_dev(np.zeros((H, W)))
        with pytest.raises(_lib.StenError) as e:
            ops.cavity_pressure(d, d.clone(), 3, 0.25, 0.25, 0.1)
        assert e.value.name == "STEN_ERR_UNSUPPORTED"


def test_pressure_beyond_int32_points(ops):
    """46400 x 46400 (2.15e9 points, past 2^31; four 17.2 GB buffers): 9 iterations as one pass (the
    LDS-ring kernel) and as two passes of 5 and 4 (the register-ring kernel, through the work buffer),
    sampled outputs bit-exact with the oracle. A window reaching nit + 1 beyond a point (clamped to the
    real walls) gives that point exactly: each iteration, and each wall rule, reads only distance 1."""
    import torch

    from tests.gpu_util import cone_window, sample_points
    from workloads import hashed_grid, hashed_rows_torch

    n, nit = 46400, 9
    prm = oc.CavityParams(n, n, lx=2.0, ly=1.3)
    dev = device()
    say(f"pressure beyond int32: fill {n}x{n}")
    p0 = torch.empty((n, n), dtype=torch.float64, device=dev)
    b = torch.empty((n, n), dtype=torch.float64, device=dev)
    for r0 in range(0, n, 2048):
        r1 = min(n, r0 + 2048)
        p0[r0:r1] = hashed_rows_torch(r0, r1, n, dev, seed=21)
        b[r0:r1] = hashed_rows_torch(r0, r1, n, dev, seed=22)
    pts = sample_points(n, n, 24, seed=3) + [(n - 1, 7), (n - 2, n - 1), (0, n - 1), (46341, 0), (46341, 46341)]
    flat = torch.tensor([i * n + j for i, j in pts], dtype=torch.int64, device=dev)
    vals = {}
    for levels in (0, 5):
        say(f"pressure beyond int32: nit={nit} levels={levels}")
        got = ops.cavity_pressure(p0, b, nit, prm.cw, prm.cn, prm.cb, levels=levels)
        vals[levels] = to_host(got.view(-1)[flat])
        del got
        torch.cuda.empty_cache()
    del p0, b
    torch.cuda.empty_cache()
    for k, (i, j) in enumerate(pts):
        r0, r1, c0, c1 = cone_window(n, n, i, j, nit)
        want = _want(hashed_grid(r0, r1 + 1, c0, c1 + 1, seed=21), hashed_grid(r0, r1 + 1, c0, c1 + 1, seed=22),
                     prm, nit)
        for levels, v in vals.items():
            assert v[k] == want[i - r0, j - c0], f"point {(i, j)} levels={levels}"


@pytest.mark.parametrize("nit,levels", [(20, 0), (25, 0), (17, 8)], ids=["lds-ring", "mixed", "register-ring"])
def test_pressure_graph_replays(ops, nit, levels):
    """The blocked pressure call (lid fill kernel + passes, no allocation, no memset) captured in a HIP graph:
    every replay, with eager work on the output and the work buffer between replays, gives the oracle's bits.
    Passes: 20 iterations at the default are 10 + 10 (LDS ring); 25 are 9 (LDS ring) + 8 + 8 (register
    ring); 17 at 8 levels are 6 + 6 + 5 (register ring)."""
    import torch

    H, W = 300, 516
    p0, b, prm = _inputs(H, W, seed=33)
    want = _want(p0, b, prm, nit)
    dp, db = to_dev(p0), to_dev(b)
    out = torch.empty_like(dp)
    work = torch.empty_like(dp)
    g = torch.cuda.CUDAGraph()
    s = torch.cuda.Stream()
    say(f"graph capture of the pressure call {H}x{W} nit={nit} levels={levels}")
    with torch.cuda.graph(g, stream=s):
        ops.cavity_pressure(dp, db, nit, prm.cw, prm.cn, prm.cb, levels=levels, out=out, work=work)
    for r in range(4):
        out.fill_(float("nan"))
        work.fill_(float("nan"))
        g.replay()
        assert np.array_equal(to_host(out), want), r
