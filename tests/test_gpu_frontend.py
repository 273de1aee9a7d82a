"""The lazy frontend running on libsten kernels, against the CPU oracle (bit-exact)."""

import numpy as np
import pytest

import oracle
from oracle.star import StarCoef, star_apply
from tests.gpu_util import device, say, to_host
from workloads import unit_ring_grid

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def fe():
    device()
    from paper_2512_19851_amd import frontend

    return frontend


@pytest.mark.parametrize("shape,T,depth", [((5, 5), 3, 1), ((64, 64), 10, 4), ((300, 517), 25, 64),
                                           ((1000, 1000), 40, 1000)])
def test_listing_program(fe, shape, T, depth):
    """The listing of the Laplace solver (Section III-A), written as in the paper."""
    ctx = fe.Context(max_depth=depth)
    H, W = shape
    u1 = ctx.create_array((H, W))
    u2 = ctx.create_array((H, W))
    u1[0, :] = u1[-1, :] = u1[:, 0] = u1[:, -1] = 1
    u2[0, :] = u2[-1, :] = u2[:, 0] = u2[:, -1] = 1
    for _ in range(T):
        u2[1:-1, 1:-1] = 0.25 * (u1[:-2, 1:-1] + u1[2:, 1:-1] + u1[1:-1, :-2] + u1[1:-1, 2:])
        u1, u2 = u2, u1
    say(f"frontend listing {shape} T={T} depth={depth}")
    got = to_host(u1.tensor())
    assert np.array_equal(got, oracle.jacobi5(unit_ring_grid(H, W), T))
    assert ctx.distinct_asts() == 2


def test_sub_rectangle_sweep(fe):
    ctx = fe.Context()
    a = ctx.create_array((40, 50))
    b = ctx.create_array((40, 50))
    a[:, :] = 1.0
    a[10:20, 5:45] = 3.0
    b[5:30, 7:41] = 0.3 * (a[4:29, 7:41] + a[6:31, 7:41] + a[5:30, 6:40] + a[5:30, 8:42])
    say("frontend sub-rectangle")
    got = to_host(b.tensor())
    ref_a = np.ones((40, 50))
    ref_a[10:20, 5:45] = 3.0
    want = np.zeros((40, 50))
    want[5:30, 7:41] = 0.3 * (ref_a[4:29, 7:41] + ref_a[6:31, 7:41] + ref_a[5:30, 6:40] + ref_a[5:30, 8:42])
    assert np.array_equal(got, want)


def test_fused_star_program(fe):
    ctx = fe.Context()
    rng = np.random.default_rng(0)
    vals = rng.standard_normal((33, 47))
    a = ctx.create_array((33, 47))
    # load values through fills of single points would be slow; set rows with fills of constants instead
    for i in range(33):
        a[i, :] = float(vals[i, 0])
    b = ctx.create_array((33, 47))
    c = ctx.create_array((33, 47))
    k1 = StarCoef(0.5, [0.25, 0.125], [0.25, -0.5], [1.5, 0.75], [-0.25, 2.0])
    k2 = StarCoef(-1.0, [0.3, 0.2], [0.1, 0.9], [0.7, 0.6], [0.5, 0.4])

    def star(x, k):
        e = k.c0 * x[2:-2, 2:-2]
        for d in (1, 2):
            e = e + k.cn[d - 1] * x[2 - d:-2 - d, 2:-2]
            e = e + k.cs[d - 1] * x[2 + d:(-2 + d) or None, 2:-2]
            e = e + k.cw[d - 1] * x[2:-2, 2 - d:-2 - d]
            e = e + k.ce[d - 1] * x[2:-2, 2 + d:(-2 + d) or None]
        return e

    b[2:-2, 2:-2] = star(a, k1)
    c[2:-2, 2:-2] = star(a, k2)
    say("frontend fused star")
    gb, gc = to_host(b.tensor()), to_host(c.tensor())
    assert ctx.stats["fused_nodes"] == 2
    ref = np.repeat(vals[:, :1], 47, axis=1)
    zb = star_apply(ref, k1)
    zc = star_apply(ref, k2)
    # outputs start as zeros outside the assigned region
    wb = np.zeros((33, 47))
    wb[2:-2, 2:-2] = zb[2:-2, 2:-2]
    wc = np.zeros((33, 47))
    wc[2:-2, 2:-2] = zc[2:-2, 2:-2]
    assert np.array_equal(gb, wb) and np.array_equal(gc, wc)


def test_in_place_rejected_on_gpu(fe):
    ctx = fe.Context()
    a = ctx.create_array((8, 8))
    with pytest.raises(fe.InPlaceDependencyError):
        a[1:-1, 1:-1] = 0.25 * (a[:-2, 1:-1] + a[2:, 1:-1] + a[1:-1, :-2] + a[1:-1, 2:])


@pytest.mark.parametrize("shape,T,depth", [((64, 64), 25, 1000), ((300, 517), 23, 7), ((257, 1030), 31, 1000),
                                           ((3, 130), 5, 1000), ((1000, 1000), 40, 12), ((512, 1024), 50, 10),
                                           ((130, 256), 33, 3)])
def test_listing_chains_keep_both_arrays(fe, shape, T, depth):
    """The listing's Jacobi nodes run as chains of blocked launches; both arrays end as after one node at a
    time (iterate T and iterate T-1)."""
    ctx = fe.Context(max_depth=depth)
    H, W = shape
    u1 = ctx.create_array((H, W))
    u2 = ctx.create_array((H, W))
    u1[0, :] = u1[-1, :] = u1[:, 0] = u1[:, -1] = 1
    u2[0, :] = u2[-1, :] = u2[:, 0] = u2[:, -1] = 1
    for _ in range(T):
        u2[1:-1, 1:-1] = 0.25 * (u1[:-2, 1:-1] + u1[2:, 1:-1] + u1[1:-1, :-2] + u1[1:-1, 2:])
        u1, u2 = u2, u1
    say(f"frontend chains {shape} T={T} depth={depth}")
    ptrs = {u1.data.data_ptr(), u2.data.data_ptr()}
    ctx.sync()
    assert ctx.stats["chained_nodes"] > 0 or H < 3
    assert {u1.data.data_ptr(), u2.data.data_ptr()} == ptrs  # buffers may be exchanged, never replaced
    if depth in (3, 10, 12):  # flushes caused by the next Jacobi node: chains that keep only iterate m
        assert ctx.stats["chains_last_only"] > 0
    u0 = unit_ring_grid(H, W)
    assert np.array_equal(to_host(u1.tensor()), oracle.jacobi5(u0, T))
    assert np.array_equal(to_host(u2.tensor()), oracle.jacobi5(u0, T - 1))


@pytest.mark.parametrize("schedule", [0, 1, 2, 3, 12])
def test_sweep_chain_abi(schedule):
    """sten_sweep_chain_f64 on two arrays with equal rings, random interiors, every chain length 0..24 and
    the schedule's levels; odd widths take single sweeps."""
    import torch

    device()
    from paper_2512_19851_amd import _lib, ops

    try:
        ops.set_schedule(schedule)
        for H, W in ((5, 7), (64, 66), (130, 257), (41, 512)):
            a0 = np.random.default_rng(H * W + schedule).standard_normal((H, W))
            b0 = np.random.default_rng(H + W).standard_normal((H, W))
            b0[0, :], b0[-1, :], b0[:, 0], b0[:, -1] = a0[0, :], a0[-1, :], a0[:, 0], a0[:, -1]
            states = [a0]
            for _ in range(24):
                states.append(oracle.jacobi5(states[-1], 1))
            for m in range(0, 25):
                say(f"chain abi schedule={schedule} {H}x{W} m={m}")
                a = torch.from_numpy(a0.copy()).cuda()
                b = torch.from_numpy(b0.copy()).cuda()
                _lib.call("sten_sweep_chain_f64", a.data_ptr(), b.data_ptr(), H, W, W, m, 0.25,
                          torch.cuda.current_stream().cuda_stream)
                last, other = (b, a) if m % 2 else (a, b)
                if m == 0:
                    assert np.array_equal(to_host(a), a0) and np.array_equal(to_host(b), b0)
                    continue
                assert np.array_equal(to_host(last), states[m]), (schedule, H, W, m)
                assert np.array_equal(to_host(other), states[m - 1]), (schedule, H, W, m)
    finally:
        ops.set_schedule(0)


@pytest.mark.parametrize("schedule", [0, 1, 2, 12])
def test_sweep_chain_last_abi(schedule):
    """sten_sweep_chain_last_f64: iterate m, bit for bit, in the array the call reports (the one the fewest
    blocked launches end in: b after an odd number of them), for every chain length 0..26; both rings
    untouched; the other array's interior is free."""
    import ctypes

    import torch

    device()
    from paper_2512_19851_amd import _lib, ops

    try:
        ops.set_schedule(schedule)
        for H, W in ((5, 7), (64, 66), (130, 257), (41, 512), (300, 1024)):
            a0 = np.random.default_rng(H * W + schedule + 1).standard_normal((H, W))
            b0 = np.random.default_rng(H + W + 1).standard_normal((H, W))
            b0[0, :], b0[-1, :], b0[:, 0], b0[:, -1] = a0[0, :], a0[-1, :], a0[:, 0], a0[:, -1]
            states = [a0]
            for _ in range(26):
                states.append(oracle.jacobi5(states[-1], 1))
            ring = np.ones((H, W), dtype=bool)
            ring[1:-1, 1:-1] = False
            lands = set()
            for m in range(0, 27):
                say(f"chain-last abi schedule={schedule} {H}x{W} m={m}")
                a = torch.from_numpy(a0.copy()).cuda()
                b = torch.from_numpy(b0.copy()).cuda()
                in_b = ctypes.c_int32(-1)
                _lib.call("sten_sweep_chain_last_f64", a.data_ptr(), b.data_ptr(), H, W, W, m, 0.25,
                          ctypes.byref(in_b), torch.cuda.current_stream().cuda_stream)
                assert in_b.value in (0, 1)
                if m == 0:
                    assert in_b.value == 0
                    assert np.array_equal(to_host(a), a0) and np.array_equal(to_host(b), b0)
                    continue
                last, other = (b, a) if in_b.value else (a, b)
                lands.add((m % 2, in_b.value))
                assert np.array_equal(to_host(last), states[m]), (schedule, H, W, m)
                assert np.array_equal(to_host(other)[ring], a0[ring]), (schedule, H, W, m)
            if schedule != 1 and min(H, W) >= 64 and W % 2 == 0:
                assert (0, 1) in lands  # an even chain in one blocked launch ends in b
    finally:
        ops.set_schedule(0)
