"""GPU parity of the adjoint (reverse mode) against the CPU oracle, via the C ABI.

dL/du0 and dL/dc of L = sum(w * u_T) from the HIP adjoint are compared with
the oracle's FP64 gradient (within the FP32 error bounds), with central
finite differences in FP64 (h = 1e-6) at 64 coordinates, and with the
complex-step derivative in c.
"""

import math

import numpy as np
import pytest

import oracle
from tests.gpu_util import device, say, to_dev, to_host
from workloads import adjoint_f32, normal_grid

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ag():
    device()
    from paper_2512_19851_amd import autograd

    return autograd


def _w32(w):
    return np.asarray(w, dtype=np.float32).astype(np.float64)


@pytest.mark.parametrize("shape", [(1, 1), (2, 7), (3, 3), (5, 6), (64, 64), (37, 301), (300, 257)],
                         ids=lambda s: f"{s[0]}x{s[1]}")
def test_adjoint_within_bound(ag, shape):
    w = _w32(normal_grid(*shape, seed=sum(shape)))
    gout = to_dev(w.astype(np.float32))
    for T in (0, 1, 2, 5):
        say(f"adjoint {shape} T={T}")
        got = to_host(ag.adjoint(gout, T)).astype(np.float64)
        ref = oracle.jacobi5_adjoint(w, T)
        assert np.all(np.abs(got - ref) <= oracle.bound_adjoint_fp32(w, T)), f"{shape} T={T}"


def test_adjoint_exact_on_dyadic(ag):
    rng = np.random.default_rng(1)
    w = rng.integers(-8, 9, (40, 70)).astype(np.float64)
    say("adjoint dyadic")
    got = to_host(ag.adjoint(to_dev(w.astype(np.float32)), 3)).astype(np.float64)
    assert np.array_equal(got, oracle.jacobi5_adjoint(w, 3))


def test_dot_product_identity(ag):
    """<J u, w> == <u, J^T w> on the GPU path (FP32 rounding only)."""
    from paper_2512_19851_amd import ops

    u = normal_grid(200, 150, seed=2, dtype=np.float32)
    w = normal_grid(200, 150, seed=3, dtype=np.float32)
    T = 7
    say("dot product")
    ju = to_host(ops.jacobi5(to_dev(u), T)).astype(np.float64)
    jtw = to_host(ag.adjoint(to_dev(w), T)).astype(np.float64)
    lhs = math.fsum((ju * w).ravel())
    rhs = math.fsum((u.astype(np.float64) * jtw).ravel())
    scale = math.fsum(np.abs(oracle.jacobi5(np.abs(u), T) * np.abs(w)).ravel())
    assert abs(lhs - rhs) <= 1e-5 * scale


def test_states_match_forward(ag):
    from paper_2512_19851_amd import ops

    u0 = normal_grid(65, 130, seed=4, dtype=np.float32)
    say("forward states")
    st = to_host(ag.forward_states(to_dev(u0), 6))
    for k in range(7):
        assert np.array_equal(st[k], oracle.jacobi5(u0, k, dtype=np.float32)), f"state {k}"
        assert np.array_equal(st[k], to_host(ops.jacobi5(to_dev(u0), k)))


def _grads(ag, u0, w32, T, c, budget):
    import torch

    x = to_dev(u0).requires_grad_(True)
    cc = torch.tensor(c, dtype=torch.float32, device=x.device, requires_grad=True)
    y = ag.jacobi5_autograd(x, T, cc, mem_budget=budget)
    L = (y.double() * to_dev(w32)).sum()
    gx, gc = torch.autograd.grad(L, (x, cc))
    return to_host(gx).astype(np.float64), float(gc.item()), to_host(y)


def test_workload_gradients_vs_oracle_and_fd(ag):
    """1024x1024 FP32 u0 N(0,1), w N(0,1), T = 10, seed 0 (the adjoint workload)."""
    u0, w, coords = adjoint_f32(0)
    w32 = _w32(w)
    T, c = 10, 0.25
    say("adjoint workload autograd")
    gx, gc, y = _grads(ag, u0, w32, T, c, budget=1 << 30)
    assert np.array_equal(y, oracle.jacobi5(u0, T, dtype=np.float32))
    u64 = u0.astype(np.float64)
    g_ref = oracle.jacobi5_adjoint(w32, T, c)
    bound = oracle.bound_adjoint_fp32(w32, T, c)
    assert np.all(np.abs(gx - g_ref) <= bound)
    say(f"grad u0 max err {np.max(np.abs(gx - g_ref)):.3e}")
    # central finite differences in FP64, h = 1e-6, on each coordinate's dependence cone
    H, W = u0.shape
    h = 1e-6
    R = 2 * T + 2
    for flat in coords:
        i, j = divmod(int(flat), W)
        r0, r1, c0, c1 = max(0, i - R), min(H - 1, i + R), max(0, j - R), min(W - 1, j + R)
        sub = u64[r0:r1 + 1, c0:c1 + 1]
        wsub = w32[r0:r1 + 1, c0:c1 + 1]
        up = sub.copy()
        dn = sub.copy()
        up[i - r0, j - c0] += h
        dn[i - r0, j - c0] -= h
        # outputs within distance T of (i, j) are exact in the window (its ring is 2T+2 away)
        mask = np.zeros_like(sub, dtype=bool)
        ii, jj = np.meshgrid(np.arange(r0, r1 + 1), np.arange(c0, c1 + 1), indexing="ij")
        mask[np.abs(ii - i) + np.abs(jj - j) <= T] = True
        lp = math.fsum((wsub * oracle.jacobi5(up, T, c))[mask].ravel())
        lm = math.fsum((wsub * oracle.jacobi5(dn, T, c))[mask].ravel())
        fd = (lp - lm) / (2 * h)
        assert abs(gx[i, j] - fd) <= bound[i, j] + 1e-7, f"coord {(i, j)}: {gx[i, j]} vs fd {fd}"
        assert abs(g_ref[i, j] - fd) <= 1e-7
    # dL/dc: oracle's FP64 value within the FP32 bound; FD in c agrees with the oracle
    gc_ref = oracle.grad_c(u64, w32, T, c)
    bc = oracle.bound_grad_c_fp32(u0, w32, T, c)
    say(f"grad c {gc} ref {gc_ref} bound {bc}")
    assert abs(gc - gc_ref) <= bc + 1e-6 * abs(gc_ref)
    hc = 1e-6
    lp = math.fsum((w32 * oracle.jacobi5(u64, T, c + hc)).ravel())
    lm = math.fsum((w32 * oracle.jacobi5(u64, T, c - hc)).ravel())
    assert abs((lp - lm) / (2 * hc) - gc_ref) <= 1e-5 * abs(gc_ref)


def test_checkpointed_equals_recorded(ag):
    """A small memory budget forces checkpoint-and-recompute: same bits as recorded states."""
    u0 = normal_grid(130, 257, seed=6, dtype=np.float32)
    w32 = _w32(normal_grid(130, 257, seed=7))
    for T in (1, 5, 10, 17):
        say(f"checkpointed T={T}")
        gx_a, gc_a, _ = _grads(ag, u0, w32, T, 0.25, budget=1 << 30)
        gx_b, gc_b, _ = _grads(ag, u0, w32, T, 0.25, budget=4 * 130 * 257 * 2)
        assert np.array_equal(gx_a, gx_b) and gc_a == gc_b


def test_grad_c_small_vs_oracle(ag):
    for shape, T, c in [((9, 11), 4, 0.25), ((30, 45), 12, 0.2), ((3, 3), 3, 0.25), ((2, 6), 3, 0.25)]:
        u0 = normal_grid(*shape, seed=T, dtype=np.float32)
        w32 = _w32(normal_grid(*shape, seed=T + 1))
        say(f"grad c {shape} T={T} c={c}")
        gx, gc, _ = _grads(ag, u0, w32, T, c, budget=1 << 30)
        assert np.all(np.abs(gx - oracle.jacobi5_adjoint(w32, T, c)) <= oracle.bound_adjoint_fp32(w32, T, c))
        ref = oracle.grad_c(u0.astype(np.float64), w32, T, c)
        assert abs(gc - ref) <= oracle.bound_grad_c_fp32(u0, w32, T, c) + 1e-6 * abs(ref) + 1e-30


def test_grad_without_c(ag):
    import torch

    u0 = normal_grid(40, 50, seed=8, dtype=np.float32)
    w32 = _w32(normal_grid(40, 50, seed=9))
    x = to_dev(u0).requires_grad_(True)
    say("autograd float c")
    y = ag.jacobi5_autograd(x, 4, 0.25)
    (gx,) = torch.autograd.grad((y.double() * to_dev(w32)).sum(), (x,))
    got = to_host(gx).astype(np.float64)
    assert np.all(np.abs(got - oracle.jacobi5_adjoint(w32, 4)) <= oracle.bound_adjoint_fp32(w32, 4))


ADJ_SHAPES = [(3, 3), (4, 5), (17, 253), (40, 260), (33, 1030), (130, 301), (9, 1024), (261, 250), (100, 1024),
              (64, 772), (257, 516)]


@pytest.mark.parametrize("shape", ADJ_SHAPES, ids=lambda s: f"{s[0]}x{s[1]}")
def test_adjoint_exact_many_steps(ag, shape):
    """Small integers: every FP32 operation of up to 8 transposed steps is exact, so the result equals the
    FP64 oracle bit for bit. Shapes cross the one-step kernel's tiles (2 rows, 256 columns) and the
    several-step streaming kernel's strips and bands: widths below 256 or not a multiple of 4 (clamped,
    element-wise strips), multiples of 4 from 256 up (grid-aligned first and last strips), and grids wide
    and tall enough for unmasked interior strips and bands (100 x 1024, 64 x 772, 257 x 516)."""
    rng = np.random.default_rng(sum(shape))
    w = rng.integers(-8, 9, shape).astype(np.float64)
    g = to_dev(w.astype(np.float32))
    for T in (1, 2, 3, 4, 5, 6, 7, 8):
        say(f"adjoint exact {shape} T={T}")
        got = to_host(ag.adjoint(g, T)).astype(np.float64)
        want = oracle.jacobi5_adjoint(w, T)
        assert np.array_equal(got, want), f"{shape} T={T}: max diff {np.max(np.abs(got - want))}"


def test_adjoint_strided_views(ag):
    """Row stride ld > W, not a multiple of 4 (the element-wise loads and stores), through the C ABI."""
    import torch

    from paper_2512_19851_amd import _lib

    H, W, ld = 50, 203, 211
    rng = np.random.default_rng(11)
    w = rng.integers(-8, 9, (H, W)).astype(np.float64)
    dev = device()
    bufs = [torch.zeros((H, ld), dtype=torch.float32, device=dev) for _ in range(3)]
    bufs[0][:, :W] = to_dev(w.astype(np.float32))
    stream = torch.cuda.current_stream().cuda_stream
    for T in (1, 4, 8):
        say(f"adjoint strided T={T}")
        _lib.call("sten_jacobi5_adjoint_f32", bufs[0].data_ptr(), bufs[1].data_ptr(), bufs[2].data_ptr(), H, W, ld,
                  T, 0.25, stream)
        got = to_host(bufs[1])[:, :W].astype(np.float64)
        assert np.array_equal(got, oracle.jacobi5_adjoint(w, T)), f"T={T}"


def test_adjoint_long_chain_within_bound(ag):
    """T = 25 (five launches of the several-step kernel) on a grid with ragged tiles, within the FP32 bound."""
    w = _w32(normal_grid(97, 517, seed=12))
    say("adjoint T=25")
    got = to_host(ag.adjoint(to_dev(w.astype(np.float32)), 25)).astype(np.float64)
    ref = oracle.jacobi5_adjoint(w, 25)
    assert np.all(np.abs(got - ref) <= oracle.bound_adjoint_fp32(w, 25))


@pytest.mark.parametrize("levels", [1, 2, 3, 4, 5, 6, 7, 8])
def test_adjoint_levels_per_launch(ag, levels):
    """Every setting of transposed steps per launch gives the oracle's bits (small integers, T = 8, so every
    FP32 operation is exact), on clamped, grid-aligned and interior strips."""
    from paper_2512_19851_amd import ops

    ops.set_adjoint_levels(levels)
    try:
        for shape in [(40, 260), (100, 1024), (33, 1030), (70, 517)]:
            rng = np.random.default_rng(levels * 131 + sum(shape))
            w = rng.integers(-8, 9, shape).astype(np.float64)
            say(f"adjoint levels={levels} {shape}")
            got = to_host(ag.adjoint(to_dev(w.astype(np.float32)), 8)).astype(np.float64)
            assert np.array_equal(got, oracle.jacobi5_adjoint(w, 8)), f"levels={levels} {shape}"
    finally:
        ops.set_adjoint_levels(0)
