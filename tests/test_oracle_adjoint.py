"""The adjoint bounds of the oracle hold for an FP32 evaluation (CPU)."""

import numpy as np
import pytest

import oracle


def adjoint_step_f32(g: np.ndarray, c: float) -> np.ndarray:
    """FP32 gather form of one transposed sweep (neighbours N, S, W, E; ring adds itself)."""
    g = g.astype(np.float32)
    H, W = g.shape
    pad = np.zeros((H + 2, W + 2), np.float32)
    pad[2:-2, 2:-2] = g[1:-1, 1:-1]  # only interior points pass values to neighbours
    s = ((pad[:-2, 1:-1] + pad[2:, 1:-1]) + pad[1:-1, :-2]) + pad[1:-1, 2:]
    out = np.float32(c) * s
    ring = np.ones((H, W), bool)
    ring[1:-1, 1:-1] = False
    out[ring] = g[ring] + out[ring]
    return out


@pytest.mark.parametrize("shape,T,c", [((50, 40), 10, 0.25), ((9, 31), 25, 0.25), ((20, 20), 6, 0.3)])
def test_fp32_adjoint_within_bound(shape, T, c):
    rng = np.random.default_rng(T)
    w = rng.standard_normal(shape).astype(np.float32).astype(np.float64)
    g = w.astype(np.float32)
    for _ in range(T):
        g = adjoint_step_f32(g, c)
    ref = oracle.jacobi5_adjoint(w, T, c)
    err = np.abs(g.astype(np.float64) - ref)
    assert np.all(err <= oracle.bound_adjoint_fp32(w, T, c))
    assert err.max() > 0


def test_fp32_gather_adjoint_equals_transpose_exactly_on_dyadic():
    """With small dyadic values every FP32 operation is exact, so gather == scatter oracle."""
    rng = np.random.default_rng(3)
    w = rng.integers(-8, 9, (7, 11)).astype(np.float64)
    g = w.astype(np.float32)
    for _ in range(3):
        g = adjoint_step_f32(g, 0.25)
    assert np.array_equal(g.astype(np.float64), oracle.jacobi5_adjoint(w, 3))


def test_fp32_grad_c_within_bound():
    rng = np.random.default_rng(4)
    H, W, T, c = 24, 30, 8, 0.25
    u0 = rng.standard_normal((H, W)).astype(np.float32)
    w = rng.standard_normal((H, W)).astype(np.float32).astype(np.float64)
    states = oracle.jacobi5_states(u0, T, c, dtype=np.float32)
    lam = w.astype(np.float32)
    total = 0.0
    for k in range(T - 1, -1, -1):
        u = states[k]
        ns = ((u[:-2, 1:-1] + u[2:, 1:-1]) + u[1:-1, :-2]) + u[1:-1, 2:]
        total += float(np.sum(lam[1:-1, 1:-1].astype(np.float64) * ns.astype(np.float64)))
        lam = adjoint_step_f32(lam, c)
    ref = oracle.grad_c(u0.astype(np.float64), w, T, c)
    assert abs(total - ref) <= oracle.bound_grad_c_fp32(u0, w, T, c)
