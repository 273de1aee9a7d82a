"""The CPU oracle against what the paper and mathematics fix (no GPU needed)."""

import math

import numpy as np
import pytest

import oracle
from tests import pins


def j5(u0, T, c):
    return oracle.jacobi5(u0, T, c)


def adj(w, T, c):
    return oracle.jacobi5_adjoint(w, T, c)


@pytest.mark.parametrize("pin", pins.FORWARD_PINS, ids=lambda p: p.__name__)
def test_forward_pin(pin):
    pin(j5)


@pytest.mark.parametrize("pin", pins.ADJOINT_PINS, ids=lambda p: p.__name__)
def test_adjoint_pin(pin):
    pin(adj, j5)


def test_unit_ring_converges_to_one():
    """The listing's initial state (unit ring) has the constant 1 as its harmonic limit."""
    from workloads import unit_ring_grid

    u = oracle.jacobi5(unit_ring_grid(7, 9), 400, 0.25)
    assert np.max(np.abs(u - 1.0)) < 1e-12


def test_states_match_forward():
    rng = np.random.default_rng(11)
    u0 = rng.standard_normal((9, 8))
    st = oracle.jacobi5_states(u0, 5)
    for k, s in enumerate(st):
        assert np.array_equal(s, oracle.jacobi5(u0, k))


def test_grad_c_complex_step():
    """dL/dc against the complex-step derivative Im L(c + i h) / h (no cancellation).

    L is a polynomial in c, hence analytic; the complex step evaluates the forward
    sweep on complex grids, which is independent of the adjoint code.
    """
    rng = np.random.default_rng(12)
    for H, W, T, c in [(9, 11, 4, 0.25), (6, 6, 7, 0.21), (3, 3, 3, 0.25)]:
        u0 = rng.standard_normal((H, W))
        w = rng.standard_normal((H, W))
        h = 1e-30
        y = oracle.jacobi5(u0.astype(np.complex128), T, complex(c, h), dtype=np.complex128)
        cs = float(np.sum(w * y).imag / h)
        g = oracle.grad_c(u0, w, T, c)
        assert abs(g - cs) <= 1e-12 * (1 + abs(cs))


def test_grad_c_empty_interior():
    u0 = np.ones((2, 5))
    assert oracle.grad_c(u0, np.ones((2, 5)), 3) == 0.0


def test_fp32_oracle_within_bound():
    """NumPy-float32 sweeps stay within the rounding-error bound of the FP64 result."""
    from workloads import normal_grid

    u0 = normal_grid(96, 80, seed=0, dtype=np.float32)
    for T, c in [(1, 0.25), (10, 0.25), (60, 0.25), (10, 0.3)]:
        y32 = oracle.jacobi5(u0, T, c, dtype=np.float32)
        y64 = oracle.jacobi5(u0.astype(np.float64), T, c)
        err = np.abs(y32.astype(np.float64) - y64)
        bound = oracle.bound_fp32(u0, T, c)
        assert np.all(err <= bound)
        assert err.max() > 0  # the comparison is not vacuous


def test_gamma():
    assert oracle.gamma(3, 2.0 ** -24) == pytest.approx(3 * 2.0 ** -24, rel=1e-6)


def test_error_report_fields():
    y = np.array([1.0, 2.0, 0.0])
    r = oracle.error_report(y + np.array([1e-12, 0, 0]), y, np.array([1.0, 2.0, 0.0]))
    assert r["normwise"] == pytest.approx(5e-13)
    assert r["componentwise"] == pytest.approx(1e-12)
    assert r["componentwise_zero_ok"]
