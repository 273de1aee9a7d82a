"""Pins for the general star-stencil oracle (CPU)."""

from fractions import Fraction

import numpy as np
import pytest

import oracle
from oracle.star import StarCoef, star_apply, star_iterate, star_lambda


def brute(A, coef: StarCoef):
    """Exact rational evaluation with plain loops (small grids, dyadic data)."""
    H, W = len(A), len(A[0])
    R = coef.R
    out = [[Fraction(v) for v in row] for row in A]
    for i in range(R, H - R):
        for j in range(R, W - R):
            s = Fraction(coef.c0) * Fraction(A[i][j])
            for k in range(1, R + 1):
                s += Fraction(coef.cn[k - 1]) * Fraction(A[i - k][j])
                s += Fraction(coef.cs[k - 1]) * Fraction(A[i + k][j])
                s += Fraction(coef.cw[k - 1]) * Fraction(A[i][j - k])
                s += Fraction(coef.ce[k - 1]) * Fraction(A[i][j + k])
            out[i][j] = s
    return np.array([[float(v) for v in row] for row in out])


COEFS = [
    StarCoef(0.5, [0.125], [0.25], [-0.5], [1.0]),
    StarCoef(-1.0, [0.5, -0.125], [0.25, 0.0625], [1.0, 2.0], [-0.25, 0.5]),
    StarCoef(0.25, [0.5, 0.25, -0.125], [0.125, -1.0, 0.5], [2.0, 0.25, 0.75], [-0.5, 0.375, 1.5]),
    StarCoef(1.0, [0.5, 0.25, 0.125, 0.0625], [0.5, 0.25, 0.125, 0.0625], [1.0, -0.5, 0.25, -0.125],
             [1.0, -0.5, 0.25, -0.125]),
]


@pytest.mark.parametrize("coef", COEFS, ids=lambda c: f"R{c.R}")
def test_star_fraction_bruteforce(coef):
    """Small dyadic data and coefficients: every FP64 operation is exact."""
    rng = np.random.default_rng(coef.R)
    A = rng.integers(-32, 33, (2 * coef.R + 5, 2 * coef.R + 7)).astype(np.float64) / 4
    assert np.array_equal(star_apply(A, coef), brute(A.tolist(), coef))


def test_star_radius1_equals_jacobi_on_exact_data():
    """c*N + c*S + c*W + c*E equals c*(N+S+W+E) when every operation is exact."""
    rng = np.random.default_rng(0)
    A = rng.integers(-100, 101, (20, 30)).astype(np.float64)
    assert np.array_equal(star_iterate(A, 3, StarCoef.jacobi()), oracle.jacobi5(A, 3))


@pytest.mark.parametrize("R", [1, 2, 3, 4])
def test_star_sine_mode(R):
    """Symmetric coefficients: one application maps sin(ai)sin(bj) to lambda times itself."""
    cn = [0.3 / k for k in range(1, R + 1)]
    cw = [0.2 / (k * k) for k in range(1, R + 1)]
    coef = StarCoef(-0.7, cn, cn, cw, cw)
    H, W, p, q = 40, 29, 3, 2
    a, b = p * np.pi / (H - 1), q * np.pi / (W - 1)
    i = np.arange(H)[:, None]
    j = np.arange(W)[None, :]
    u = np.sin(a * i) * np.sin(b * j)
    y = star_apply(u, coef)
    lam = star_lambda(coef, a, b)
    assert np.max(np.abs(y[R:-R, R:-R] - lam * u[R:-R, R:-R])) < 1e-14
    assert np.array_equal(y[:R], u[:R]) and np.array_equal(y[:, -R:], u[:, -R:])


def test_star_linear_functions():
    """Symmetric coefficients with sum s map a linear function f to s*f exactly (small integers)."""
    coef = StarCoef(0.5, [0.25, 0.125], [0.25, 0.125], [0.5, -0.25], [0.5, -0.25])
    s = coef.c0 + 2 * sum(coef.cn) + 2 * sum(coef.cw)
    i = np.arange(15, dtype=np.float64)[:, None]
    j = np.arange(17, dtype=np.float64)[None, :]
    f = 3 + 2 * i - 5 * j
    y = star_apply(f, coef)
    assert np.array_equal(y[2:-2, 2:-2], s * f[2:-2, 2:-2])


def test_star_small_grid_untouched():
    A = np.arange(12.0).reshape(3, 4)
    assert np.array_equal(star_apply(A, COEFS[1]), A)  # R = 2 needs at least 5 x 5


ORDER_CASE = {
    # Hand-derived (FP64, round to nearest even): radius 1, all coefficients 1;
    # centre 1, N = 2^-53, S = 2^-53, W = -1, E = 0. Left to right:
    # 1*1 = 1; 1 + 2^-53 ties to 1; again 1; 1 + (-1) = 0; 0 + 0 = 0.
    # Summing N and S first would give 2^-52 instead.
    "grid": [[0.0, 2.0 ** -53, 0.0], [-1.0, 1.0, 0.0], [0.0, 2.0 ** -53, 0.0]],
    "centre": 0.0,
}


def test_star_left_to_right_order():
    coef = StarCoef(1.0, [1.0], [1.0], [1.0], [1.0])
    y = star_apply(np.array(ORDER_CASE["grid"]), coef)
    assert y[1, 1] == ORDER_CASE["centre"]


@pytest.mark.parametrize("mutant", ["swap_ns", "drop_center", "shift_far", "fuse_order"])
def test_star_mutants_caught(mutant):
    """Planted mistakes in a copy of the oracle fail the brute-force or sine-mode pins."""
    coef = COEFS[1]

    def bad_apply(A):
        A = np.asarray(A, dtype=np.float64)
        out = A.copy()
        R, (H, W) = coef.R, A.shape

        def sl(di, dj):
            return A[R + di:H - R + di, R + dj:W - R + dj]

        acc = (0.0 if mutant == "drop_center" else coef.c0) * sl(0, 0)
        for k in range(1, R + 1):
            kn = k + 1 if (mutant == "shift_far" and k == R - 1) else k
            n, s_ = (sl(k, 0), sl(-k, 0)) if mutant == "swap_ns" else (sl(-kn, 0), sl(k, 0))
            if mutant == "fuse_order":
                acc = acc + (coef.cn[k - 1] * n + coef.cs[k - 1] * s_)
            else:
                acc = acc + coef.cn[k - 1] * n
                acc = acc + coef.cs[k - 1] * s_
            acc = acc + coef.cw[k - 1] * sl(0, -k)
            acc = acc + coef.ce[k - 1] * sl(0, k)
        out[R:H - R, R:W - R] = acc
        return out

    rng = np.random.default_rng(9)
    A = rng.integers(-32, 33, (11, 13)).astype(np.float64) / 4
    exact = brute(A.tolist(), coef)
    caught = not np.array_equal(bad_apply(A), exact)
    if not caught:  # rounding-order mutants show on the hand-derived order case
        coef = StarCoef(1.0, [1.0, 0.0], [1.0, 0.0], [1.0, 0.0], [1.0, 0.0])
        g = np.zeros((5, 5))
        g[1:4, 1:4] = ORDER_CASE["grid"]
        caught = bad_apply(g)[2, 2] != ORDER_CASE["centre"]
    assert caught
