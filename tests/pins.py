"""Pins for the forward and adjoint oracle: checks fixed by the paper or by mathematics.

Each pin takes the implementation under test as a callable, so the same checks
run on the oracle (where they must pass) and on deliberately broken copies of
it (where at least one must fail). None of them re-derives its expected value
by calling the oracle on the same input.

Forward callable signature: ``j5(u0, T, c) -> ndarray`` (FP64).
Adjoint callable signature: ``adj(w, T, c) -> ndarray`` (FP64).
"""

from __future__ import annotations

import math
import os
from fractions import Fraction

import numpy as np

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def read_golden(name: str):
    """Parse a worked-example fixture: returns (c, [grid_0, grid_1, ...])."""
    c = None
    grids = []
    cur = None
    H = W = None
    with open(os.path.join(GOLDEN, name)) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            parts = line.split()
            if parts[0] == "shape":
                H, W = int(parts[1]), int(parts[2])
            elif parts[0] == "c":
                c = float(parts[1])
            elif parts[0] == "grid":
                cur = []
                grids.append(cur)
            else:
                cur.append([float(v) for v in parts])
    out = [np.array(g, dtype=np.float64) for g in grids]
    for g in out:
        assert g.shape == (H, W)
    return c, out


# ---------------------------------------------------------------------------
# Forward pins
# ---------------------------------------------------------------------------

def pin_golden(j5) -> None:
    """Hand-derived worked examples (listing of the Laplace solver, Section III-A).

    Two of them fix the rounding order: the left-to-right sum and the single
    multiplication by c of the listing's expression.
    """
    for name in ("worked_example_5x5.txt", "worked_example_3x4.txt",
                 "order_c025_3x3.txt", "order_c3_3x3.txt"):
        c, grids = read_golden(name)
        for T in range(len(grids)):
            got = j5(grids[0], T, c)
            assert np.array_equal(got, grids[T]), f"{name}: sweep {T} differs"


def brute_fraction(u0, T: int, c: Fraction):
    """Exact rational evaluation of T sweeps with plain loops (tiny grids only)."""
    H = len(u0)
    W = len(u0[0])
    a = [[Fraction(v) for v in row] for row in u0]
    for _ in range(T):
        b = [row[:] for row in a]
        for i in range(1, H - 1):
            for j in range(1, W - 1):
                b[i][j] = c * (a[i - 1][j] + a[i + 1][j] + a[i][j - 1] + a[i][j + 1])
        a = b
    return a


def pin_fraction(j5, seed: int = 1) -> None:
    """Exact rational arithmetic on small dyadic grids: every FP64 op is exact there."""
    rng = np.random.default_rng(seed)
    for H, W in [(3, 3), (3, 5), (4, 7), (6, 5), (8, 8)]:
        u0 = rng.integers(-64, 65, (H, W)).astype(np.float64) / 8.0
        for T in range(0, 7):
            exact = brute_fraction(u0.tolist(), T, Fraction(1, 4))
            got = j5(u0, T, 0.25)
            want = np.array([[float(v) for v in row] for row in exact])
            assert np.array_equal(got, want), f"fraction pin {H}x{W} T={T}"


def pin_eigen(j5) -> None:
    """Closed form: discrete sine modes with a zero ring decay by a fixed factor.

    With u0[i,j] = sin(p pi i/(H-1)) sin(q pi j/(W-1)) and a zero ring, one sweep
    maps u to lam*u with lam = 2c (cos(p pi/(H-1)) + cos(q pi/(W-1))), because
    sin(a(i-1)) + sin(a(i+1)) = 2 cos(a) sin(a i).
    """
    for H, W, p, q, c, T in [(33, 17, 3, 2, 0.25, 50), (12, 21, 1, 4, 0.25, 20),
                             (17, 9, 2, 1, 0.2, 15)]:
        i = np.arange(H)[:, None]
        j = np.arange(W)[None, :]
        u0 = np.sin(p * np.pi * i / (H - 1)) * np.sin(q * np.pi * j / (W - 1))
        u0[0, :] = u0[-1, :] = 0.0
        u0[:, 0] = u0[:, -1] = 0.0
        lam = 2 * c * (np.cos(p * np.pi / (H - 1)) + np.cos(q * np.pi / (W - 1)))
        got = j5(u0, T, c)
        want = lam ** T * u0
        assert np.max(np.abs(got - want)) <= 1e-13, f"eigen pin {H}x{W} p={p} q={q}"


def pin_harmonic(j5) -> None:
    """Invariant: discrete-harmonic grids are fixed points, bit for bit.

    u = a + b i + g j + d i j + e (i^2 - j^2) has a zero five-point Laplacian, so
    the four neighbours sum to exactly 4u; with small integers every operation
    is exact and c = 1/4 returns u unchanged.
    """
    H, W = 9, 13
    i = np.arange(H, dtype=np.float64)[:, None]
    j = np.arange(W, dtype=np.float64)[None, :]
    for a, b, g, d, e in [(3, 1, -2, 0, 0), (0, 0, 0, 1, 0), (1, 2, 3, -1, 1), (-5, 0, 7, 2, -3)]:
        u = a + b * i + g * j + d * i * j + e * (i * i - j * j)
        for T in (1, 2, 5):
            assert np.array_equal(j5(u, T, 0.25), u), f"harmonic pin {(a, b, g, d, e)} T={T}"


def pin_max_principle(j5, seed: int = 2) -> None:
    """Invariant: with c = 1/4 each sweep averages, so values stay in [min, max] exactly."""
    rng = np.random.default_rng(seed)
    u0 = rng.standard_normal((23, 31))
    prev = u0
    for T in range(1, 8):
        cur = j5(u0, T, 0.25)
        assert cur.min() >= prev.min() and cur.max() <= prev.max(), f"max principle T={T}"
        prev = cur


def pin_scaling_and_ring(j5, seed: int = 3) -> None:
    """Invariants: the ring never changes; scaling by 2^k commutes with a sweep."""
    rng = np.random.default_rng(seed)
    u0 = rng.standard_normal((14, 19))
    y = j5(u0, 4, 0.25)
    for sl in (np.s_[0, :], np.s_[-1, :], np.s_[:, 0], np.s_[:, -1]):
        assert np.array_equal(y[sl], u0[sl]), "ring changed"
    for k in (-3, 5):
        assert np.array_equal(j5(u0 * 2.0 ** k, 4, 0.25), y * 2.0 ** k), "scaling"


def laplace_dense_solution(ring: np.ndarray) -> np.ndarray:
    """Solve the 5-point Dirichlet Laplace problem by a dense linear solve.

    The interior unknowns satisfy 4 u[i,j] - sum of interior neighbours = sum of
    ring neighbours; the matrix is assembled with Kronecker products of 1-D
    second-difference matrices, independently of any sweep code.
    """
    H, W = ring.shape
    m, n = H - 2, W - 2
    Tm = 2 * np.eye(m) - np.eye(m, k=1) - np.eye(m, k=-1)
    Tn = 2 * np.eye(n) - np.eye(n, k=1) - np.eye(n, k=-1)
    A = np.kron(Tm, np.eye(n)) + np.kron(np.eye(m), Tn)
    rhs = np.zeros((m, n))
    rhs[0, :] += ring[0, 1:-1]
    rhs[-1, :] += ring[-1, 1:-1]
    rhs[:, 0] += ring[1:-1, 0]
    rhs[:, -1] += ring[1:-1, -1]
    x = np.linalg.solve(A, rhs.ravel())
    out = ring.copy()
    out[1:-1, 1:-1] = x.reshape(m, n)
    return out


def pin_dense_solve(j5, seed: int = 4) -> None:
    """Library routine: many sweeps converge to the dense solve of the Laplace problem."""
    rng = np.random.default_rng(seed)
    u0 = rng.standard_normal((10, 12))
    want = laplace_dense_solution(u0)
    got = j5(u0, 2000, 0.25)
    assert np.max(np.abs(got - want)) <= 1e-12, "dense-solve pin"


def pin_correlate(j5, seed: int = 5) -> None:
    """Library routine: one sweep's interior is a correlation with the cross kernel.

    With small-integer inputs every sum is exact, so scipy's correlate (whatever
    its summation order) must agree bit for bit.
    """
    from scipy import ndimage

    rng = np.random.default_rng(seed)
    u0 = rng.integers(-100, 101, (16, 23)).astype(np.float64)
    kern = np.array([[0, 1, 0], [1, 0, 1], [0, 1, 0]], dtype=np.float64) * 0.25
    ref = ndimage.correlate(u0, kern, mode="constant")
    got = j5(u0, 1, 0.25)
    assert np.array_equal(got[1:-1, 1:-1], ref[1:-1, 1:-1]), "correlate pin"


def pin_degenerate(j5, seed: int = 6) -> None:
    """Empty interior (fewer than 3 rows or columns) and T = 0 return the input."""
    rng = np.random.default_rng(seed)
    for shape in [(1, 1), (2, 7), (7, 2), (1, 9), (2, 2)]:
        u0 = rng.standard_normal(shape)
        assert np.array_equal(j5(u0, 3, 0.25), u0), f"degenerate {shape}"
    u0 = rng.standard_normal((6, 6))
    assert np.array_equal(j5(u0, 0, 0.25), u0), "T=0"


FORWARD_PINS = [pin_golden, pin_fraction, pin_eigen, pin_harmonic, pin_max_principle,
                pin_scaling_and_ring, pin_dense_solve, pin_correlate, pin_degenerate]


# ---------------------------------------------------------------------------
# Adjoint pins (the transpose is pinned against the forward map, which the
# forward pins above fix independently)
# ---------------------------------------------------------------------------

def pin_adjoint_dot(adj, j5, seed: int = 7) -> None:
    """Dot-product test: <J u, w> = <u, J^T w> for random u, w (FP64, exact sums)."""
    rng = np.random.default_rng(seed)
    for H, W, T in [(7, 9, 3), (16, 11, 6), (3, 3, 2), (2, 5, 2)]:
        u = rng.standard_normal((H, W))
        w = rng.standard_normal((H, W))
        lhs = math.fsum((j5(u, T, 0.25) * w).ravel())
        rhs = math.fsum((u * adj(w, T, 0.25)).ravel())
        assert abs(lhs - rhs) <= 1e-13 * (1 + abs(lhs)), f"dot test {H}x{W}"


def pin_adjoint_matrix(adj, j5) -> None:
    """Brute-force Jacobian on a 5x6 grid: the adjoint equals its transpose exactly."""
    H, W, c = 5, 6, 0.25
    n = H * W
    J = np.zeros((n, n))
    for k in range(n):
        e = np.zeros(n)
        e[k] = 1.0
        J[:, k] = j5(e.reshape(H, W), 1, c).ravel()
    # entries of one sweep are exactly 0, c or 1
    assert set(np.unique(J)).issubset({0.0, c, 1.0})
    JT = np.zeros((n, n))
    for k in range(n):
        e = np.zeros(n)
        e[k] = 1.0
        JT[:, k] = adj(e.reshape(H, W), 1, c).ravel()
    assert np.array_equal(JT, J.T), "adjoint matrix pin"


def pin_adjoint_fd(adj, j5, seed: int = 8) -> None:
    """Central finite differences of L = sum(w * J(u0)) at sampled coordinates.

    L is linear in u0, so the central difference has no truncation error; the
    sums use math.fsum so rounding stays near 1e-9 for h = 1e-6.
    """
    rng = np.random.default_rng(seed)
    H, W, T, h = 12, 10, 5, 1e-6
    u0 = rng.standard_normal((H, W))
    w = rng.standard_normal((H, W))
    g = adj(w, T, 0.25)
    for k in rng.choice(H * W, 20, replace=False):
        up = u0.copy()
        dn = u0.copy()
        up.flat[k] += h
        dn.flat[k] -= h
        fd = (math.fsum((w * j5(up, T, 0.25)).ravel()) - math.fsum((w * j5(dn, T, 0.25)).ravel())) / (2 * h)
        assert abs(fd - g.flat[k]) <= 1e-7 * (1 + abs(g.flat[k])), f"fd pin at {k}"


ADJOINT_PINS = [pin_adjoint_dot, pin_adjoint_matrix, pin_adjoint_fd]
