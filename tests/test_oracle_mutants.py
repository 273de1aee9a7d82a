"""Plausible mistakes planted in copies of the oracle must fail at least one pin.

This shows the pins constrain every term, index and operand of the sweep and of
its transpose. The mutants live only here, on the CPU.
"""

import numpy as np
import pytest

import oracle
from tests import pins


def make_j5(rhs):
    """A forward solver with the same ping-pong as the oracle and a planted right side."""

    def j5(u0, T, c):
        a = np.array(u0, dtype=np.float64, copy=True)
        b = a.copy()
        for _ in range(T):
            if a.shape[0] >= 3 and a.shape[1] >= 3:
                b[1:-1, 1:-1] = rhs(a, c)
            a, b = b, a
        return a

    return j5


FORWARD_MUTANTS = {
    "dropped_east": lambda A, c: c * (A[:-2, 1:-1] + A[2:, 1:-1] + A[1:-1, :-2]),
    "north_twice": lambda A, c: c * (A[:-2, 1:-1] + A[:-2, 1:-1] + A[1:-1, :-2] + A[1:-1, 2:]),
    "south_off_by_one": lambda A, c: c * (A[:-2, 1:-1] + A[1:-1, 1:-1] + A[1:-1, :-2] + A[1:-1, 2:]),
    "west_uses_center": lambda A, c: c * (A[:-2, 1:-1] + A[2:, 1:-1] + A[1:-1, 1:-1] + A[1:-1, 2:]),
    "sign_flip": lambda A, c: c * (A[:-2, 1:-1] - A[2:, 1:-1] + A[1:-1, :-2] + A[1:-1, 2:]),
    "coef_third": lambda A, c: (c * 4 / 3) * (A[:-2, 1:-1] + A[2:, 1:-1] + A[1:-1, :-2] + A[1:-1, 2:]) / 4 * 3 / 3,
    "diagonal_neighbor": lambda A, c: c * (A[:-2, :-2] + A[2:, 1:-1] + A[1:-1, :-2] + A[1:-1, 2:]),
    "reassociated_sum": lambda A, c: c * ((A[:-2, 1:-1] + A[1:-1, 2:]) + (A[2:, 1:-1] + A[1:-1, :-2])),
    "fused_scale": lambda A, c: c * A[:-2, 1:-1] + c * A[2:, 1:-1] + c * A[1:-1, :-2] + c * A[1:-1, 2:],
}


def transposed_j5(u0, T, c):
    """Operand transposed: runs the method on u0.T and transposes back."""
    return oracle.jacobi5(np.asarray(u0).T, T, c).T.copy()


def in_place_j5(u0, T, c):
    """Single-buffer update (reads values already overwritten in this sweep)."""
    a = np.array(u0, dtype=np.float64, copy=True)
    H, W = a.shape
    for _ in range(T):
        for i in range(1, H - 1):
            for j in range(1, W - 1):
                a[i, j] = c * (((a[i - 1, j] + a[i + 1, j]) + a[i, j - 1]) + a[i, j + 1])
    return a


def ring_zeroed_j5(u0, T, c):
    """Second buffer starts with a zero ring instead of u0's ring."""
    a = np.array(u0, dtype=np.float64, copy=True)
    b = np.zeros_like(a)
    for _ in range(T):
        oracle.sweep(a, b, c)
        a, b = b, a
    return a


def _fails_some_pin(j5, pin_list):
    for pin in pin_list:
        try:
            pin(j5)
        except AssertionError:
            return pin.__name__
        except Exception:  # a crash on a broken copy also counts as caught
            return pin.__name__
    return None


@pytest.mark.parametrize("name", sorted(FORWARD_MUTANTS))
def test_forward_mutant_is_caught(name):
    j5 = make_j5(FORWARD_MUTANTS[name])
    assert _fails_some_pin(j5, pins.FORWARD_PINS) is not None, f"mutant {name} passed every pin"


@pytest.mark.parametrize("j5", [transposed_j5, in_place_j5, ring_zeroed_j5],
                         ids=["transposed", "in_place", "ring_zeroed"])
def test_forward_structural_mutant_is_caught(j5):
    assert _fails_some_pin(j5, pins.FORWARD_PINS) is not None


def _adj_from(scatter):
    def adj(w, T, c):
        g = np.array(w, dtype=np.float64, copy=True)
        for _ in range(T):
            g = scatter(g, c)
        return g

    return adj


def _scatter(g, c, skip=None, ring_identity=True, swap_ns=False):
    H, W = g.shape
    out = g.copy() if ring_identity else np.zeros_like(g)
    if H < 3 or W < 3:
        return g.copy()
    gi = g[1:-1, 1:-1].copy()
    out[1:-1, 1:-1] = 0.0
    dirs = {"n": np.s_[:-2, 1:-1], "s": np.s_[2:, 1:-1], "w": np.s_[1:-1, :-2], "e": np.s_[1:-1, 2:]}
    for k, sl in dirs.items():
        if k == skip:
            continue
        out[sl] += c * gi
    if swap_ns:
        out[1:-1, 1:-1] += g[1:-1, 1:-1]
    return out


ADJOINT_MUTANTS = {
    "adj_dropped_south": _adj_from(lambda g, c: _scatter(g, c, skip="s")),
    "adj_no_ring_identity": _adj_from(lambda g, c: _scatter(g, c, ring_identity=False)),
    "adj_keeps_interior": _adj_from(lambda g, c: _scatter(g, c, swap_ns=True)),
    "adj_is_forward": lambda w, T, c: oracle.jacobi5(w, T, c),
}


@pytest.mark.parametrize("name", sorted(ADJOINT_MUTANTS))
def test_adjoint_mutant_is_caught(name):
    adj = ADJOINT_MUTANTS[name]
    j5 = lambda u0, T, c: oracle.jacobi5(u0, T, c)  # noqa: E731
    caught = False
    for pin in pins.ADJOINT_PINS:
        try:
            pin(adj, j5)
        except AssertionError:
            caught = True
            break
    assert caught, f"adjoint mutant {name} passed every pin"
