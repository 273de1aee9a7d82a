"""The C + OpenMP twin of the oracle is bit-identical to the NumPy oracle."""

import numpy as np
import pytest

import oracle
from oracle import cref
from workloads import normal_grid


@pytest.mark.parametrize("dtype", [np.float64, np.float32])
@pytest.mark.parametrize("shape,T", [((64, 64), 10), ((37, 129), 3), ((3, 3), 5), ((2, 9), 4), ((200, 150), 7)])
def test_cref_matches_numpy(dtype, shape, T):
    u0 = normal_grid(*shape, seed=5, dtype=dtype)
    want = oracle.jacobi5(u0, T, 0.25, dtype=dtype)
    for nt in (1, 3):
        got = cref.jacobi5(u0, T, 0.25, nthreads=nt)
        assert got.dtype == dtype
        assert np.array_equal(got, want)


def test_cref_general_c():
    u0 = normal_grid(33, 47, seed=6)
    assert np.array_equal(cref.jacobi5(u0, 6, 0.3), oracle.jacobi5(u0, 6, 0.3))


def test_cref_threads():
    assert cref.threads(2) == 2
