"""Host checks of the seeded input generators (no GPU, no method arithmetic)."""

import numpy as np

import workloads as w


def test_hashed_grid_host_and_torch_agree():
    """Any window rebuilt on the host equals the same rows filled block by block with torch."""
    torch_rows = w.hashed_rows_torch(46390, 46400, 46400, "cpu", seed=5).numpy()
    assert np.array_equal(w.hashed_grid(46390, 46400, 46370, 46400, seed=5), torch_rows[:, 46370:])
    assert np.array_equal(w.hashed_grid(0, 7, 0, 9), w.hashed_rows_torch(0, 7, 9, "cpu").numpy())


def test_hashed_grid_values():
    g = w.hashed_grid(0, 256, 0, 256, seed=1)
    assert g.dtype == np.float64 and g.min() >= -1.0 and g.max() < 1.0
    assert abs(g.mean()) < 0.02 and 0.3 < g.std() < 0.65  # uniform on [-1, 1): std 0.577
    assert len(np.unique(g)) > 0.99 * g.size
    assert not np.array_equal(g, w.hashed_grid(0, 256, 0, 256, seed=2))
