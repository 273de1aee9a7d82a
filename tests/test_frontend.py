"""The lazy frontend's host logic: ASTs, the in-place rule, the DAG, flushing and fusion (CPU).

A recording backend executes each node with plain NumPy slicing, so the
frontend's semantics can be checked against running the same program
eagerly in NumPy, without a GPU.
"""

import numpy as np
import pytest

from paper_2512_19851_amd import frontend as fe
from tests.numpy_backend import NumpyBackend


def listing(ctx, H, W, T):
    u1 = ctx.create_array((H, W))
    u2 = ctx.create_array((H, W))
    u1[0, :] = u1[-1, :] = u1[:, 0] = u1[:, -1] = 1
    u2[0, :] = u2[-1, :] = u2[:, 0] = u2[:, -1] = 1
    for _ in range(T):
        u2[1:-1, 1:-1] = 0.25 * (u1[:-2, 1:-1] + u1[2:, 1:-1] + u1[1:-1, :-2] + u1[1:-1, 2:])
        u1, u2 = u2, u1
    ctx.sync()
    return u1


def numpy_listing(H, W, T):
    u1 = np.zeros((H, W))
    u2 = np.zeros((H, W))
    for u in (u1, u2):
        u[0, :] = u[-1, :] = u[:, 0] = u[:, -1] = 1
    for _ in range(T):
        u2[1:-1, 1:-1] = 0.25 * (u1[:-2, 1:-1] + u1[2:, 1:-1] + u1[1:-1, :-2] + u1[1:-1, 2:])
        u1, u2 = u2, u1
    return u1


@pytest.mark.parametrize("depth", [1, 3, 7, 1000])
def test_listing_program_semantics(depth):
    be = NumpyBackend()
    ctx = fe.Context(max_depth=depth, backend=be)
    u = listing(ctx, 9, 12, 10)
    assert np.array_equal(u.data, numpy_listing(9, 12, 10))
    # the ten iterations share one parameterised AST; the eight fills share another
    assert ctx.distinct_asts() == 2
    assert ctx.stats["nodes"] == 8 + 10
    assert all(j for g in be.groups for (_, j, _) in g if "*" in g[0][0])


def test_in_place_assignment_rejected():
    ctx = fe.Context(backend=NumpyBackend())
    a = ctx.create_array((6, 6))
    with pytest.raises(fe.InPlaceDependencyError):
        a[1:-1, 1:-1] = 0.25 * (a[:-2, 1:-1] + a[2:, 1:-1] + a[1:-1, :-2] + a[1:-1, 2:])


def test_dag_depth_and_flush_policy():
    be = NumpyBackend()
    ctx = fe.Context(max_depth=4, backend=be)
    a = ctx.create_array((8, 8))
    b = ctx.create_array((8, 8))
    a[0, :] = 1        # depth 1
    b[0, :] = 2        # independent of a: depth 1
    assert ctx.depth() == 1
    b[1:-1, 1:-1] = 0.25 * (a[:-2, 1:-1] + a[2:, 1:-1] + a[1:-1, :-2] + a[1:-1, 2:])  # true dep on a, output dep on b
    assert ctx.depth() == 2
    a[1:-1, 1:-1] = 0.25 * (b[:-2, 1:-1] + b[2:, 1:-1] + b[1:-1, :-2] + b[1:-1, 2:])  # true + anti: depth 3
    assert ctx.depth() == 3 and ctx.stats["flushes"] == 0
    b[1:-1, 1:-1] = 0.25 * (a[:-2, 1:-1] + a[2:, 1:-1] + a[1:-1, :-2] + a[1:-1, 2:])  # depth 4
    b[2, 2] = 5.0  # would be depth 5 > max: the DAG is flushed first
    assert ctx.stats["flushes"] == 1 and ctx.depth() == 1
    ctx.sync()
    assert ctx.stats["flushes"] == 2


def test_fusion_of_independent_star_nodes():
    be = NumpyBackend()
    ctx = fe.Context(backend=be)
    a = ctx.create_array((12, 14))
    a[:, :] = 1.5
    b = ctx.create_array((12, 14))
    c = ctx.create_array((12, 14))
    s1 = 0.5 * a[1:-1, 1:-1] + 0.25 * a[:-2, 1:-1] + 0.125 * a[2:, 1:-1] + 0.0625 * a[1:-1, :-2] + 2.0 * a[1:-1, 2:]
    b[1:-1, 1:-1] = s1
    c[1:-1, 1:-1] = -1.0 * a[1:-1, 1:-1] + 1.0 * a[:-2, 1:-1] + 1.0 * a[2:, 1:-1] + 1.0 * a[1:-1, :-2] + 1.0 * a[1:-1, 2:]
    ctx.sync()
    sizes = [len(g) for g in be.groups]
    assert sizes == [1, 2]  # the fill, then b and c fused (same shape, no path between them)
    assert ctx.stats["fused_nodes"] == 2
    ref = np.full((12, 14), 1.5)
    want_b = np.zeros((12, 14))
    want_b[1:-1, 1:-1] = 0.5 * ref[1:-1, 1:-1] + 0.25 * ref[:-2, 1:-1] + 0.125 * ref[2:, 1:-1] + \
        0.0625 * ref[1:-1, :-2] + 2.0 * ref[1:-1, 2:]
    assert np.array_equal(b.data, want_b)


def test_dependent_nodes_not_fused():
    be = NumpyBackend()
    ctx = fe.Context(backend=be)
    a = ctx.create_array((10, 10))
    b = ctx.create_array((10, 10))
    c = ctx.create_array((10, 10))
    star = lambda x: (0.5 * x[1:-1, 1:-1] + 0.25 * x[:-2, 1:-1] + 0.25 * x[2:, 1:-1]  # noqa: E731
                      + 0.25 * x[1:-1, :-2] + 0.25 * x[1:-1, 2:])
    b[1:-1, 1:-1] = star(a)
    c[1:-1, 1:-1] = star(b)  # reads b: a path b -> c, so no fusion
    ctx.sync()
    assert [len(g) for g in be.groups] == [1, 1]


def test_pattern_matchers():
    ctx = fe.Context(backend=NumpyBackend())
    a = ctx.create_array((7, 9))
    b = ctx.create_array((7, 9))
    b[1:-1, 1:-1] = 0.3 * (a[:-2, 1:-1] + a[2:, 1:-1] + a[1:-1, :-2] + a[1:-1, 2:])
    assert fe.match_jacobi(ctx.nodes[-1])[1] == 0.3
    b[1:-1, 1:-1] = 0.3 * (a[2:, 1:-1] + a[:-2, 1:-1] + a[1:-1, :-2] + a[1:-1, 2:])  # S before N
    assert fe.match_jacobi(ctx.nodes[-1]) is None
    b[2:-2, 2:-2] = 1.0 * a[2:-2, 2:-2] + 0.5 * a[1:-3, 2:-2] + 0.5 * a[3:-1, 2:-2] + 0.5 * a[2:-2, 1:-3] + \
        0.5 * a[2:-2, 3:-1] + 0.25 * a[:-4, 2:-2] + 0.25 * a[4:, 2:-2] + 0.25 * a[2:-2, :-4] + 0.25 * a[2:-2, 4:]
    m = fe.match_star(ctx.nodes[-1])
    assert m is not None and m[1] == (1.0, [0.5, 0.25], [0.5, 0.25], [0.5, 0.25], [0.5, 0.25])


def test_unsupported_strided_view():
    ctx = fe.Context(backend=NumpyBackend())
    a = ctx.create_array((8, 8))
    with pytest.raises(NotImplementedError):
        a[::2, :]


def numpy_listing_pair(H, W, T, ring2=1.0):
    u1 = np.zeros((H, W))
    u2 = np.zeros((H, W))
    for u, v in ((u1, 1.0), (u2, ring2)):
        u[0, :] = u[-1, :] = u[:, 0] = u[:, -1] = v
    for _ in range(T):
        u2[1:-1, 1:-1] = 0.25 * (u1[:-2, 1:-1] + u1[2:, 1:-1] + u1[1:-1, :-2] + u1[1:-1, 2:])
        u1, u2 = u2, u1
    return u1, u2


def listing_pair(ctx, H, W, T, ring2=1.0):
    u1 = ctx.create_array((H, W))
    u2 = ctx.create_array((H, W))
    u1[0, :] = u1[-1, :] = u1[:, 0] = u1[:, -1] = 1
    u2[0, :] = u2[-1, :] = u2[:, 0] = u2[:, -1] = ring2
    for _ in range(T):
        u2[1:-1, 1:-1] = 0.25 * (u1[:-2, 1:-1] + u1[2:, 1:-1] + u1[1:-1, :-2] + u1[1:-1, 2:])
        u1, u2 = u2, u1
    ctx.sync()
    return u1, u2


def test_ring_tracking():
    ctx = fe.Context(backend=NumpyBackend())
    z = fe._ZERO_BITS
    one = fe.struct.pack("<d", 1.0)
    a = ctx.create_array((5, 6))
    assert a.ring == (z,) * 8                      # arrays start as zeros
    a[0, :] = 1.0                                  # top row: both top corners and the top part
    assert a.ring[0] == a.ring[1] == a.ring[4] == one and a.ring[2] == z
    a[1:3, 0] = 2.0                                # part of the left column: unknown
    assert a.ring[6] is None and a.ring[0] == one
    a[:, 0] = -0.0                                 # the whole left column, corners included
    assert a.ring[6] == a.ring[0] == a.ring[2] == fe.struct.pack("<d", -0.0) != z
    a[1:-1, 1:-1] = 3.0                            # interior only: ring untouched
    assert a.ring[6] is not None
    b = ctx.create_array((5, 6))
    c = ctx.create_array((5, 6))
    b[0:2, 0:2] = c[1:3, 1:3] + 1.0                # an expression touching the top-left corner
    assert b.ring[0] is None and b.ring[4] is None and b.ring[6] is None and b.ring[1] == z
    ctx.invalidate(b)
    assert b.ring == (None,) * 8
    a.tensor()                                     # handed out: forgotten
    assert a.ring == (None,) * 8
    assert ctx.create_array((2, 9)).ring is None   # no interior: not tracked


@pytest.mark.parametrize("levels", [1, 2, 3, 10])
@pytest.mark.parametrize("depth", [1, 2, 7, 1000])
def test_listing_chains_keep_both_arrays(levels, depth):
    """Chains of Jacobi nodes (the library's plan modelled on the CPU) leave both arrays as one node at a
    time would: iterate T in one, iterate T-1 in the other."""
    for T in (1, 2, 3, 9, 10, 11, 25):
        be = NumpyBackend(chain_levels=levels)
        ctx = fe.Context(max_depth=depth, backend=be)
        u1, u2 = listing_pair(ctx, 9, 12, T)
        w1, w2 = numpy_listing_pair(9, 12, T)
        assert np.array_equal(u1.data, w1) and np.array_equal(u2.data, w2), (levels, depth, T)
        if depth == 1 or T == 1:
            assert ctx.stats["chained_nodes"] == 0
        elif depth >= 1000:
            assert ctx.stats["chained_nodes"] == T and be.chains == [T]


def test_listing_chain_skips_dead_iterate():
    """A chain flushed because the next Jacobi node needs a new DAG leaves iterate m-1 behind only to have
    that node overwrite it: the chain then produces iterate m alone (the model poisons the other array),
    and the final state still equals one node at a time."""
    for depth, T in ((2, 9), (7, 25), (10, 200)):
        be = NumpyBackend(chain_levels=10)
        ctx = fe.Context(max_depth=depth, backend=be)
        u1, u2 = listing_pair(ctx, 9, 12, T)
        w1, w2 = numpy_listing_pair(9, 12, T)
        assert np.array_equal(u1.data, w1) and np.array_equal(u2.data, w2), (depth, T)
        assert ctx.stats["chains_last_only"] > 0 and any(m < 0 for m in be.chains)
        if depth == 10:  # chains of 10 sweeps: one pass of 10 levels, which ends in the other array
            assert be.swaps > 0


def _jac(dst, src):
    dst[1:-1, 1:-1] = 0.25 * (src[:-2, 1:-1] + src[2:, 1:-1] + src[1:-1, :-2] + src[1:-1, 2:])


def test_chain_keeps_iterate_that_is_read_or_partly_overwritten():
    """The dead-iterate shortcut needs both: the chain is the flush's last launch group, and the node that
    caused the flush overwrites the whole interior of the array holding iterate m-1."""
    rng = np.random.default_rng(3)
    init = rng.standard_normal((7, 9))
    init[0, :] = init[-1, :] = init[:, 0] = init[:, -1] = 1.0
    for case in ("partial", "read_after"):
        be = NumpyBackend(chain_levels=3)
        ctx = fe.Context(max_depth=3, backend=be)  # the node after the chain starts a new DAG
        a, b, d = (ctx.create_array((7, 9)) for _ in range(3))
        for u in (a, b):
            u[0, :] = u[-1, :] = u[:, 0] = u[:, -1] = 1.0
            u[1:-1, 1:-1] = 0.0
        ref_a, ref_b, ref_d = np.zeros((7, 9)), np.zeros((7, 9)), np.zeros((7, 9))
        for r in (ref_a, ref_b):
            r[0, :] = r[-1, :] = r[:, 0] = r[:, -1] = 1.0
        ctx.sync()
        a.data[1:-1, 1:-1] = init[1:-1, 1:-1]
        ref_a[1:-1, 1:-1] = init[1:-1, 1:-1]
        src, dst, rs, rd = a, b, ref_a, ref_b
        for _ in range(3):  # a chain of 3: iterate 3 in b, iterate 2 in a
            dst[1:-1, 1:-1] = 0.25 * (src[:-2, 1:-1] + src[2:, 1:-1] + src[1:-1, :-2] + src[1:-1, 2:])
            _jac(rd, rs)
            src, dst, rs, rd = dst, src, rd, rs
        if case == "partial":
            a[1:3, 1:-1] = b[1:3, 1:-1] * 2.0  # overwrites only part of iterate 2, and causes the flush
            ref_a[1:3, 1:-1] = ref_b[1:3, 1:-1] * 2.0
            for _ in range(3):
                a[1:3, 1:-1] = b[1:3, 1:-1] * 2.0
        else:
            d[1:-1, 1:-1] = a[1:-1, 1:-1] * 2.0  # reads iterate 2 after the chain, in the same DAG; the
            # next node overwrites iterate 2 whole and causes the flush
            ref_d[1:-1, 1:-1] = ref_a[1:-1, 1:-1] * 2.0
            a[1:-1, 1:-1] = 0.25 * (b[:-2, 1:-1] + b[2:, 1:-1] + b[1:-1, :-2] + b[1:-1, 2:])
            _jac(ref_a, ref_b)
        ctx.sync()
        for got, want in ((a, ref_a), (b, ref_b), (d, ref_d)):
            assert np.array_equal(got.data, want), case
        assert be.chains and all(m > 0 for m in be.chains), (case, be.chains)


def test_no_chain_when_rings_differ():
    be = NumpyBackend()
    ctx = fe.Context(max_depth=1000, backend=be)
    u1, u2 = listing_pair(ctx, 8, 10, 12, ring2=2.0)
    w1, w2 = numpy_listing_pair(8, 10, 12, ring2=2.0)
    assert np.array_equal(u1.data, w1) and np.array_equal(u2.data, w2)
    assert ctx.stats["chained_nodes"] == 0 and not be.chains


def test_no_chain_after_data_handed_out():
    be = NumpyBackend()
    ctx = fe.Context(max_depth=1000, backend=be)
    u1 = ctx.create_array((8, 8))
    u2 = ctx.create_array((8, 8))
    for u in (u1, u2):
        u[0, :] = u[-1, :] = u[:, 0] = u[:, -1] = 1.0
    u2.tensor()[0, 3] = 7.0  # written outside the frontend
    for _ in range(4):
        u2[1:-1, 1:-1] = 0.25 * (u1[:-2, 1:-1] + u1[2:, 1:-1] + u1[1:-1, :-2] + u1[1:-1, 2:])
        u1, u2 = u2, u1
    ctx.sync()
    assert ctx.stats["chained_nodes"] == 0


def test_no_chain_for_partial_regions_or_other_coefficients():
    be = NumpyBackend()
    ctx = fe.Context(max_depth=1000, backend=be)
    a = ctx.create_array((8, 8))
    b = ctx.create_array((8, 8))
    b[1:-2, 1:-1] = 0.25 * (a[:-3, 1:-1] + a[2:-1, 1:-1] + a[1:-2, :-2] + a[1:-2, 2:])
    a[1:-2, 1:-1] = 0.25 * (b[:-3, 1:-1] + b[2:-1, 1:-1] + b[1:-2, :-2] + b[1:-2, 2:])
    b[1:-1, 1:-1] = 0.25 * (a[:-2, 1:-1] + a[2:, 1:-1] + a[1:-1, :-2] + a[1:-1, 2:])
    a[1:-1, 1:-1] = 0.5 * (b[:-2, 1:-1] + b[2:, 1:-1] + b[1:-1, :-2] + b[1:-1, 2:])
    ctx.sync()
    assert ctx.stats["chained_nodes"] == 0
