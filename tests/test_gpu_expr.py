"""Generated kernels for slice expressions (run-time code generation) against NumPy, via the C ABI.

NumPy evaluating the same slice expression element by element in FP64 is the
reference: every operation rounds once, in the expression's order, and the
generated kernels must give the same bits.
"""

import numpy as np
import pytest

from paper_2512_19851_amd import frontend as fe
from tests.gpu_util import device, say, to_dev, to_host
from tests.numpy_backend import NumpyBackend
from workloads import normal_grid

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ops():
    device()
    from paper_2512_19851_amd import ops

    return ops


def program_a(ctx_arrays):
    a, b, c, out1, out2, out3 = ctx_arrays
    out1[1:-1, 2:-1] = (a[:-2, 2:-1] - 3.0 * b[2:, 1:-2]) / (c[1:-1, 3:] * c[1:-1, 3:] + 1.5) - a[1:-1, 2:-1]
    out2[1:-1, 2:-1] = -(b[1:-1, 1:-2] ** 2) + 0.1 * a[2:, 3:] / 7.0   # fused with out1 (same shape, no path)
    out3[2:, :] = (a[:-2, :] + b[2:, :] - c[1:-1, :]) * (a[1:-1, :] - 0.3)


def run_program(backend, shape, seed):
    ctx = fe.Context(backend=backend)
    arrs = [ctx.create_array(shape) for _ in range(6)]
    for k, x in enumerate(arrs[:3]):
        x.data[...] = backend_input(backend, normal_grid(*shape, seed=seed + k))
    program_a(arrs)
    ctx.sync()
    return [np.asarray(to_host(x.data) if not isinstance(x.data, np.ndarray) else x.data) for x in arrs[3:]], backend


def backend_input(backend, a):
    return a if isinstance(backend, NumpyBackend) else to_dev(a)


@pytest.mark.parametrize("shape", [(5, 6), (37, 300), (130, 1031), (1000, 257)], ids=lambda s: f"{s[0]}x{s[1]}")
def test_generated_kernels_bit_exact(ops, shape):
    say(f"expr program {shape}")
    want, nb = run_program(NumpyBackend(), shape, 11)
    got, _ = run_program(fe.GpuBackend(), shape, 11)
    for g, w in zip(got, want):
        assert np.array_equal(g, w)
    assert [len(g) for g in nb.groups] == [2, 1]


def test_expr_run_direct_and_checks(ops):
    import torch

    H, W = 70, 333
    a = to_dev(normal_grid(H, W, seed=3))
    out = torch.zeros((H, W), dtype=torch.float64, device=device())
    prog = "L0,-1,0 L0,1,0 + L0,0,-1 + L0,0,1 + C0x1p-2 *"
    say("expr direct jacobi form")
    ops.expr_run(prog, [(a, 1, 1)], [(out, 1, 1)], H - 2, W - 2)
    ah = to_host(a)
    want = np.zeros((H, W))
    want[1:-1, 1:-1] = 0.25 * (ah[:-2, 1:-1] + ah[2:, 1:-1] + ah[1:-1, :-2] + ah[1:-1, 2:])
    assert np.array_equal(to_host(out), want)
    # a load one row past the array: rejected before any launch
    with pytest.raises(ops._lib.StenError) as e:
        ops.expr_run("L0,1,0", [(a, 1, 1)], [(out, 1, 1)], H - 1, W - 2)
    assert e.value.name == "STEN_ERR_ARG" and "extent" in ops.expr_log()
    # output overlapping an input: the paper's no-self-read rule
    with pytest.raises(ops._lib.StenError) as e:
        ops.expr_run("L0,0,0", [(a, 0, 0)], [(a, 0, 0)], 4, 4)
    assert e.value.name == "STEN_ERR_ALIAS"
    with pytest.raises(ops._lib.StenError):
        ops.expr_run("L0,0,0 +", [(a, 0, 0)], [(out, 0, 0)], 4, 4)
    ops.expr_run("L0,0,0", [(a, 0, 0)], [(out, 0, 0)], 0, 5)  # empty region: nothing to do


def test_many_outputs_split_into_kernels(ops):
    """More than 8 fused outputs run as consecutive generated kernels with the same results."""
    shape = (20, 70)
    res = []
    for be in (NumpyBackend(), fe.GpuBackend()):
        ctx = fe.Context(backend=be)
        src = ctx.create_array(shape)
        src.data[...] = backend_input(be, normal_grid(*shape, seed=4))
        outs = [ctx.create_array(shape) for _ in range(11)]
        for k, o in enumerate(outs):
            o[1:-1, 1:-1] = src[1:-1, 1:-1] * float(k + 1) - src[:-2, 1:-1] / 3.0
        ctx.sync()
        res.append([np.asarray(o.data if isinstance(o.data, np.ndarray) else to_host(o.data)) for o in outs])
    say("expr split group")
    for g, w in zip(res[1], res[0]):
        assert np.array_equal(g, w)
