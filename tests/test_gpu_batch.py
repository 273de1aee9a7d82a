"""GPU parity of the batched persistent form against the CPU oracle, via the C ABI.

Every grid of a batch must be bit-identical to the oracle's FP32 evaluation
of the listing's sweep, whatever path the plan chose (LDS-resident, global
memory, copy) and whatever launch configuration the tuner picked.
"""

import os

import numpy as np
import pytest

import oracle
from tests.gpu_util import device, say, to_dev, to_host
from workloads import batch_f32, batch_shapes, normal_grid

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ops():
    device()
    from paper_2512_19851_amd import ops

    return ops


MIXED_SHAPES = [(1, 1), (2, 5), (5, 2), (3, 3), (16, 16), (17, 33), (64, 64), (100, 257), (256, 255), (300, 250),
                (3, 700), (700, 3), (45, 61), (128, 130), (150, 180), (190, 129), (33, 200)]


def _check(outs, u0s, T):
    for k, (o, u) in enumerate(zip(outs, u0s)):
        want = oracle.jacobi5(u, T, dtype=np.float32)
        got = to_host(o)
        assert np.array_equal(got, want), f"grid {k} shape {u.shape} T={T}"


@pytest.mark.parametrize("T", [0, 1, 2, 3, 10])
def test_mixed_batch_bit_exact(ops, T):
    u0s = [normal_grid(*s, seed=k, dtype=np.float32) for k, s in enumerate(MIXED_SHAPES)]
    say(f"batch mixed T={T}")
    plan = ops.BatchPlan([to_dev(u) for u in u0s], T)
    outs = plan.run()
    _check(outs, u0s, T)


@pytest.mark.parametrize("reg", [True, False], ids=["reg", "noreg"])
@pytest.mark.parametrize("cfg", [(256, 32 * 1024, 4), (512, 64 * 1024, 2), (1024, 160 * 1024, 1),
                                 (64, 8 * 1024, 8), (128, 2048, 2), (1024, 64 * 1024, 1)])
def test_launch_configurations(ops, cfg, reg):
    """Each configuration moves a different set of grids between register, LDS and global sweeps."""
    u0s = [normal_grid(*s, seed=10 + k, dtype=np.float32) for k, s in enumerate(MIXED_SHAPES)]
    plan = ops.BatchPlan([to_dev(u) for u in u0s], 5)
    plan.set_register_mode(reg)
    plan.configure(*cfg)
    info = plan.info()
    say(f"batch cfg {cfg} reg={reg} -> {info}")
    _check(plan.run(), u0s, 5)


def test_register_mode_covers_workload(ops):
    """With 1024-lane workgroups every grid of the batch workload fits the register mode."""
    u0s = batch_f32(0)[:64]
    plan = ops.BatchPlan([to_dev(u) for u in u0s], 7)
    plan.configure(1024, 160 * 1024, 1)
    info = plan.info()
    say(f"batch reg coverage {info}")
    assert info["n_reg"] == len(u0s)
    _check(plan.run(), u0s, 7)


def test_workload_batch_T10(ops):
    """1024 grids, point counts log-uniform in [2^8, 2^16], FP32 N(0,1), seed 0; T = 10."""
    u0s = batch_f32(0)
    assert len(u0s) == 1024
    say("batch workload T=10")
    plan = ops.BatchPlan([to_dev(u) for u in u0s], 10)
    say(f"plan {plan.info()}")
    _check(plan.run(), u0s, 10)


def test_workload_batch_T100_sampled(ops):
    """The benchmarked call (T = 100): the 16 largest grids and 32 others, bit-exact."""
    u0s = batch_f32(0)
    say("batch workload T=100")
    plan = ops.BatchPlan([to_dev(u) for u in u0s], 100)
    outs = plan.run()
    sizes = np.array([u.size for u in u0s])
    pick = list(np.argsort(-sizes)[:16]) + list(np.random.default_rng(5).choice(1024, 32, replace=False))
    for k in sorted(set(int(x) for x in pick)):
        assert np.array_equal(to_host(outs[k]), oracle.jacobi5(u0s[k], 100, dtype=np.float32)), f"grid {k}"


def test_autotune_and_cache(ops, tmp_path):
    u0s = [normal_grid(*s, seed=20 + k, dtype=np.float32) for k, s in enumerate(MIXED_SHAPES)]
    dev_u = [to_dev(u) for u in u0s]
    cache = str(tmp_path / "batch_tune.txt")
    say("batch autotune")
    plan = ops.BatchPlan(dev_u, 4)
    best = plan.autotune(cache, reps=1)
    assert best > 0 and os.path.exists(cache)
    chosen = plan.info()
    _check(plan.run(), u0s, 4)
    plan2 = ops.BatchPlan(dev_u, 4, tune_cache=cache)
    info2 = plan2.info()
    assert (info2["block"], info2["lds_bytes"]) == (chosen["block"], chosen["lds_bytes"])
    _check(plan2.run(), u0s, 4)


def test_graph_capture_replays(ops):
    """plan.run() captured in a HIP graph; every replay matches the eager result."""
    import torch

    u0s = [normal_grid(*s, seed=30 + k, dtype=np.float32) for k, s in enumerate(MIXED_SHAPES)]
    plan = ops.BatchPlan([to_dev(u) for u in u0s], 6)
    eager = [to_host(o).copy() for o in plan.run()]
    for o in plan.outs:
        o.zero_()
    s = torch.cuda.Stream()
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=s):
        plan.run()
    say("batch graph replays")
    for rep in range(3):
        for o in plan.outs:
            o.fill_(float(rep + 1))  # eager work between replays
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        for k, o in enumerate(plan.outs):
            assert np.array_equal(to_host(o), eager[k]), f"replay {rep} grid {k}"


def test_batch_errors(ops):
    import ctypes

    import torch

    from paper_2512_19851_amd import _lib

    lib = _lib.load()
    u = to_dev(normal_grid(8, 8, dtype=np.float32))
    arr = (_lib.StenInst * 1)()
    arr[0].u0, arr[0].out, arr[0].work = u.data_ptr(), u.data_ptr(), None
    arr[0].H = arr[0].W = arr[0].ld = 8
    ws = torch.empty(4096, dtype=torch.uint8, device=u.device)
    h = ctypes.c_void_p()
    stream = torch.cuda.current_stream().cuda_stream
    say("batch error paths")
    assert lib.sten_batch_plan(ctypes.cast(arr, ctypes.c_void_p), 1, 3, 0.25, None, ws.data_ptr(), 4096,
                               ctypes.byref(h), stream) == -2  # out aliases u0
    out = torch.empty_like(u)
    arr[0].out = out.data_ptr()
    assert lib.sten_batch_plan(ctypes.cast(arr, ctypes.c_void_p), 1, 3, 0.25, None, ws.data_ptr(), 10,
                               ctypes.byref(h), stream) == -4  # workspace too small
    assert lib.sten_batch_plan(ctypes.cast(arr, ctypes.c_void_p), 1, -1, 0.25, None, ws.data_ptr(), 4096,
                               ctypes.byref(h), stream) == -1
    torch.cuda.synchronize()


def test_batch_shapes_recipe():
    """Shape recipe: 1024 grids, sides >= 3, point counts within [2^8, 2^16] up to rounding."""
    shapes = batch_shapes(0)
    n = np.array([h * w for h, w in shapes])
    assert len(shapes) == 1024 and min(min(s) for s in shapes) >= 3
    assert n.min() >= 200 and n.max() <= 66000


def test_reconfigure_rejects_global_grid_without_work(ops):
    """A plan whose grids have no `work` buffer stays valid: any configuration that would
    sweep such a grid in global memory (T >= 2) is refused with STEN_ERR_PTR, the plan keeps
    its previous configuration, and the autotuner skips those candidates."""
    # every grid fits registers or LDS by default (300 x 250 and 100 x 257 need global memory)
    shapes = [s for s in MIXED_SHAPES if s not in ((300, 250), (100, 257))]
    u0s = [normal_grid(*s, seed=40 + k, dtype=np.float32) for k, s in enumerate(shapes)]
    plan = ops.BatchPlan([to_dev(u) for u in u0s], 3, works=[None] * len(u0s))
    before = plan.info()
    assert before["n_global"] == 0
    say(f"batch no-work plan {before}")
    with pytest.raises(RuntimeError, match="STEN_ERR_PTR|-3"):
        plan.configure(64, 1024, 1)  # 1 KiB of LDS: the larger grids would sweep in global memory
    assert plan.info() == before
    with pytest.raises(RuntimeError, match="STEN_ERR_PTR|-3"):
        plan.set_register_mode(False)  # 256 x 255 needs 510 KiB in LDS mode
    assert plan.info() == before
    _check(plan.run(), u0s, 3)
    plan.autotune(None, reps=1)
    assert plan.info()["n_global"] == 0
    _check(plan.run(), u0s, 3)
