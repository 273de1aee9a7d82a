"""The lid-driven cavity flow on the frontend (generated and hand-written kernels) against the oracle."""

import numpy as np
import pytest

from oracle import cavity as oc
from paper_2512_19851_amd import frontend as fe
from paper_2512_19851_amd.cavity import CavityFlow
from tests.gpu_util import device, say, to_host

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("shape,nit,nt", [((41, 41), 50, 10), ((33, 65), 20, 5), ((5, 5), 3, 3),
                                          ((257, 513), 10, 2)], ids=["41x41", "33x65", "5x5", "257x513"])
def test_cavity_bit_exact(shape, nit, nt):
    device()
    H, W = shape
    say(f"cavity {shape} nit={nit} nt={nt}")
    ctx = fe.Context(max_depth=64)
    flow = CavityFlow(ctx, H, W, nit=nit)
    flow.run(nt)
    u, v, p = (to_host(x) for x in flow.fields())
    uo, vo, po = oc.run(nt, oc.CavityParams(H, W, nit=nit))
    assert np.array_equal(u, uo)
    assert np.array_equal(v, vo)
    assert np.array_equal(p, po)
    assert ctx.stats["fused_nodes"] >= 2 * nt  # u and v updates fused every step


@pytest.mark.parametrize("blocked", [True, False], ids=["blocked", "per_node"])
@pytest.mark.parametrize("shape,nit,nt", [((130, 256), 50, 3), ((64, 128), 7, 4), ((3, 130), 5, 2)],
                         ids=["130x256", "64x128", "3x130"])
def test_cavity_blocked_pressure_bit_exact(shape, nit, nt, blocked):
    """The pressure iterations as one blocked call per step give the per-node program's bits."""
    device()
    H, W = shape
    say(f"cavity {shape} nit={nit} nt={nt} blocked={blocked}")
    ctx = fe.Context(max_depth=64)
    flow = CavityFlow(ctx, H, W, nit=nit, blocked_pressure=blocked)
    assert flow.blocked_pressure == blocked
    flow.run(nt)
    u, v, p = (to_host(x) for x in flow.fields())
    uo, vo, po = oc.run(nt, oc.CavityParams(H, W, nit=nit))
    assert np.array_equal(u, uo)
    assert np.array_equal(v, vo)
    assert np.array_equal(p, po)
