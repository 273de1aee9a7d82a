"""The generated-kernel source, on the host (no GPU): its structure and that the run-time compiler takes it.

The GPU tests compare generated kernels with NumPy bit for bit; these pin what the generator emits: each
thread computes two adjacent elements of a row, every distinct (slot, row offset, column offset) operand
is one 16-byte pair load shared by both elements, every output pair one 16-byte store, the operations of
each element stay in program order, and the last column of an odd-width row has a single-element path.
"""

import re

import pytest

JACOBI = "L0,-1,0 L0,1,0 + L0,0,-1 + L0,0,1 + C0x1p-2 *"


@pytest.fixture(scope="module")
def ops():
    from paper_2512_19851_amd import ops

    return ops


def test_pairs_and_program_order(ops):
    src = ops.expr_source(JACOBI, 1, 1)
    pair_loads = re.findall(r"const sten_pair (p\d+) = \*reinterpret_cast<const sten_pair\*>\(([^;]*)\);", src)
    scalar_loads = re.findall(r"const double (l\d+) = \*\(([^;]*)\);", src)
    assert len(pair_loads) == 4 and len(scalar_loads) == 4   # one per distinct operand, in each path
    # the pair path evaluates element 0 from the .x halves, then element 1 from the .y halves, each in the
    # program's order: ((N + S) + W) + E, then * c
    names = [p for p, _ in pair_loads]
    for half, first_tmp in ((".x", 0), (".y", 4)):
        t = first_tmp
        assert f"const double t{t} = {names[0]}{half} + {names[1]}{half};" in src
        assert f"const double t{t + 1} = t{t} + {names[2]}{half};" in src
        assert f"const double t{t + 2} = t{t + 1} + {names[3]}{half};" in src
        assert f"const double t{t + 3} = t{t + 2} * (0x1p-2);" in src
    assert src.count("*reinterpret_cast<sten_pair*>(a.out[0]") == 1       # one pair store
    assert "if (j + 1 < a.cols)" in src and "a.out[0][r * a.ldo[0] + j] = t11;" in src  # the odd tail
    # no contraction: the source has no fused multiply-add calls
    assert "fma" not in src


def test_shared_operands_are_loaded_once(ops):
    # the same operand used by two outputs and twice in one expression is one load per path
    src = ops.expr_source("L0,0,1 L0,0,1 * ; L0,0,1 N", 1, 2)
    assert len(re.findall(r"const sten_pair p\d+ =", src)) == 1
    assert len(re.findall(r"const double l\d+ = \*\(", src)) == 1
    assert src.count("*reinterpret_cast<sten_pair*>(a.out[0]") == 1
    assert src.count("*reinterpret_cast<sten_pair*>(a.out[1]") == 1


def test_generated_source_compiles(ops):
    ops.expr_compile(JACOBI, 1, 1)
    ops.expr_compile("L0,0,-3 L1,2,5 * L0,0,3 - ; L1,-1,-1 N Q", 2, 2)
    with pytest.raises(ops._lib.StenError):
        ops.expr_source("L0,0,0 +", 1, 1)
