"""libsten loads without a GPU and exports every symbol include/sten.h declares.

No compute call is made here; only host-side helpers are exercised.
"""

import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "sten.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"^\s*(?:[A-Za-z_][\w\s\*]*?)\b(sten_\w+)\s*\(", text, flags=re.M)
    return sorted(set(names))


@pytest.fixture(scope="module")
def lib():
    from paper_2512_19851_amd import _lib

    return _lib.load()


def test_header_declares_functions():
    names = declared_functions()
    assert "sten_jacobi5_f64" in names and "sten_status_string" in names
    assert len(names) >= 8


def test_every_declared_symbol_is_exported(lib):
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, f"declared but not exported: {missing}"


def test_binding_covers_header():
    from paper_2512_19851_amd import _lib

    missing = [n for n in declared_functions() if n not in _lib.SIGNATURES]
    assert not missing, f"no ctypes signature for: {missing}"


def test_single_hip_runtime(lib):
    from paper_2512_19851_amd import _lib

    assert len(_lib._hip_runtimes_mapped()) <= 1


def test_status_strings(lib):
    for code in (0, -1, -2, -3, -4, -5, -6):
        s = lib.sten_status_string(code).decode()
        assert s.startswith("STEN_")
    assert b"gfx950" in lib.sten_version()


@pytest.mark.parametrize("nb", [1, 2, 7, 8, 9, 15, 16, 17, 255, 256, 1000, 1024, 2047, 8191])
def test_xcd_map_is_bijective_and_banded(lib, nb):
    tiles = [lib.sten_xcd_tile_of_block(b, nb) for b in range(nb)]
    assert sorted(tiles) == list(range(nb))
    # every XCD (b mod 8) walks a contiguous, increasing range of tiles
    for x in range(8):
        mine = [tiles[b] for b in range(x, nb, 8)]
        assert mine == list(range(mine[0], mine[0] + len(mine))) if mine else True


def test_tune_hook_rejects_bad_rows(lib):
    assert lib.sten_tune_sweep_rows(5) == -1
    assert lib.sten_tune_sweep_rows(0) == 0


def test_tune_hooks_validate_and_restore(lib):
    """Host-only hooks: bad values are rejected, 0 restores the built-in choice."""
    assert lib.sten_tune_tb(3, 0, 0) == -1          # no such variant
    assert lib.sten_tune_tb(-1, 0, 0) == -1
    assert lib.sten_tune_tb(2, -1, 0) == -1         # negative band
    assert lib.sten_tune_tb(2, 0, 3) == -1          # depth not 0 or 4
    assert lib.sten_tune_tb(2, 0, 7) == -1
    assert lib.sten_tune_tb(2, 17, 4) == 0
    assert lib.sten_tune_tb(0, 0, 0) == 0
    assert lib.sten_tune_schedule(15) == -1
    assert lib.sten_tune_schedule(-1) == -1
    assert lib.sten_tune_schedule(14) == 0
    assert lib.sten_tune_schedule(12) == 0
    assert lib.sten_tune_schedule(0) == 0
    assert lib.sten_tune_tb_rows(5) == -1
    assert lib.sten_tune_tb_rows(0) == 0


def test_validation_before_any_hip_call(lib):
    """Argument errors are reported without touching the GPU (no device here)."""
    f = lib.sten_jacobi5_f64
    assert f(None, None, None, -1, 4, 4, 1, 0.25, None) == -1     # H < 0
    assert f(None, None, None, 4, 4, 3, 1, 0.25, None) == -1      # ld < W
    assert f(None, None, None, 4, 4, 4, -2, 0.25, None) == -1     # T < 0
    assert f(None, None, None, 0, 4, 4, 1, 0.25, None) == 0       # empty grid: no-op
    assert f(None, None, None, 4, 4, 4, 1, 0.25, None) == -3      # NULL pointers
    # overlapping buffers are rejected before any pointer query
    assert f(4096, 4096 + 8, 1 << 20, 4, 4, 4, 1, 0.25, None) == -2
    assert f(4096, 1 << 20, 1 << 20, 4, 4, 4, 2, 0.25, None) == -2


def test_tiled_workspace_query(lib):
    """Host-only layout query: valid tilings need space, invalid ones report 0."""
    assert lib.sten_tiled_workspace_bytes(64, 64, 2, 2) > 2 * 64 * 64 * 8
    assert lib.sten_tiled_workspace_bytes(64, 64, 65, 1) == 0
    assert lib.sten_tiled_workspace_bytes(0, 64, 1, 1) == 0
    one = lib.sten_tiled_workspace_bytes(100, 100, 1, 1)
    many = lib.sten_tiled_workspace_bytes(100, 100, 4, 4)
    assert many > one  # ghost frames and send buffers grow with the tile count


def test_tiled_ghost_workspace_query(lib):
    """Deeper ghost frames need more space; a tile thinner than the ghost depth across a shared edge is refused."""
    ws = lib.sten_tiled_workspace_bytes_ex
    g1 = ws(64, 64, 2, 2, 1, 0)
    assert g1 == lib.sten_tiled_workspace_bytes(64, 64, 2, 2)
    assert ws(64, 64, 2, 2, 8, 0) > g1
    assert 0 < ws(64, 64, 2, 2, 8, 1) < ws(64, 64, 2, 2, 8, 0)  # direct mode has no send buffers
    assert ws(64, 64, 2, 2, 1, 2) == 0                           # unknown mode
    assert ws(64, 64, 2, 2, 0, 0) == 0
    assert ws(64, 64, 2, 2, 13, 0) == 0
    assert ws(20, 64, 4, 1, 5, 0) > 0   # tiles 5 rows tall
    assert ws(20, 64, 4, 1, 6, 0) == 0  # thinner than the ghost depth
    assert ws(3, 64, 1, 4, 12, 1) > 0   # one tile row: row count is free


def _plan(lib, H, W, pr, pc, g, mode=0):
    import ctypes

    info = (ctypes.c_int64 * 4)()
    st = lib.sten_tiled_plan_check(H, W, pr, pc, g, mode, info, 4)
    return st, list(info)


@pytest.mark.parametrize("mode", [0, 1], ids=["packed", "direct"])
@pytest.mark.parametrize("g", [1, 2, 3, 7, 12])
def test_tiled_plan_in_bounds(lib, g, mode):
    """Every exchange copy, owned block and sweep view of a plan lies inside its buffer (host check, no
    device), over square, ragged, single-row and single-column tilings."""
    shapes = [(5, 7), (64, 64), (130, 513), (257, 1031), (100, 300), (3, 600), (600, 3), (4096, 4096),
              (97, 143), (50, 50)]
    tilings = [(1, 1), (2, 2), (3, 5), (1, 6), (7, 1), (4, 4), (2, 3)]
    checked = 0
    for H, W in shapes:
        for pr, pc in tilings:
            valid = lib.sten_tiled_workspace_bytes_ex(H, W, pr, pc, g, mode) > 0
            st, info = _plan(lib, H, W, pr, pc, g, mode)
            if not valid:
                assert st == -1, (H, W, pr, pc, g)
                continue
            assert st == 0, (H, W, pr, pc, g)
            tiles, msgs, launches, nbytes = info
            assert tiles == pr * pc
            # one message per edge shared by two tiles in each direction, and for g > 1 one per
            # diagonal pair of tiles in each direction
            edges = 2 * (pr * (pc - 1) + pc * (pr - 1))
            corners = 4 * (pr - 1) * (pc - 1) if g > 1 else 0
            assert msgs == edges + corners
            assert launches == (0 if msgs == 0 else (2 if mode == 0 else 1))
            assert nbytes == lib.sten_tiled_workspace_bytes_ex(H, W, pr, pc, g, mode)
            checked += 1
    assert checked > 20


def test_tiled_plan_rejects(lib):
    import ctypes

    assert _plan(lib, 64, 64, 65, 1, 1)[0] == -1
    assert _plan(lib, 64, 64, 2, 2, 0)[0] == -1
    assert _plan(lib, 8, 64, 2, 1, 5)[0] == -1
    assert _plan(lib, 64, 64, 2, 2, 2, mode=5)[0] == -1
    assert lib.sten_tiled_plan_check(64, 64, 2, 2, 2, 0, None, 4) == -1
    info = (ctypes.c_int64 * 3)()
    assert lib.sten_tiled_plan_check(64, 64, 2, 2, 2, 0, info, 3) == -1


def test_cavity_pressure_rejects_before_any_hip_call(lib):
    """Sizes, pointers, aliasing and the blocked kernel's layout are checked on the host (fake pointers)."""
    f = lib.sten_cavity_pressure_f64
    A, B, O, K = 1 << 30, 2 << 30, 3 << 30, 4 << 30  # disjoint fake addresses, 16-byte aligned
    assert f(A, B, O, K, -1, 128, 128, 3, 0.2, 0.3, 0.1, 0, None) == -1   # H < 0
    assert f(A, B, O, K, 8, 128, 127, 3, 0.2, 0.3, 0.1, 0, None) == -1    # ld < W
    assert f(A, B, O, K, 8, 128, 128, -1, 0.2, 0.3, 0.1, 0, None) == -1   # nit < 0
    assert f(A, B, O, K, 8, 128, 128, 3, 0.2, 0.3, 0.1, 13, None) == -1   # levels > 12
    assert f(A, B, O, K, 0, 128, 128, 3, 0.2, 0.3, 0.1, 0, None) == 0     # empty: no-op
    assert f(None, B, O, K, 8, 128, 128, 3, 0.2, 0.3, 0.1, 0, None) == -3
    assert f(A, B, O, None, 8, 128, 128, 13, 0.2, 0.3, 0.1, 0, None) == -3  # two passes need work
    assert f(A, B, O, None, 8, 128, 128, 9, 0.2, 0.3, 0.1, 8, None) == -3   # ... also at 8 levels
    assert f(A, B, A + 64, K, 8, 128, 128, 3, 0.2, 0.3, 0.1, 0, None) == -2  # out overlaps p0
    assert f(A, B, O, B, 8, 128, 128, 13, 0.2, 0.3, 0.1, 0, None) == -2      # work overlaps b
    assert f(A, B, O, K, 8, 126, 128, 3, 0.2, 0.3, 0.1, 0, None) == -6      # W < 128
    assert f(A, B, O, K, 8, 129, 130, 3, 0.2, 0.3, 0.1, 0, None) == -6      # odd W
    assert f(A, B, O, K, 2, 128, 128, 3, 0.2, 0.3, 0.1, 0, None) == -6      # H < 3
    assert f(A + 8, B, O, K, 8, 128, 128, 3, 0.2, 0.3, 0.1, 0, None) == -6  # unaligned
    assert lib.sten_tune_pressure(-1) == -1
    assert lib.sten_tune_pressure(0) == 0
    assert lib.sten_tune_adjoint_levels(-1) == -1
    assert lib.sten_tune_adjoint_levels(9) == -1
    assert lib.sten_tune_adjoint_levels(0) == 0


def test_expr_run_rejects_before_any_hip_call(lib):
    """Program syntax, load extents and aliasing are checked on the host (fake pointers, no device)."""
    import ctypes

    from paper_2512_19851_amd import _lib

    ins = (_lib.StenExprIn * 1)()
    ins[0].base, ins[0].ld = 0x10000000, 100
    ins[0].row_lo, ins[0].row_hi, ins[0].col_lo, ins[0].col_hi = -1, 8, -1, 98
    outs = (_lib.StenExprOut * 1)()
    outs[0].base, outs[0].ld = 0x20000000, 100
    run = lambda prog, rows, cols: lib.sten_expr_run(  # noqa: E731
        prog, ctypes.cast(ins, ctypes.c_void_p), 1, ctypes.cast(outs, ctypes.c_void_p), 1, rows, cols, None)
    assert run(b"L0,1,0 L0,-1,0 +", 9, 98) == -1          # last row 8, plus 1, leaves the extent
    assert run(b"L0,1,0 L0,-1,0 +", 8, 98) == -3          # inside: checks pass, the fake pointer does not
    assert run(b"L0,0,0 *", 4, 4) == -1                   # bad postfix
    assert run(b"L1,0,0", 4, 4) == -1                     # no slot 1
    assert run(b"L0,0,0; L0,0,0", 4, 4) == -1             # two expressions, one output
    outs[0].base = 0x10000000 + 8 * 50                    # output inside the input's extent
    assert run(b"L0,0,0", 4, 4) == -2
    outs[0].base = 0x20000000
    assert run(b"L0,0,0", 0, 4) == 0                      # empty region
    assert run(b"L0,0,0", 1, 2**31 - 200) == -1           # column indices would pass 32 bits
    assert b"expression" in lib.sten_expr_log() or lib.sten_expr_log() == b""


def test_workspace_query_per_op(lib):
    """sten_workspace_bytes agrees with each op's own query and with the buffers the calls take."""
    from paper_2512_19851_amd import _lib

    q = lib.sten_workspace_bytes
    bad = _lib.WORKSPACE_INVALID
    H, W = 4096, 4096
    assert q(_lib.OP_F64, H, W, 100) == H * W * 8
    assert q(_lib.OP_F32, H, W, 100) == H * W * 4
    assert q(_lib.OP_ADJ, 1024, 1024, 10) == 1024 * 1024 * 4
    assert q(_lib.OP_HILO, H, W, 100) == lib.sten_jacobi5_f64_hilo_work_bytes(H, W)
    assert q(_lib.OP_HILO, H, W, 0) == lib.sten_jacobi5_f64_hilo_work_bytes(H, W)  # encode/decode staging
    assert q(_lib.OP_BATCH, 1024, 0, 0) == lib.sten_batch_workspace_bytes(1024)
    assert q(_lib.OP_STATES, 1024, 1024, 10) == 11 * 1024 * 1024 * 4
    # no second buffer: T < 2 or an empty interior
    for op in (_lib.OP_F64, _lib.OP_F32, _lib.OP_ADJ):
        assert q(op, H, W, 0) == 0 and q(op, H, W, 1) == 0
        assert q(op, 2, W, 10) == 0 and q(op, H, 2, 10) == 0
    assert q(_lib.OP_HILO, 0, W, 3) == 0 and q(_lib.OP_STATES, H, 0, 3) == 0
    assert q(_lib.OP_BATCH, 0, 0, 0) == lib.sten_batch_workspace_bytes(0)


def test_workspace_query_errors(lib):
    from paper_2512_19851_amd import _lib

    q = lib.sten_workspace_bytes
    bad = _lib.WORKSPACE_INVALID
    assert bad == 2**64 - 1
    for op in (-1, 6, 99):
        assert q(op, 64, 64, 2) == bad  # unknown op
    for op in range(6):
        assert q(op, -1, 64, 2) == bad
        assert q(op, 64, -1, 2) == bad
        assert q(op, 64, 64, -1) == bad
        assert q(op, (1 << 30) + 1, 64, 2) == bad
    assert q(_lib.OP_BATCH, 2**31, 0, 0) == bad
    # 2^30 x 2^30 FP32 states x (2^31) grids overflow size_t
    assert q(_lib.OP_STATES, 1 << 30, 1 << 30, 2**31 - 1) == bad


def test_tiled_tile_count_capped(lib):
    """A tiling of more than 65536 tiles is refused (the planner's host tables grow with the tile count)."""
    assert lib.sten_tiled_workspace_bytes(4096, 4096, 256, 256) > 0      # 65536 tiles
    assert lib.sten_tiled_workspace_bytes(4096, 4096, 257, 256) == 0     # one row of tiles more
    assert lib.sten_tiled_workspace_bytes(2**30, 2**30, 2, 2**30) == 0


def test_tiled_plan_check_large_ghost_strips(lib):
    """Ghost blocks of more than 2^31 elements (12 x a 2^28-column tile) are planned without overflow."""
    import ctypes

    info = (ctypes.c_int64 * 4)()
    st = lib.sten_tiled_plan_check(2 * 2**28, 2**28, 2, 1, 1, 1, info, 4)
    assert st in (0, -6)  # planned (or refused by a layout check), never a crash or garbage
