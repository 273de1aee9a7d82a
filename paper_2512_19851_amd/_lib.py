"""ctypes loader for libsten.so: argument marshalling only.

torch is imported before the library is loaded so that libsten's HIP runtime
dependency resolves to the runtime torch already mapped; a second HIP runtime
in the process would not understand torch's stream handles. The loader checks
that exactly one HIP runtime is mapped and fails loudly otherwise, and fails
loudly when the library has not been built.
"""

from __future__ import annotations

import ctypes
import os

import torch  # noqa: F401  (must precede loading libsten; see module docstring)

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libsten.so")

# sten_op values of include/sten.h
OP_F64, OP_F32, OP_HILO, OP_BATCH, OP_ADJ, OP_STATES = range(6)
WORKSPACE_INVALID = ctypes.c_size_t(-1).value

STATUS = {
    0: "STEN_OK",
    -1: "STEN_ERR_ARG",
    -2: "STEN_ERR_ALIAS",
    -3: "STEN_ERR_PTR",
    -4: "STEN_ERR_WORKSPACE",
    -5: "STEN_ERR_HIP",
    -6: "STEN_ERR_UNSUPPORTED",
}


class StenError(RuntimeError):
    """A libsten call returned a non-zero status."""

    def __init__(self, fn: str, code: int, hip: int | None = None):
        self.code = code
        self.name = STATUS.get(code, str(code))
        msg = f"{fn} failed: {self.name}"
        if hip:
            msg += f" (hipError {hip})"
        super().__init__(msg)


_i64 = ctypes.c_int64
_i32 = ctypes.c_int32
_u32 = ctypes.c_uint32
_vp = ctypes.c_void_p
_sz = ctypes.c_size_t
_f64 = ctypes.c_double
_f32 = ctypes.c_float

# name -> (restype, argtypes); mirrors include/sten.h
SIGNATURES = {
    "sten_status_string": (ctypes.c_char_p, [ctypes.c_int]),
    "sten_last_hip_error": (ctypes.c_int, []),
    "sten_workspace_bytes": (_sz, [ctypes.c_int, _i64, _i64, _i32]),
    "sten_version": (ctypes.c_char_p, []),
    "sten_xcd_tile_of_block": (_u32, [_u32, _u32]),
    "sten_jacobi5_f64": (ctypes.c_int, [_vp, _vp, _vp, _i64, _i64, _i64, _i32, _f64, _vp]),
    "sten_jacobi5_f32": (ctypes.c_int, [_vp, _vp, _vp, _i64, _i64, _i64, _i32, _f32, _vp]),
    "sten_tune_sweep_rows": (ctypes.c_int, [_i32]),
    "sten_sweep_f64": (ctypes.c_int, [_vp, _vp, _i64, _i64, _i64, _f64, _vp]),
    "sten_sweep_f32": (ctypes.c_int, [_vp, _vp, _i64, _i64, _i64, _f32, _vp]),
    "sten_fill_rect_f64": (ctypes.c_int, [_vp, _i64, _i64, _i64, _i64, _i64, _i64, _i64, _f64, _vp]),
    "sten_jacobi5_f64_tb": (ctypes.c_int, [_vp, _vp, _vp, _i64, _i64, _i64, _i32, _f64, _i32, _vp]),
    "sten_jacobi5_f32_tb": (ctypes.c_int, [_vp, _vp, _vp, _i64, _i64, _i64, _i32, _f32, _i32, _vp]),
    "sten_tune_tb_rows": (ctypes.c_int, [_i32]),
    "sten_tune_tb": (ctypes.c_int, [_i32, _i32, _i32]),
    "sten_tune_schedule": (ctypes.c_int, [_i32]),
    "sten_hilo_bytes": (_sz, [_i64, _i64]),
    "sten_jacobi5_f64_hilo_work_bytes": (_sz, [_i64, _i64]),
    "sten_hilo_encode": (ctypes.c_int, [_vp, _vp, _i64, _i64, _i64, _vp]),
    "sten_hilo_decode": (ctypes.c_int, [_vp, _vp, _i64, _i64, _i64, _vp]),
    "sten_jacobi5_hilo": (ctypes.c_int, [_vp, _vp, _vp, _i64, _i64, _i64, _i32, _f64, _vp]),
    "sten_jacobi5_f64_hilo": (ctypes.c_int, [_vp, _vp, _vp, _sz, _i64, _i64, _i64, _i32, _f64, _vp]),
    "sten_tune_hilo_variant": (ctypes.c_int, [_i32]),
    "sten_batch_workspace_bytes": (_sz, [_i32]),
    "sten_batch_plan": (ctypes.c_int, [_vp, _i32, _i32, _f32, ctypes.c_char_p, _vp, _sz,
                                       ctypes.POINTER(_vp), _vp]),
    "sten_batch_run": (ctypes.c_int, [_vp, _vp]),
    "sten_batch_autotune": (ctypes.c_int, [_vp, ctypes.c_char_p, _i32, ctypes.POINTER(_f32), _vp]),
    "sten_batch_plan_info": (ctypes.c_int, [_vp, ctypes.POINTER(_i32), _i32]),
    "sten_batch_configure": (ctypes.c_int, [_vp, _i32, _i32, _i32, _vp]),
    "sten_batch_set_modes": (ctypes.c_int, [_vp, _i32, _vp]),
    "sten_batch_destroy": (ctypes.c_int, [_vp]),
    "sten_adjoint_partials_len": (_sz, [_i64, _i64]),
    "sten_jacobi5_f32_states": (ctypes.c_int, [_vp, _vp, _i64, _i64, _i64, _i32, _f32, _vp]),
    "sten_jacobi5_adjoint_f32": (ctypes.c_int, [_vp, _vp, _vp, _i64, _i64, _i64, _i32, _f32, _vp]),
    "sten_jacobi5_adjoint_f32_seg": (ctypes.c_int, [_vp, _vp, _i32, _vp, _vp, _vp, _i32, _i64, _i64, _i64,
                                                    _f32, _vp]),
    "sten_reduce_f64": (ctypes.c_int, [_vp, _i64, _vp, _vp]),
    "sten_jacobi5_adjoint_f32_seg_noalloc": (ctypes.c_int, [_vp, _vp, _i32, _vp, _vp, _i32, _vp, _i64, _i64, _i64,
                                                            _f32, _vp]),
    "sten_tiled_workspace_bytes": (_sz, [_i64, _i64, _i32, _i32]),
    "sten_tiled_create": (ctypes.c_int, [_i64, _i64, _i32, _i32, _vp, _sz, ctypes.POINTER(_vp)]),
    "sten_sweep_chain_f64": (ctypes.c_int, [_vp, _vp, _i64, _i64, _i64, _i32, _f64, _vp]),
    "sten_sweep_chain_last_f64": (ctypes.c_int, [_vp, _vp, _i64, _i64, _i64, _i32, _f64, _vp, _vp]),
    "sten_cavity_pressure_f64": (ctypes.c_int, [_vp, _vp, _vp, _vp, _i64, _i64, _i64, _i32, _f64, _f64, _f64, _i32,
                                                _vp]),
    "sten_tune_pressure": (ctypes.c_int, [_i32]),
    "sten_tune_adjoint_levels": (ctypes.c_int, [_i32]),
    "sten_tiled_workspace_bytes_ex": (_sz, [_i64, _i64, _i32, _i32, _i32, _i32]),
    "sten_tiled_create_ex": (ctypes.c_int, [_i64, _i64, _i32, _i32, _i32, _i32, _vp, _sz, ctypes.POINTER(_vp)]),
    "sten_tiled_plan_check": (ctypes.c_int, [_i64, _i64, _i32, _i32, _i32, _i32, ctypes.POINTER(ctypes.c_int64),
                                             _i32]),
    "sten_tiled_scatter": (ctypes.c_int, [_vp, _vp, _i64, _vp]),
    "sten_tiled_run": (ctypes.c_int, [_vp, _i32, _f64, _vp, _vp]),
    "sten_tiled_exchange": (ctypes.c_int, [_vp, _vp, _vp]),
    "sten_tiled_gather": (ctypes.c_int, [_vp, _vp, _i64, _vp]),
    "sten_tiled_stats": (ctypes.c_int, [_vp, ctypes.POINTER(ctypes.c_int64), _i32]),
    "sten_tiled_destroy": (ctypes.c_int, [_vp]),
    "sten_star_f64": (ctypes.c_int, [_vp, _vp, _vp, _i32, _i64, _i64, _i64, _vp]),
    "sten_star_iterate_f64": (ctypes.c_int, [_vp, _vp, _vp, _vp, _i64, _i64, _i64, _i32, _vp]),
    "sten_expr_run": (ctypes.c_int, [ctypes.c_char_p, _vp, _i32, _vp, _i32, _i64, _i64, _vp]),
    "sten_expr_source": (ctypes.c_int, [ctypes.c_char_p, _i32, _i32, _vp, _sz, ctypes.POINTER(_sz)]),
    "sten_expr_compile": (ctypes.c_int, [ctypes.c_char_p, _i32, _i32, ctypes.c_char_p]),
    "sten_expr_log": (ctypes.c_char_p, []),
}


class StarCoefC(ctypes.Structure):
    """Mirror of sten_star_coef in include/sten.h."""

    _fields_ = [("radius", _i32), ("reserved", _i32), ("c0", _f64), ("cn", _f64 * 4), ("cs", _f64 * 4),
                ("cw", _f64 * 4), ("ce", _f64 * 4)]


class StenExprIn(ctypes.Structure):
    """Mirror of sten_expr_in in include/sten.h."""

    _fields_ = [("base", _vp), ("ld", _i64), ("row_lo", _i64), ("row_hi", _i64), ("col_lo", _i64),
                ("col_hi", _i64)]


class StenExprOut(ctypes.Structure):
    """Mirror of sten_expr_out in include/sten.h."""

    _fields_ = [("base", _vp), ("ld", _i64)]


class StenInst(ctypes.Structure):
    """Mirror of sten_inst in include/sten.h."""

    _fields_ = [("u0", _vp), ("out", _vp), ("work", _vp), ("H", _i32), ("W", _i32), ("ld", _i32),
                ("reserved", _i32)]

_lib = None


def _hip_runtimes_mapped() -> list[str]:
    try:
        with open("/proc/self/maps") as f:
            paths = {line.split()[-1] for line in f if "libamdhip64" in line}
    except OSError:
        return []
    return sorted(paths)


def load():
    """Load libsten.so once; raise if it is missing or a second HIP runtime appears."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(
            f"{LIB_PATH} is not built; run `python -c 'import __graft_entry__ as g; g.build()'` "
            "(there is no CPU fallback)"
        )
    lib = ctypes.CDLL(LIB_PATH)
    runtimes = _hip_runtimes_mapped()
    if len(runtimes) > 1:
        raise RuntimeError(f"two HIP runtimes are mapped ({runtimes}); import torch before libsten")
    for name, (res, args) in SIGNATURES.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def declare(name: str, restype, argtypes) -> None:
    """Register the ctypes signature of a further entry point."""
    SIGNATURES[name] = (restype, argtypes)
    if _lib is not None:
        fn = getattr(_lib, name)
        fn.restype = restype
        fn.argtypes = argtypes


def check(fn_name: str, code: int) -> None:
    if code != 0:
        hip = load().sten_last_hip_error() if code == -5 else None
        raise StenError(fn_name, code, hip)


def call(fn_name: str, *args) -> None:
    """Call an entry point and raise StenError on a non-zero status."""
    check(fn_name, getattr(load(), fn_name)(*args))


def exported_symbols() -> list[str]:
    return list(SIGNATURES)
