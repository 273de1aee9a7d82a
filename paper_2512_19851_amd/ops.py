"""Python entry points over libsten (argument marshalling only).

Every step of the computation runs in libsten's HIP kernels; torch provides
device memory and the current stream. Grids are 2-D tensors on the current
HIP device, row-major with unit column stride (row stride = tensor.stride(0)).
"""

from __future__ import annotations

import torch

from . import _lib


def _stream_ptr(stream=None) -> int:
    s = stream if stream is not None else torch.cuda.current_stream()
    return int(s.cuda_stream)


def _check_grid(t: torch.Tensor, dtype, name: str) -> None:
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name} must be a torch.Tensor")
    if t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}, got {t.dtype}")
    if t.dim() != 2:
        raise ValueError(f"{name} must be 2-D")
    if not t.is_cuda:
        raise ValueError(f"{name} must be on the GPU (libsten has no CPU path)")
    if t.numel() > 0 and t.stride(1) != 1:
        raise ValueError(f"{name} must have unit column stride")


def _ld(t: torch.Tensor) -> int:
    return int(t.stride(0)) if t.shape[0] > 1 else int(max(t.shape[1], 1))


def jacobi5(u0: torch.Tensor, T: int, c: float = 0.25, out: torch.Tensor | None = None,
            work: torch.Tensor | None = None, stream=None) -> torch.Tensor:
    """T five-point Jacobi sweeps of u0 (FP64 or FP32) on the GPU; returns the result grid.

    The method of the listing of the Laplace solver (Section III-A): the ring
    is kept, each interior point becomes c*(((N+S)+W)+E), buffers swap each
    sweep. `out` and `work` (same shape/stride as u0) are allocated when not given.
    """
    if u0.dtype == torch.float64:
        fn = "sten_jacobi5_f64"
    elif u0.dtype == torch.float32:
        fn = "sten_jacobi5_f32"
    else:
        raise TypeError("u0 must be float32 or float64")
    _check_grid(u0, u0.dtype, "u0")
    H, W = u0.shape
    if out is None:
        out = torch.empty_strided(u0.shape, u0.stride(), dtype=u0.dtype, device=u0.device)
    _check_grid(out, u0.dtype, "out")
    if out.shape != u0.shape or (H > 1 and out.stride() != u0.stride()):
        raise ValueError("out must match u0's shape and strides")
    need_work = T >= 2 and H >= 3 and W >= 3
    if work is None and need_work:
        work = torch.empty_strided(u0.shape, u0.stride(), dtype=u0.dtype, device=u0.device)
    if work is not None:
        _check_grid(work, u0.dtype, "work")
        if work.shape != u0.shape or (H > 1 and work.stride() != u0.stride()):
            raise ValueError("work must match u0's shape and strides")
    _lib.call(fn, u0.data_ptr(), out.data_ptr(), work.data_ptr() if work is not None else None,
              H, W, _ld(u0), int(T), float(c), _stream_ptr(stream))
    return out


def jacobi5_tb(u0: torch.Tensor, T: int, c: float = 0.25, levels: int = 2, out: torch.Tensor | None = None,
               work: torch.Tensor | None = None, stream=None) -> torch.Tensor:
    """Temporally blocked method: `levels` sweeps per HBM pass, bit-identical to `jacobi5`.

    Grids the blocked kernels do not handle (misaligned, no interior, T = 0) go
    through the single-sweep path.
    """
    fn = {torch.float64: "sten_jacobi5_f64_tb", torch.float32: "sten_jacobi5_f32_tb"}.get(u0.dtype)
    if fn is None:
        raise TypeError("u0 must be float32 or float64")
    _check_grid(u0, u0.dtype, "u0")
    H, W = u0.shape
    if out is None:
        out = torch.empty_strided(u0.shape, u0.stride(), dtype=u0.dtype, device=u0.device)
    if work is None and T > levels and H >= 3 and W >= 3:
        work = torch.empty_strided(u0.shape, u0.stride(), dtype=u0.dtype, device=u0.device)
    code = getattr(_lib.load(), fn)(u0.data_ptr(), out.data_ptr(), work.data_ptr() if work is not None else None,
                                    H, W, _ld(u0), int(T), float(c), int(levels), _stream_ptr(stream))
    if code == -6:
        return jacobi5(u0, T, c, out=out, work=work, stream=stream)
    _lib.check(fn, code)
    return out


def set_schedule(levels: int) -> None:
    """Sweeps per launch of `jacobi5` (1: one per launch; 2..14: temporal blocking, FP32 at most 12; 0: built-in)."""
    _lib.call("sten_tune_schedule", int(levels))


def set_tb(variant: int = 0, band: int = 0, depth: int = 0) -> None:
    """Tuning hook for the temporally blocked kernels (0 everywhere restores the built-in choice).

    variant: 1 = register tile (levels 1..6), 2 = streaming (levels 1..12);
    band: output rows per streaming band; depth: rows the streaming kernel loads ahead (0 or 4).
    """
    _lib.call("sten_tune_tb", int(variant), int(band), int(depth))


def set_tb_rows(rows: int) -> None:
    """Tuning hook: output rows per temporally blocked tile (4, 8, 12, 16; 0 = built-in)."""
    _lib.call("sten_tune_tb_rows", int(rows))


def sweep(src: torch.Tensor, dst: torch.Tensor, c: float = 0.25, stream=None) -> torch.Tensor:
    """One sweep: dst's interior from src (dst's ring untouched); returns dst."""
    fn = {torch.float64: "sten_sweep_f64", torch.float32: "sten_sweep_f32"}.get(src.dtype)
    if fn is None:
        raise TypeError("src must be float32 or float64")
    _check_grid(src, src.dtype, "src")
    _check_grid(dst, src.dtype, "dst")
    if dst.shape != src.shape or (src.shape[0] > 1 and dst.stride() != src.stride()):
        raise ValueError("dst must match src's shape and strides")
    H, W = src.shape
    _lib.call(fn, src.data_ptr(), dst.data_ptr(), H, W, _ld(src), float(c), _stream_ptr(stream))
    return dst


def set_sweep_rows(rows: int) -> None:
    """Tuning hook: rows per tile of the sweep kernels (4, 8, 16; 0 = built-in)."""
    _lib.call("sten_tune_sweep_rows", int(rows))


# ---------------------------------------------------------------------------
# hi/lo reduced-precision form
# ---------------------------------------------------------------------------

def cavity_pressure(p0: torch.Tensor, b: torch.Tensor, nit: int, cw: float, cn: float, cb: float, levels: int = 0,
                    out: torch.Tensor | None = None, work: torch.Tensor | None = None,
                    stream=None) -> torch.Tensor:
    """nit pressure iterations of the lid-driven cavity flow (interior update, then the wall conditions), up to
    `levels` (1..12, 0 = 12) per pass over HBM; bit-identical to one iteration at a time. FP64 grids of one
    shape and stride. Raises StenError with name STEN_ERR_UNSUPPORTED for layouts the blocked kernel does not
    take (fewer than 3 rows or 128 columns, odd width or stride, unaligned data)."""
    for t, name in ((p0, "p0"), (b, "b")):
        _check_grid(t, torch.float64, name)
    if b.shape != p0.shape or (p0.shape[0] > 1 and b.stride() != p0.stride()):
        raise ValueError("b must match p0's shape and strides")
    H, W = p0.shape
    if out is None:
        out = torch.empty_strided(p0.shape, p0.stride(), dtype=p0.dtype, device=p0.device)
    lev = levels if levels > 0 else 12
    if work is None and nit > lev:
        work = torch.empty_strided(p0.shape, p0.stride(), dtype=p0.dtype, device=p0.device)
    for t, name in ((out, "out"), (work, "work")):
        if t is None:
            continue
        _check_grid(t, torch.float64, name)
        if t.shape != p0.shape or (H > 1 and t.stride() != p0.stride()):
            raise ValueError(f"{name} must match p0's shape and strides")
    _lib.call("sten_cavity_pressure_f64", p0.data_ptr(), b.data_ptr(), out.data_ptr(),
              work.data_ptr() if work is not None else None, H, W, _ld(p0), int(nit), float(cw), float(cn),
              float(cb), int(levels), _stream_ptr(stream))
    return out


def set_pressure_band(band: int) -> None:
    """Rows per band of the blocked pressure kernel (0: built-in). Results are unchanged."""
    _lib.call("sten_tune_pressure", int(band))


def set_adjoint_levels(levels: int) -> None:
    """Transposed steps per launch of the several-step adjoint kernel (1..8; 0: built-in). Results are
    unchanged."""
    _lib.call("sten_tune_adjoint_levels", int(levels))


class HiLoGrid:
    """An encoded grid in a device byte buffer: FP32 hi plane + int16 q plane."""

    def __init__(self, buf: torch.Tensor, H: int, W: int, ld: int):
        self.buf, self.H, self.W, self.ld = buf, H, W, ld

    @property
    def q_offset(self) -> int:
        return (self.H * self.ld * 4 + 255) // 256 * 256

    def hi(self) -> torch.Tensor:
        n = self.H * self.ld
        return self.buf[: n * 4].view(torch.float32).view(self.H, self.ld)[:, : self.W]

    def q(self) -> torch.Tensor:
        n = self.H * self.ld
        o = self.q_offset
        return self.buf[o: o + n * 2].view(torch.int16).view(self.H, self.ld)[:, : self.W]


def hilo_empty(H: int, W: int, ld: int | None = None, device=None) -> HiLoGrid:
    ld = W if ld is None else ld
    nbytes = int(_lib.load().sten_hilo_bytes(H, ld))
    buf = torch.empty(max(nbytes, 1), dtype=torch.uint8, device=device or torch.device("cuda"))
    return HiLoGrid(buf, H, W, ld)


def hilo_encode(x: torch.Tensor, out: HiLoGrid | None = None, stream=None) -> HiLoGrid:
    """FP64 grid -> encoded grid (hi = RN32(x), q = rint((x - hi) / delta(hi))), into `out` when given."""
    _check_grid(x, torch.float64, "x")
    H, W = x.shape
    g = out if out is not None else hilo_empty(H, W, _ld(x), x.device)
    if (g.H, g.W, g.ld) != (H, W, _ld(x)):
        raise ValueError("out must be an encoded grid of x's shape and row stride")
    _lib.call("sten_hilo_encode", x.data_ptr(), g.buf.data_ptr(), H, W, g.ld, _stream_ptr(stream))
    return g


def hilo_decode(g: HiLoGrid, out: torch.Tensor | None = None, stream=None) -> torch.Tensor:
    """Encoded grid -> FP64 (exact)."""
    if out is None:
        out = torch.empty_strided((g.H, g.W), (g.ld, 1), dtype=torch.float64, device=g.buf.device)
    _check_grid(out, torch.float64, "out")
    _lib.call("sten_hilo_decode", g.buf.data_ptr(), out.data_ptr(), g.H, g.W, g.ld, _stream_ptr(stream))
    return out


def jacobi5_hilo_encoded(src: HiLoGrid, T: int, c: float = 0.25, dst: HiLoGrid | None = None,
                         work: HiLoGrid | None = None, stream=None) -> HiLoGrid:
    """T sweeps on encoded grids (state stays encoded between calls)."""
    dev = src.buf.device
    if dst is None:
        dst = hilo_empty(src.H, src.W, src.ld, dev)
    if work is None and T >= 2:
        work = hilo_empty(src.H, src.W, src.ld, dev)
    _lib.call("sten_jacobi5_hilo", src.buf.data_ptr(), dst.buf.data_ptr(),
              work.buf.data_ptr() if work is not None else None,
              src.H, src.W, src.ld, int(T), float(c), _stream_ptr(stream))
    return dst


def jacobi5_hilo(u0: torch.Tensor, T: int, c: float = 0.25, out: torch.Tensor | None = None,
                 work: torch.Tensor | None = None, stream=None) -> torch.Tensor:
    """FP64 in/out through the hi/lo form: encode, T encoded sweeps, decode (ring exact)."""
    _check_grid(u0, torch.float64, "u0")
    H, W = u0.shape
    ld = _ld(u0)
    if out is None:
        out = torch.empty_strided(u0.shape, u0.stride(), dtype=torch.float64, device=u0.device)
    _check_grid(out, torch.float64, "out")
    need = int(_lib.load().sten_jacobi5_f64_hilo_work_bytes(H, ld))
    if work is None:
        work = torch.empty(max(need, 1), dtype=torch.uint8, device=u0.device)
    _lib.call("sten_jacobi5_f64_hilo", u0.data_ptr(), out.data_ptr(), work.data_ptr(), work.numel(),
              H, W, ld, int(T), float(c), _stream_ptr(stream))
    return out


def hilo_work_bytes(H: int, W: int, ld: int | None = None) -> int:
    return int(_lib.load().sten_jacobi5_f64_hilo_work_bytes(H, W if ld is None else ld))


def set_hilo_variant(variant: int) -> None:
    """Tuning hook: kernel variant of the hi/lo sweep (1..10, see sten.h; 0 = built-in)."""
    _lib.call("sten_tune_hilo_variant", int(variant))


# ---------------------------------------------------------------------------
# Batched form: many grids, one persistent launch
# ---------------------------------------------------------------------------

class BatchPlan:
    """A plan over a list of FP32 grids (u0 tensors) with their out/work tensors.

    plan = BatchPlan(u0s, T, c, tune_cache=path)  # allocates outs, works, workspace
    plan.run()                                      # one persistent launch (graph-capturable)
    plan.outs                                       # results
    """

    def __init__(self, u0s, T: int, c: float = 0.25, outs=None, works=None, tune_cache: str | None = None,
                 stream=None):
        import ctypes

        lib = _lib.load()
        self.T, self.c = int(T), float(c)
        self.u0s = list(u0s)
        for k, t in enumerate(self.u0s):
            _check_grid(t, torch.float32, f"u0s[{k}]")
        dev = self.u0s[0].device if self.u0s else torch.device("cuda")
        self.outs = outs if outs is not None else [torch.empty_like(t) for t in self.u0s]
        if works is None:
            works = [torch.empty_like(t) if (T >= 2 and t.shape[0] >= 3 and t.shape[1] >= 3) else None
                     for t in self.u0s]
        self.works = works
        n = len(self.u0s)
        arr = (_lib.StenInst * max(n, 1))()
        for k in range(n):
            u, o, w = self.u0s[k], self.outs[k], self.works[k]
            arr[k].u0 = u.data_ptr()
            arr[k].out = o.data_ptr()
            arr[k].work = w.data_ptr() if w is not None else None
            arr[k].H, arr[k].W = int(u.shape[0]), int(u.shape[1])
            arr[k].ld = _ld(u)
            arr[k].reserved = 0
        self._arr = arr
        nbytes = int(lib.sten_batch_workspace_bytes(n))
        self.ws = torch.empty(max(nbytes, 256), dtype=torch.uint8, device=dev)
        self._handle = ctypes.c_void_p()
        path = tune_cache.encode() if tune_cache else None
        _lib.check("sten_batch_plan", lib.sten_batch_plan(ctypes.cast(arr, ctypes.c_void_p), n, self.T, self.c,
                                                          path, self.ws.data_ptr(), self.ws.numel(),
                                                          ctypes.byref(self._handle), _stream_ptr(stream)))

    def run(self, stream=None) -> list:
        _lib.call("sten_batch_run", self._handle, _stream_ptr(stream))
        return self.outs

    def autotune(self, tune_cache: str | None = None, reps: int = 3, stream=None) -> float:
        import ctypes

        best = ctypes.c_float(0.0)
        path = tune_cache.encode() if tune_cache else None
        _lib.call("sten_batch_autotune", self._handle, path, int(reps), ctypes.byref(best), _stream_ptr(stream))
        return float(best.value)

    def configure(self, block: int, lds_bytes: int, wg_per_cu: int = 1, stream=None) -> None:
        """Set block size, LDS budget per workgroup and workgroups per CU explicitly."""
        _lib.call("sten_batch_configure", self._handle, int(block), int(lds_bytes), int(wg_per_cu),
                  _stream_ptr(stream))

    def set_register_mode(self, on: bool, stream=None) -> None:
        """Register-resident mode for grids that fit (on by default)."""
        _lib.call("sten_batch_set_modes", self._handle, 1 if on else 0, _stream_ptr(stream))

    def info(self) -> dict:
        import ctypes

        buf = (ctypes.c_int32 * 9)()
        _lib.call("sten_batch_plan_info", self._handle, buf, 9)
        keys = ["block", "lds_bytes", "wg_per_cu", "grid", "n_lds", "n_global", "n_copy", "n_reg", "use_reg"]
        return dict(zip(keys, list(buf)))

    def close(self) -> None:
        if getattr(self, "_handle", None) is not None and self._handle.value:
            _lib.load().sten_batch_destroy(self._handle)
            self._handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ---------------------------------------------------------------------------
# Tiled execution on one GPU (chares with ghost exchange)
# ---------------------------------------------------------------------------

class TiledGrid:
    """An H x W FP64 grid split into pr x pc tiles with ghost frames of depth `ghost`, on one GPU.

    t = TiledGrid(H, W, pr, pc); t.scatter(u); t.run(T, c); u2 = t.gather()
    `ghost` (1..12) is the number of sweeps a tile runs between two ghost exchanges.
    `exchange` is "packed" (pack and unpack kernels through send buffers) or "direct" (one copy kernel
    from each neighbour's boundary block into the ghost frame).
    `comm_stream` (optional) carries the ghost exchanges; sweeps go on the current stream.
    """

    MODES = {"packed": 0, "direct": 1}

    def __init__(self, H: int, W: int, pr: int, pc: int, device=None, comm_stream=None, ghost: int = 1,
                 exchange: str = "packed"):
        import ctypes

        lib = _lib.load()
        if exchange not in self.MODES:
            raise ValueError(f"exchange must be one of {sorted(self.MODES)}")
        self.H, self.W, self.pr, self.pc, self.ghost = int(H), int(W), int(pr), int(pc), int(ghost)
        self.mode = self.MODES[exchange]
        nbytes = int(lib.sten_tiled_workspace_bytes_ex(self.H, self.W, self.pr, self.pc, self.ghost, self.mode))
        if nbytes == 0:
            raise ValueError("invalid tiling")
        self.ws = torch.empty(nbytes, dtype=torch.uint8, device=device or torch.device("cuda"))
        self.comm_stream = comm_stream
        self._h = ctypes.c_void_p()
        _lib.check("sten_tiled_create_ex",
                   lib.sten_tiled_create_ex(self.H, self.W, self.pr, self.pc, self.ghost, self.mode,
                                            self.ws.data_ptr(), nbytes, ctypes.byref(self._h)))

    def _comm(self) -> int:
        return _stream_ptr(self.comm_stream) if self.comm_stream is not None else _stream_ptr()

    def scatter(self, u: torch.Tensor) -> None:
        _check_grid(u, torch.float64, "u")
        if tuple(u.shape) != (self.H, self.W):
            raise ValueError("shape mismatch")
        _lib.call("sten_tiled_scatter", self._h, u.data_ptr(), _ld(u), _stream_ptr())

    def run(self, T: int, c: float = 0.25) -> None:
        _lib.call("sten_tiled_run", self._h, int(T), float(c), _stream_ptr(), self._comm())

    def exchange(self) -> None:
        _lib.call("sten_tiled_exchange", self._h, _stream_ptr(), self._comm())

    def gather(self, out: torch.Tensor | None = None) -> torch.Tensor:
        if out is None:
            out = torch.empty((self.H, self.W), dtype=torch.float64, device=self.ws.device)
        _check_grid(out, torch.float64, "out")
        _lib.call("sten_tiled_gather", self._h, out.data_ptr(), _ld(out), _stream_ptr())
        return out

    def stats(self) -> dict:
        import ctypes

        buf = (ctypes.c_int64 * 7)()
        _lib.call("sten_tiled_stats", self._h, buf, 7)
        return dict(zip(["tiles", "exchanges", "skipped", "sweep_launches", "strips", "ghost", "mode"], list(buf)))

    def close(self) -> None:
        if getattr(self, "_h", None) is not None and self._h.value:
            _lib.load().sten_tiled_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ---------------------------------------------------------------------------
# General star stencils with node fusion
# ---------------------------------------------------------------------------

def _star_coef(spec):
    """spec = (c0, cn, cs, cw, ce) with four equal-length lists (the radius)."""
    c0, cn, cs, cw, ce = spec
    R = len(cn)
    if not (1 <= R <= 4 and len(cs) == len(cw) == len(ce) == R):
        raise ValueError("a star stencil needs radius 1..4 and four lists of that length")
    s = _lib.StarCoefC()
    s.radius = R
    s.c0 = float(c0)
    for k in range(R):
        s.cn[k], s.cs[k], s.cw[k], s.ce[k] = float(cn[k]), float(cs[k]), float(cw[k]), float(ce[k])
    return s


def star(u: torch.Tensor, specs, outs=None, stream=None) -> list:
    """Apply 1..4 star stencils of one radius to u in one fused kernel; returns the outputs.

    Each output starts as a copy of u (so its frame of width R is u's) unless `outs` is given.
    """
    import ctypes

    _check_grid(u, torch.float64, "u")
    specs = list(specs)
    if outs is None:
        outs = [u.clone() for _ in specs]
    coefs = (_lib.StarCoefC * len(specs))(*[_star_coef(sp) for sp in specs])
    ptrs = (ctypes.c_void_p * len(specs))(*[o.data_ptr() for o in outs])
    H, W = u.shape
    _lib.call("sten_star_f64", u.data_ptr(), ctypes.cast(ptrs, ctypes.c_void_p), ctypes.cast(coefs, ctypes.c_void_p),
              len(specs), H, W, _ld(u), _stream_ptr(stream))
    return outs


def star_iterate(u0: torch.Tensor, T: int, spec, out=None, work=None, stream=None) -> torch.Tensor:
    """T applications of one star stencil with a ping-pong swap."""
    import ctypes

    _check_grid(u0, torch.float64, "u0")
    coef = _star_coef(spec)
    out = out if out is not None else torch.empty_like(u0)
    if work is None and T >= 2:
        work = torch.empty_like(u0)
    H, W = u0.shape
    _lib.call("sten_star_iterate_f64", u0.data_ptr(), out.data_ptr(), work.data_ptr() if work is not None else None,
              ctypes.cast(ctypes.pointer(coef), ctypes.c_void_p), H, W, _ld(u0), int(T), _stream_ptr(stream))
    return out


# ---------------------------------------------------------------------------
# Generated kernels for slice expressions
# ---------------------------------------------------------------------------

def expr_source(program: str, nin: int, nout: int) -> str:
    """The HIP source libsten generates for an expression program (host only, no GPU)."""
    import ctypes

    n = ctypes.c_size_t(0)
    _lib.check("sten_expr_source", _lib.load().sten_expr_source(program.encode(), nin, nout, None, 0,
                                                                 ctypes.byref(n)))
    buf = ctypes.create_string_buffer(n.value + 1)
    _lib.call("sten_expr_source", program.encode(), nin, nout, ctypes.cast(buf, ctypes.c_void_p), n.value + 1,
              ctypes.byref(n))
    return buf.value.decode()


def expr_compile(program: str, nin: int, nout: int, arch: str = "gfx950") -> None:
    """Compile an expression program with the run-time compiler (host only, no GPU); raises on failure."""
    code = _lib.load().sten_expr_compile(program.encode(), nin, nout, arch.encode())
    if code != 0:
        raise _lib.StenError("sten_expr_compile", code, None) from RuntimeError(expr_log())


def expr_log() -> str:
    """The last expression-program or compiler message of this thread."""
    return _lib.load().sten_expr_log().decode()


def expr_run(program: str, ins, outs, rows: int, cols: int, stream=None) -> None:
    """Run an expression program over a rows x cols region.

    ins / outs: lists of (tensor, r0, c0): FP64 grids and the element of each that is aligned with
    output point (0, 0). Input extents are the whole tensors; libsten checks every load against them.
    """
    import ctypes

    ia = (_lib.StenExprIn * max(1, len(ins)))()
    for k, (t, r0, c0) in enumerate(ins):
        _check_grid(t, torch.float64, f"input {k}")
        H, W = t.shape
        ld = _ld(t)
        ia[k].base = t.data_ptr() + (r0 * ld + c0) * 8
        ia[k].ld = ld
        ia[k].row_lo, ia[k].row_hi = -r0, H - 1 - r0
        ia[k].col_lo, ia[k].col_hi = -c0, W - 1 - c0
    oa = (_lib.StenExprOut * max(1, len(outs)))()
    for k, (t, r0, c0) in enumerate(outs):
        _check_grid(t, torch.float64, f"output {k}")
        H, W = t.shape
        if r0 < 0 or c0 < 0 or r0 + rows > H or c0 + cols > W:
            raise ValueError(f"output {k}: region leaves the array")
        ld = _ld(t)
        oa[k].base = t.data_ptr() + (r0 * ld + c0) * 8
        oa[k].ld = ld
    code = _lib.load().sten_expr_run(program.encode(), ctypes.cast(ia, ctypes.c_void_p), len(ins),
                                     ctypes.cast(oa, ctypes.c_void_p), len(outs), int(rows), int(cols),
                                     _stream_ptr(stream))
    if code != 0:
        raise _lib.StenError("sten_expr_run", code, _lib.load().sten_last_hip_error() if code == -5 else None) \
            from RuntimeError(expr_log())
