"""torch.autograd binding of the FP32 method: gradients through the HIP adjoint kernels.

``jacobi5_autograd(u0, T, c)`` returns u_T = T sweeps of u0 and lets
torch.autograd compute dL/du0 (and dL/dc when c is a tensor that requires
grad). All forward, reverse and reduction steps run in libsten kernels; this
module only allocates buffers and sequences calls.

Memory: dL/dc needs the forward states u_0..u_{T-1}. When they fit in
`mem_budget` bytes they are recorded during the forward pass; otherwise only
checkpoints every ~sqrt(T) sweeps are kept and each segment's states are
recomputed in the backward pass. Both schedules run the same kernels in the
same order of accumulation, so they give the same bits.
"""

from __future__ import annotations

import ctypes
import math

import torch

from . import _lib
from .ops import _check_grid, _stream_ptr

DEFAULT_MEM_BUDGET = 1 << 30  # bytes of recorded forward states before checkpointing


def _empty_like_grid(t: torch.Tensor) -> torch.Tensor:
    return torch.empty_strided(t.shape, t.stride(), dtype=t.dtype, device=t.device)


def _copy_grid(src: torch.Tensor, dst: torch.Tensor) -> None:
    H, W = src.shape
    _lib.call("sten_jacobi5_f32", src.data_ptr(), dst.data_ptr(), None, H, W, W, 0, 0.0, _stream_ptr())


def _states(u0: torch.Tensor, T: int, c: float) -> torch.Tensor:
    """(T+1, H, W) tensor of u_0..u_T (contiguous planes)."""
    H, W = u0.shape
    st = torch.empty((T + 1, H, W), dtype=torch.float32, device=u0.device)
    _lib.call("sten_jacobi5_f32_states", u0.data_ptr(), st.data_ptr(), H, W, W, int(T), float(c), _stream_ptr())
    return st


def _forward_plain(u0: torch.Tensor, T: int, c: float) -> torch.Tensor:
    H, W = u0.shape
    out = _empty_like_grid(u0)
    work = _empty_like_grid(u0) if T >= 2 else None
    _lib.call("sten_jacobi5_f32", u0.data_ptr(), out.data_ptr(), work.data_ptr() if work is not None else None,
              H, W, W, int(T), float(c), _stream_ptr())
    return out


class Jacobi5Fn(torch.autograd.Function):
    """u_T = method(u0, T, c) in FP32 with a hand-written adjoint.

    forward(u0, c, T, mem_budget): u0 contiguous FP32 2-D CUDA tensor; c a
    Python float or a 0-d FP32 tensor (differentiable).
    """

    @staticmethod
    def forward(ctx, u0, c, T, mem_budget):
        T = int(T)
        cval = float(c.item()) if isinstance(c, torch.Tensor) else float(c)
        H, W = u0.shape
        ctx.T, ctx.cval, ctx.shape = T, cval, (H, W)
        ctx.c_is_tensor = isinstance(c, torch.Tensor)
        need_c = ctx.c_is_tensor and ctx.needs_input_grad[1]
        ctx.mode = "none"
        if not need_c:
            out = _forward_plain(u0, T, cval)
            return out
        plane = H * W * 4
        if (T + 1) * plane <= mem_budget:
            st = _states(u0, T, cval)
            out = _empty_like_grid(u0)
            _copy_grid(st[T], out)
            ctx.mode = "states"
            ctx.save_for_backward(st)
            return out
        # checkpoints every s sweeps: ckpt j holds u_{j*s}
        s = max(1, int(math.ceil(math.sqrt(T))))
        ckpts = [u0.detach().clone()]
        cur = ckpts[0]
        k = 0
        while k + s < T:
            cur = _forward_plain(cur, s, cval)
            ckpts.append(cur)
            k += s
        out = _forward_plain(cur, T - k, cval)
        ctx.mode = "checkpoints"
        ctx.seg = s
        ctx.save_for_backward(*ckpts)
        return out

    @staticmethod
    def backward(ctx, grad_out):
        T, cval = ctx.T, ctx.cval
        H, W = ctx.shape
        g = grad_out.to(torch.float32).contiguous()
        dev = g.device
        gin = torch.empty((H, W), dtype=torch.float32, device=dev)
        work = torch.empty((H, W), dtype=torch.float32, device=dev) if T >= 2 else None
        wptr = work.data_ptr() if work is not None else None
        grad_c = None
        if ctx.mode == "none":
            _lib.call("sten_jacobi5_adjoint_f32", g.data_ptr(), gin.data_ptr(), wptr, H, W, W, T, cval,
                      _stream_ptr())
            return gin, None, None, None
        nparts = int(_lib.load().sten_adjoint_partials_len(H, W))
        partials = torch.empty(nparts, dtype=torch.float64, device=dev)
        gc = torch.empty((), dtype=torch.float64, device=dev)
        if ctx.mode == "states":
            (st,) = ctx.saved_tensors
            _lib.call("sten_jacobi5_adjoint_f32_seg", g.data_ptr(), st.data_ptr(), T, gin.data_ptr(), wptr,
                      partials.data_ptr(), 1, H, W, W, cval, _stream_ptr())
        else:
            ckpts = ctx.saved_tensors
            s = ctx.seg
            lam_a = g
            lam_b = torch.empty((H, W), dtype=torch.float32, device=dev)
            lam_c = torch.empty((H, W), dtype=torch.float32, device=dev)
            first = True
            for j in range(len(ckpts) - 1, -1, -1):
                k0 = j * s
                n = min(s, T - k0)
                if n <= 0:
                    continue
                seg_states = _states(ckpts[j], n - 1, cval)  # u_{k0} .. u_{k0+n-1}
                dst = gin if j == 0 else (lam_b if lam_a is not lam_b else lam_c)
                _lib.call("sten_jacobi5_adjoint_f32_seg", lam_a.data_ptr(), seg_states.data_ptr(), n,
                          dst.data_ptr(), wptr, partials.data_ptr(), 1 if first else 0, H, W, W, cval,
                          _stream_ptr())
                first = False
                lam_a = dst
            if first:  # T == 0
                _lib.call("sten_jacobi5_adjoint_f32_seg", g.data_ptr(), None, 0, gin.data_ptr(), wptr,
                          partials.data_ptr(), 1, H, W, W, cval, _stream_ptr())
        _lib.call("sten_reduce_f64", partials.data_ptr(), nparts, gc.data_ptr(), _stream_ptr())
        grad_c = gc.to(torch.float32)
        return gin, grad_c, None, None


def jacobi5_autograd(u0: torch.Tensor, T: int, c=0.25, mem_budget: int = DEFAULT_MEM_BUDGET) -> torch.Tensor:
    """Differentiable T-sweep FP32 method. c: float, or a 0-d FP32 tensor to get dL/dc."""
    _check_grid(u0, torch.float32, "u0")
    if not u0.is_contiguous():
        u0 = u0.contiguous()
    return Jacobi5Fn.apply(u0, c, int(T), int(mem_budget))


def adjoint(gout: torch.Tensor, T: int, c: float = 0.25) -> torch.Tensor:
    """dL/du0 for dL/du_T = gout (FP32, contiguous): T transposed sweeps."""
    _check_grid(gout, torch.float32, "gout")
    g = gout.contiguous()
    H, W = g.shape
    gin = torch.empty_like(g)
    work = torch.empty_like(g) if T >= 2 else None
    _lib.call("sten_jacobi5_adjoint_f32", g.data_ptr(), gin.data_ptr(), work.data_ptr() if work is not None else None,
              H, W, W, int(T), float(c), _stream_ptr())
    return gin


def forward_states(u0: torch.Tensor, T: int, c: float = 0.25) -> torch.Tensor:
    """(T+1, H, W) tensor of every state of the FP32 method."""
    _check_grid(u0, torch.float32, "u0")
    return _states(u0.contiguous(), int(T), float(c))


__all__ = ["Jacobi5Fn", "jacobi5_autograd", "adjoint", "forward_states", "DEFAULT_MEM_BUDGET", "ctypes"]
