"""Lid-driven cavity flow written as NumPy-style slice assignments on the frontend.

The paper's second benchmark (Section V) is a cavity flow solved with the
incompressible Navier-Stokes equations, written in its NumPy-like syntax. This
module is that application on this repository's frontend: every update is a
slice assignment, so each becomes a DAG node, and nodes run as hand-written or
generated kernels (fusion of the u and v updates into one kernel included).

Method (explicit finite differences on H rows x W columns; row 0 is the bottom
wall, row H-1 the lid moving with u = 1):

1. source b = rho ((u_x + v_y) / dt - u_x^2 - 2 u_y v_x - v_y^2), central
   differences, interior only;
2. nit Jacobi iterations of p_xx + p_yy = b, each followed by dp/dx = 0 on the
   side walls, dp/dy = 0 on the bottom wall and p = 0 on the lid;
3. u, v: forward Euler, backward differences for convection, central
   differences for the pressure gradient and diffusion;
4. no-slip walls, lid row u = 1.

The frontend rejects an assignment that reads the array it writes (the
paper's rule), so the pressure iteration ping-pongs between two arrays and
each boundary row or column of the new iterate is evaluated directly from the
old one (the wall copies of the new iterate equal the interior formula one
cell inwards). Velocities ping-pong the same way.

With `blocked_pressure` (the default on the GPU backend, for grids of even
width >= 128), the nit pressure iterations of a step run as one library call
that applies several iterations per pass over HBM, walls included, with the
same bits as the per-iteration nodes; the frontend DAG is flushed to the
stream first, so the call sees b, and the nodes after it see its result.
"""

from __future__ import annotations

from .frontend import Context

__all__ = ["CavityFlow"]


class CavityFlow:
    """State and time stepping of the cavity on a frontend Context (FP64)."""

    def __init__(self, ctx: Context, H: int, W: int, lx: float = 2.0, ly: float = 2.0, rho: float = 1.0,
                 nu: float = 0.1, dt: float = 0.001, nit: int = 50, blocked_pressure: bool = True):
        if H < 3 or W < 3:
            raise ValueError("the cavity needs at least 3 x 3 points")
        self.ctx = ctx
        self.H, self.W = int(H), int(W)
        dx = lx / (W - 1)
        dy = ly / (H - 1)
        self.dx, self.dy, self.rho, self.nu, self.dt, self.nit = dx, dy, float(rho), float(nu), float(dt), int(nit)
        s = 2.0 * (dx * dx + dy * dy)
        self.cw = dy * dy / s
        self.cn = dx * dx / s
        self.cb = dx * dx * dy * dy / s
        self.cx = self.dt / dx
        self.cy = self.dt / dy
        self.cpx = self.dt / (2.0 * self.rho * dx)
        self.cpy = self.dt / (2.0 * self.rho * dy)
        self.kx = self.nu * self.dt / (dx * dx)
        self.ky = self.nu * self.dt / (dy * dy)
        shape = (self.H, self.W)
        self.u, self.u_next = ctx.create_array(shape), ctx.create_array(shape)
        self.v, self.v_next = ctx.create_array(shape), ctx.create_array(shape)
        self.p, self.p_next = ctx.create_array(shape), ctx.create_array(shape)
        self.b = ctx.create_array(shape)
        from .frontend import GpuBackend

        # the blocked kernel's layout: 16-byte vectors in strips of 128 columns
        self.blocked_pressure = bool(blocked_pressure) and isinstance(ctx.backend, GpuBackend) and \
            self.H >= 3 and self.W >= 128 and self.W % 2 == 0
        self._p_work = ctx.backend.alloc(shape) if self.blocked_pressure else None

    # -- one Jacobi update of the pressure, on rows [i0, i1) x columns [j0, j1) --------------------
    def _pressure_formula(self, p, i0: int, i1: int, j0: int, j1: int):
        b = self.b
        return self.cw * (p[i0:i1, j0 + 1:j1 + 1] + p[i0:i1, j0 - 1:j1 - 1]) \
            + self.cn * (p[i0 + 1:i1 + 1, j0:j1] + p[i0 - 1:i1 - 1, j0:j1]) - self.cb * b[i0:i1, j0:j1]

    def _pressure_iteration(self) -> None:
        H, W = self.H, self.W
        p, q = self.p, self.p_next
        f = self._pressure_formula
        q[1:H - 1, 1:W - 1] = f(p, 1, H - 1, 1, W - 1)   # interior
        q[1:H - 1, W - 1:W] = f(p, 1, H - 1, W - 2, W - 1)  # east wall: dp/dx = 0
        q[1:H - 1, 0:1] = f(p, 1, H - 1, 1, 2)             # west wall: dp/dx = 0
        q[0:1, 1:W - 1] = f(p, 1, 2, 1, W - 1)             # bottom wall: dp/dy = 0
        q[0:1, 0:1] = f(p, 1, 2, 1, 2)                     # bottom corners take the inner corner value
        q[0:1, W - 1:W] = f(p, 1, 2, W - 2, W - 1)
        q[H - 1:H, :] = 0.0                                # lid: p = 0
        self.p, self.p_next = q, p

    def step(self) -> None:
        """One time step (source, nit pressure iterations, velocities, walls)."""
        u, v, b = self.u, self.v, self.b
        dx, dy, dt, rho = self.dx, self.dy, self.dt, self.rho
        dudx = (u[1:-1, 2:] - u[1:-1, :-2]) / (2.0 * dx)
        dvdy = (v[2:, 1:-1] - v[:-2, 1:-1]) / (2.0 * dy)
        dudy = (u[2:, 1:-1] - u[:-2, 1:-1]) / (2.0 * dy)
        dvdx = (v[1:-1, 2:] - v[1:-1, :-2]) / (2.0 * dx)
        b[1:-1, 1:-1] = rho * ((dudx + dvdy) / dt - dudx * dudx - 2.0 * dudy * dvdx - dvdy * dvdy)
        if self.blocked_pressure:
            from . import ops

            self.ctx.flush()  # b's node goes to the stream before the call that reads it
            ops.cavity_pressure(self.p.data, self.b.data, self.nit, self.cw, self.cn, self.cb,
                                out=self.p_next.data, work=self._p_work)
            self.ctx.invalidate(self.p_next)  # written outside the frontend
            self.p, self.p_next = self.p_next, self.p
        else:
            for _ in range(self.nit):
                self._pressure_iteration()
        p = self.p
        un, vn, u2, v2 = self.u, self.v, self.u_next, self.v_next
        cx, cy, kx, ky = self.cx, self.cy, self.kx, self.ky
        C = un[1:-1, 1:-1]
        V = vn[1:-1, 1:-1]
        # the two updates have one output shape and no dependence: one fused generated kernel
        u2[1:-1, 1:-1] = C - cx * C * (C - un[1:-1, :-2]) - cy * V * (C - un[:-2, 1:-1]) \
            - self.cpx * (p[1:-1, 2:] - p[1:-1, :-2]) \
            + kx * (un[1:-1, 2:] - 2.0 * C + un[1:-1, :-2]) + ky * (un[2:, 1:-1] - 2.0 * C + un[:-2, 1:-1])
        v2[1:-1, 1:-1] = V - cx * C * (V - vn[1:-1, :-2]) - cy * V * (V - vn[:-2, 1:-1]) \
            - self.cpy * (p[2:, 1:-1] - p[:-2, 1:-1]) \
            + kx * (vn[1:-1, 2:] - 2.0 * V + vn[1:-1, :-2]) + ky * (vn[2:, 1:-1] - 2.0 * V + vn[:-2, 1:-1])
        u2[0, :] = 0.0
        u2[:, 0] = 0.0
        u2[:, -1] = 0.0
        u2[-1, :] = 1.0
        v2[0, :] = 0.0
        v2[-1, :] = 0.0
        v2[:, 0] = 0.0
        v2[:, -1] = 0.0
        self.u, self.u_next = u2, un
        self.v, self.v_next = v2, vn

    def run(self, nt: int) -> None:
        for _ in range(nt):
            self.step()

    def fields(self):
        """(u, v, p) backend arrays after everything queued so far has run."""
        self.ctx.sync()
        return self.u.data, self.v.data, self.p.data
