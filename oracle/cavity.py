"""CPU oracle for the lid-driven cavity flow step (test infrastructure).

TEST INFRASTRUCTURE. Only the test suite, the smoke check and the benchmark's
CPU-baseline leg may use this module. It shares no code with the GPU library.

The paper's second benchmark (Section V, weak scaling) is a cavity flow solved
with the incompressible Navier-Stokes equations, written as NumPy-style slice
assignments (16k x 16k per GPU, 50 iterations). Its source program is cited,
not printed, so this module states the standard explicit finite-difference
method for that problem, from the equations:

    u_t + u u_x + v u_y = -p_x / rho + nu (u_xx + u_yy)
    v_t + u v_x + v v_y = -p_y / rho + nu (v_xx + v_yy)
    p_xx + p_yy = b,  b = rho ((u_x + v_y) / dt - u_x^2 - 2 u_y v_x - v_y^2)

on a grid of H rows (y, row 0 at the bottom, row H-1 the moving lid) by W
columns (x), spacings dx, dy. One time step:

1. b on the interior from (u, v) with central differences;
2. nit Jacobi iterations of the pressure equation on the interior, each
   followed by the boundary conditions dp/dx = 0 on the side walls (edge column
   := its inner neighbour), dp/dy = 0 on the bottom wall (row 0 := row 1, after
   the side walls, so corners take the inner corner value) and p = 0 on the lid;
3. u and v on the interior from the old (u, v) and the new p: forward Euler in
   time, backward (upwind for positive velocity) differences for convection,
   central differences for the pressure gradient and the diffusion;
4. walls: u = v = 0 on rows 0 and the side columns, v = 0 and u = 1 on the lid
   row (set last, so the lid row's corners have u = 1).

Every update is one slice expression evaluated by NumPy left to right in FP64,
with scalar factors computed once in Python; the expressions below are the
definition of the method used everywhere in this repository.
"""

from __future__ import annotations

import numpy as np

__all__ = ["CavityParams", "source_term", "pressure_iteration", "momentum", "apply_velocity_walls", "step",
           "run"]


class CavityParams:
    """Physical and numerical parameters; scalar factors of the update formulas."""

    def __init__(self, H: int, W: int, lx: float = 2.0, ly: float = 2.0, rho: float = 1.0, nu: float = 0.1,
                 dt: float = 0.001, nit: int = 50):
        if H < 3 or W < 3:
            raise ValueError("the cavity needs at least 3 x 3 points")
        self.H, self.W = int(H), int(W)
        self.dx = lx / (W - 1)
        self.dy = ly / (H - 1)
        self.rho, self.nu, self.dt, self.nit = float(rho), float(nu), float(dt), int(nit)
        dx, dy = self.dx, self.dy
        s = 2.0 * (dx * dx + dy * dy)
        self.cw = dy * dy / s           # weight of the east + west pressure neighbours
        self.cn = dx * dx / s           # weight of the north + south pressure neighbours
        self.cb = dx * dx * dy * dy / s  # weight of the source term
        self.cx = self.dt / dx           # convection, x
        self.cy = self.dt / dy           # convection, y
        self.cpx = self.dt / (2.0 * self.rho * dx)  # pressure gradient in the u equation
        self.cpy = self.dt / (2.0 * self.rho * dy)  # pressure gradient in the v equation
        self.kx = self.nu * self.dt / (dx * dx)     # diffusion, x
        self.ky = self.nu * self.dt / (dy * dy)     # diffusion, y


def source_term(u: np.ndarray, v: np.ndarray, prm: CavityParams) -> np.ndarray:
    """b on the interior (zero on the boundary ring)."""
    dx, dy, dt, rho = prm.dx, prm.dy, prm.dt, prm.rho
    b = np.zeros_like(u)
    dudx = (u[1:-1, 2:] - u[1:-1, :-2]) / (2.0 * dx)
    dvdy = (v[2:, 1:-1] - v[:-2, 1:-1]) / (2.0 * dy)
    dudy = (u[2:, 1:-1] - u[:-2, 1:-1]) / (2.0 * dy)
    dvdx = (v[1:-1, 2:] - v[1:-1, :-2]) / (2.0 * dx)
    b[1:-1, 1:-1] = rho * ((dudx + dvdy) / dt - dudx * dudx - 2.0 * dudy * dvdx - dvdy * dvdy)
    return b


def pressure_iteration(p: np.ndarray, b: np.ndarray, prm: CavityParams) -> np.ndarray:
    """One Jacobi iteration of the pressure equation, then the pressure boundary conditions."""
    pn = p.copy()
    q = p.copy()
    q[1:-1, 1:-1] = prm.cw * (pn[1:-1, 2:] + pn[1:-1, :-2]) + prm.cn * (pn[2:, 1:-1] + pn[:-2, 1:-1]) \
        - prm.cb * b[1:-1, 1:-1]
    q[1:-1, -1] = q[1:-1, -2]  # dp/dx = 0, east wall
    q[1:-1, 0] = q[1:-1, 1]    # dp/dx = 0, west wall
    q[0, :] = q[1, :]          # dp/dy = 0, bottom wall
    q[-1, :] = 0.0             # p = 0, lid
    return q


def momentum(u: np.ndarray, v: np.ndarray, p: np.ndarray, prm: CavityParams) -> tuple:
    """New u and v on the interior (boundary ring copied from the old fields)."""
    un, vn = u, v
    cx, cy, kx, ky = prm.cx, prm.cy, prm.kx, prm.ky
    C = un[1:-1, 1:-1]
    V = vn[1:-1, 1:-1]
    u2 = un.copy()
    v2 = vn.copy()
    u2[1:-1, 1:-1] = C - cx * C * (C - un[1:-1, :-2]) - cy * V * (C - un[:-2, 1:-1]) \
        - prm.cpx * (p[1:-1, 2:] - p[1:-1, :-2]) \
        + kx * (un[1:-1, 2:] - 2.0 * C + un[1:-1, :-2]) + ky * (un[2:, 1:-1] - 2.0 * C + un[:-2, 1:-1])
    v2[1:-1, 1:-1] = V - cx * C * (V - vn[1:-1, :-2]) - cy * V * (V - vn[:-2, 1:-1]) \
        - prm.cpy * (p[2:, 1:-1] - p[:-2, 1:-1]) \
        + kx * (vn[1:-1, 2:] - 2.0 * V + vn[1:-1, :-2]) + ky * (vn[2:, 1:-1] - 2.0 * V + vn[:-2, 1:-1])
    return u2, v2


def apply_velocity_walls(u: np.ndarray, v: np.ndarray) -> None:
    """No-slip walls; the lid (last row) moves with u = 1."""
    u[0, :] = 0.0
    u[:, 0] = 0.0
    u[:, -1] = 0.0
    u[-1, :] = 1.0
    v[0, :] = 0.0
    v[-1, :] = 0.0
    v[:, 0] = 0.0
    v[:, -1] = 0.0


def step(u: np.ndarray, v: np.ndarray, p: np.ndarray, prm: CavityParams) -> tuple:
    """One time step; returns the new (u, v, p)."""
    b = source_term(u, v, prm)
    for _ in range(prm.nit):
        p = pressure_iteration(p, b, prm)
    u2, v2 = momentum(u, v, p, prm)
    apply_velocity_walls(u2, v2)
    return u2, v2, p


def run(nt: int, prm: CavityParams, u=None, v=None, p=None) -> tuple:
    """nt time steps from rest (zero fields) unless initial fields are given."""
    H, W = prm.H, prm.W
    u = np.zeros((H, W)) if u is None else np.array(u, dtype=np.float64, copy=True)
    v = np.zeros((H, W)) if v is None else np.array(v, dtype=np.float64, copy=True)
    p = np.zeros((H, W)) if p is None else np.array(p, dtype=np.float64, copy=True)
    for _ in range(nt):
        u, v, p = step(u, v, p, prm)
    return u, v, p
