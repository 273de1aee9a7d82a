"""Pins for the cavity-flow oracle (CPU), and the frontend program checked against it.

The oracle's difference operators are exact on low-degree polynomials:
central differences on linear and quadratic fields, backward differences on
linear fields, second differences on quadratics. On dyadic grids (power-of-two
spacings, small integer coefficients) every FP64 operation is then exact too,
so each update has a closed form that the oracle must reproduce bit for bit.
The pressure iteration's fixed point must solve the five-point Poisson system
with the walls' conditions, assembled here from the PDE and solved directly.
Planted mistakes in a copy of the oracle fail these pins.
"""

from fractions import Fraction

import numpy as np
import pytest

from oracle import cavity as oc
from paper_2512_19851_amd import frontend as fe
from paper_2512_19851_amd.cavity import CavityFlow
from tests.numpy_backend import NumpyBackend


def dyadic_params(H=9, W=11, square=False, **kw):
    # dx = 1/8; dy = 1/16 (or 1/8 when square): lx = (W-1)/8, ly = (H-1)/16
    ly = (H - 1) / 8.0 if square else (H - 1) / 16.0
    kw.setdefault("dt", 1.0 / 256)
    kw.setdefault("rho", 2.0)
    kw.setdefault("nu", 1.0 / 16)
    return oc.CavityParams(H, W, lx=(W - 1) / 8.0, ly=ly, **kw)


def coords(prm):
    i = np.arange(prm.H)[:, None]
    j = np.arange(prm.W)[None, :]
    return j * prm.dx + 0 * i, i * prm.dy + 0 * j  # x, y as full grids


def test_source_term_linear_fields_exact():
    prm = dyadic_params()
    x, y = coords(prm)
    a0, a1, a2, b0, b1, b2 = 1, 3, -2, -1, 5, 4
    u = a0 + a1 * x + a2 * y
    v = b0 + b1 * x + b2 * y
    b = oc.source_term(u, v, prm)
    F = Fraction
    want = F(prm.rho) * ((F(a1) + F(b2)) / F(prm.dt) - F(a1) ** 2 - 2 * F(a2) * F(b1) - F(b2) ** 2)
    assert np.all(b[1:-1, 1:-1] == float(want))
    assert np.all(b[0, :] == 0) and np.all(b[:, -1] == 0)


def test_momentum_linear_fields_exact():
    """Linear u, v, p: diffusion vanishes, every difference is exact."""
    prm = dyadic_params()
    x, y = coords(prm)
    a1, a2, b1, b2, c1, c2 = 2, -1, 1, 3, 5, -7
    u = 1 + a1 * x + a2 * y
    v = -2 + b1 * x + b2 * y
    p = 3 + c1 * x + c2 * y
    u2, v2 = oc.momentum(u, v, p, prm)
    F = Fraction
    dt, rho = F(prm.dt), F(prm.rho)
    for i in range(1, prm.H - 1):
        for j in range(1, prm.W - 1):
            U, V = F(u[i, j]), F(v[i, j])
            assert F(u2[i, j]) == U - dt * U * a1 - dt * V * a2 - dt / rho * c1, (i, j)
            assert F(v2[i, j]) == V - dt * U * b1 - dt * V * b2 - dt / rho * c2, (i, j)


def test_momentum_quadratic_upwind_and_diffusion():
    """u = x^2 (v = 0): backward difference 2x - dx, second difference 2 dx^2; same for v = y^2."""
    prm = dyadic_params()
    x, y = coords(prm)
    zero = np.zeros((prm.H, prm.W))
    F = Fraction
    dt, nu, dx, dy = F(prm.dt), F(prm.nu), F(prm.dx), F(prm.dy)
    u2, _ = oc.momentum(x * x, zero, zero, prm)
    v2 = oc.momentum(zero, y * y, zero, prm)[1]
    for i in range(1, prm.H - 1):
        for j in range(1, prm.W - 1):
            X, Y = F(x[i, j]), F(y[i, j])
            assert F(u2[i, j]) == X * X - dt * X * X * (2 * X - dx) + 2 * nu * dt, (i, j)
            assert F(v2[i, j]) == Y * Y - dt * Y * Y * (2 * Y - dy) + 2 * nu * dt, (i, j)


def test_pressure_fixed_point_quadratic():
    """p = x^2 + y^2 solves p_xx + p_yy = 4: one iteration leaves the interior unchanged."""
    prm = dyadic_params(H=10, W=10, square=True)
    x, y = coords(prm)
    p = x * x + y * y
    b = np.full((prm.H, prm.W), 4.0)
    q = oc.pressure_iteration(p, b, prm)
    assert np.array_equal(q[1:-1, 1:-1], p[1:-1, 1:-1])
    # the walls: copies of the inner neighbours, lid zero
    assert np.array_equal(q[1:-1, -1], q[1:-1, -2]) and np.array_equal(q[1:-1, 0], q[1:-1, 1])
    assert np.array_equal(q[0, :], q[1, :]) and np.all(q[-1, :] == 0)


def poisson_direct(b, prm):
    """Solve (p_E - 2p + p_W)/dx^2 + (p_N - 2p + p_S)/dy^2 = b on the interior, with p on the side
    walls equal to its inner neighbour, the bottom row equal to the row above, and p = 0 on the lid."""
    H, W = prm.H, prm.W
    idx = {(i, j): k for k, (i, j) in enumerate((i, j) for i in range(1, H - 1) for j in range(1, W - 1))}
    n = len(idx)
    A = np.zeros((n, n))
    rhs = np.zeros(n)
    for (i, j), k in idx.items():
        rhs[k] = b[i, j]
        for (di, dj, w) in ((0, 1, 1 / prm.dx ** 2), (0, -1, 1 / prm.dx ** 2), (1, 0, 1 / prm.dy ** 2),
                            (-1, 0, 1 / prm.dy ** 2)):
            A[k, k] -= w
            ni, nj = i + di, j + dj
            if ni == H - 1:
                continue                          # lid: p = 0
            ni = max(ni, 1)                       # bottom wall copies row 1
            nj = min(max(nj, 1), W - 2)           # side walls copy their inner column
            A[k, idx[(ni, nj)]] += w
    sol = np.linalg.solve(A, rhs)
    p = np.zeros((H, W))
    for (i, j), k in idx.items():
        p[i, j] = sol[k]
    return p


def test_pressure_iteration_converges_to_direct_solve():
    prm = oc.CavityParams(7, 9, lx=1.0, ly=1.5)  # dx = 1/8, dy = 1/4: unequal weights
    rng = np.random.default_rng(5)
    b = np.zeros((prm.H, prm.W))
    b[1:-1, 1:-1] = rng.standard_normal((prm.H - 2, prm.W - 2))
    p = np.zeros((prm.H, prm.W))
    for _ in range(6000):
        p = oc.pressure_iteration(p, b, prm)
    want = poisson_direct(b, prm)
    assert np.max(np.abs(p[1:-1, 1:-1] - want[1:-1, 1:-1])) < 1e-10 * max(1.0, np.max(np.abs(want)))


def test_walls_and_rest_state():
    prm = oc.CavityParams(12, 15, nit=5)
    u, v, p = oc.run(3, prm)
    assert np.all(u[-1, :] == 1) and np.all(u[0, :] == 0) and np.all(u[:-1, 0] == 0) and np.all(u[:-1, -1] == 0)
    assert np.all(v[0, :] == 0) and np.all(v[-1, :] == 0) and np.all(v[:, 0] == 0) and np.all(v[:, -1] == 0)
    assert np.all(p[-1, :] == 0)
    # the lid drags the fluid under it along: u > 0 just below the lid, away from the corners
    assert np.all(u[-2, 2:-2] > 0)
    # a fluid at rest with a resting lid stays at rest
    prm0 = oc.CavityParams(8, 8, nit=3)
    z = np.zeros((8, 8))
    u0, v0, p0 = oc.momentum(z, z, z, prm0)[0], z, z
    assert np.all(u0 == 0)


# -- planted mistakes ---------------------------------------------------------------------------

_true_momentum = oc.momentum


def _mutant_momentum(kind):
    """The oracle's momentum with one planted mistake in the u update (v stays correct)."""
    def momentum(u, v, p, prm):
        un, vn = u, v
        cx, cy, kx, ky = prm.cx, prm.cy, prm.kx, prm.ky
        C, V = un[1:-1, 1:-1], vn[1:-1, 1:-1]
        west = un[1:-1, 2:] if kind == "forward_difference" else un[1:-1, :-2]
        sgn = -1.0 if kind == "pressure_sign" else 1.0
        south = un[:-2, 1:-1] if kind != "transposed" else un[1:-1, :-2]
        u2, v2 = un.copy(), _true_momentum(u, v, p, prm)[1]
        u2[1:-1, 1:-1] = C - cx * C * (C - west) - cy * V * (C - south) \
            - sgn * prm.cpx * (p[1:-1, 2:] - p[1:-1, :-2]) \
            + kx * (un[1:-1, 2:] - 2.0 * C + un[1:-1, :-2]) \
            + (0.0 if kind == "dropped_diffusion_y" else ky) * (un[2:, 1:-1] - 2.0 * C + un[:-2, 1:-1])
        return u2, v2
    return momentum


@pytest.mark.parametrize("kind", ["forward_difference", "pressure_sign", "transposed", "dropped_diffusion_y"])
def test_momentum_mutants_caught(kind, monkeypatch):
    monkeypatch.setattr(oc, "momentum", _mutant_momentum(kind))
    failed = 0
    for t in (test_momentum_linear_fields_exact, test_momentum_quadratic_upwind_and_diffusion):
        try:
            t()
        except AssertionError:
            failed += 1
    if kind == "dropped_diffusion_y":  # only a y-quadratic shows the y diffusion; x^2 + y^2 test below
        prm = dyadic_params()
        x, y = coords(prm)
        z = np.zeros((prm.H, prm.W))
        u2 = oc.momentum(y * y, z, z, prm)[0]
        failed += int(not np.all(u2[1:-1, 1:-1] == (y * y)[1:-1, 1:-1] + 2 * prm.nu * prm.dt))
    assert failed > 0


@pytest.mark.parametrize("kind", ["swapped_weights", "source_sign", "bottom_from_row2"])
def test_pressure_mutants_caught(kind, monkeypatch):
    def pressure_iteration(p, b, prm):
        pn, q = p.copy(), p.copy()
        cw, cn = (prm.cn, prm.cw) if kind == "swapped_weights" else (prm.cw, prm.cn)
        sgn = -1.0 if kind == "source_sign" else 1.0
        q[1:-1, 1:-1] = cw * (pn[1:-1, 2:] + pn[1:-1, :-2]) + cn * (pn[2:, 1:-1] + pn[:-2, 1:-1]) \
            - sgn * prm.cb * b[1:-1, 1:-1]
        q[1:-1, -1] = q[1:-1, -2]
        q[1:-1, 0] = q[1:-1, 1]
        q[0, :] = q[2, :] if kind == "bottom_from_row2" else q[1, :]
        q[-1, :] = 0.0
        return q

    monkeypatch.setattr(oc, "pressure_iteration", pressure_iteration)
    with pytest.raises(AssertionError):
        test_pressure_iteration_converges_to_direct_solve()


def test_source_mutant_caught(monkeypatch):
    def source_term(u, v, prm):
        b = np.zeros_like(u)
        dudx = (u[1:-1, 2:] - u[1:-1, :-2]) / (2.0 * prm.dx)
        dvdy = (v[2:, 1:-1] - v[:-2, 1:-1]) / (2.0 * prm.dy)
        dudy = (u[2:, 1:-1] - u[:-2, 1:-1]) / (2.0 * prm.dy)
        dvdx = (v[1:-1, 2:] - v[1:-1, :-2]) / (2.0 * prm.dx)
        b[1:-1, 1:-1] = prm.rho * ((dudx + dvdy) / prm.dt - dudx * dudx - dudy * dvdx - dvdy * dvdy)  # lost 2
        return b

    monkeypatch.setattr(oc, "source_term", source_term)
    with pytest.raises(AssertionError):
        test_source_term_linear_fields_exact()


# -- the frontend program against the oracle (NumPy backend: host logic only) ----------------------

@pytest.mark.parametrize("shape,nit,nt", [((9, 11), 4, 3), ((16, 13), 7, 4), ((5, 5), 2, 2)])
def test_frontend_cavity_matches_oracle_on_numpy_backend(shape, nit, nt):
    H, W = shape
    be = NumpyBackend()
    ctx = fe.Context(max_depth=16, backend=be)
    flow = CavityFlow(ctx, H, W, nit=nit)
    flow.run(nt)
    u, v, p = flow.fields()
    uo, vo, po = oc.run(nt, oc.CavityParams(H, W, nit=nit))
    assert np.array_equal(u, uo) and np.array_equal(v, vo) and np.array_equal(p, po)
    # u and v updates run fused in one group each step
    fused = [g for g in be.groups if len(g) == 2]
    assert len(fused) == nt


def test_frontend_cavity_programs_compile():
    """Every generated program of one cavity step is valid and compiles for gfx950 (hiprtc, no GPU)."""
    from paper_2512_19851_amd import ops

    class Collect(NumpyBackend):
        def __init__(self):
            super().__init__()
            self.programs = set()

        def run(self, group):
            if fe.node_kind(group[0]) == "expr":
                for text, ins, outs, _, _ in fe.split_for_limits(group):
                    self.programs.add((text, len(ins), len(outs)))
            super().run(group)

    be = Collect()
    ctx = fe.Context(backend=be)
    CavityFlow(ctx, 12, 10, nit=2).run(1)
    ctx.sync()
    assert len(be.programs) >= 6
    for text, nin, nout in sorted(be.programs):
        ops.expr_compile(text, nin, nout)
