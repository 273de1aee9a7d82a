"""General star stencils with node fusion against the CPU oracle, via the C ABI (bit-exact)."""

import numpy as np
import pytest

from oracle.star import StarCoef, star_apply, star_iterate
from tests.gpu_util import device, say, to_dev, to_host
from workloads import large_f64, normal_grid

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ops():
    device()
    from paper_2512_19851_amd import ops

    return ops


def rand_coef(R, seed):
    rng = np.random.default_rng(seed)
    v = lambda: list(rng.standard_normal(R) * 0.3)  # noqa: E731
    return StarCoef(float(rng.standard_normal()), v(), v(), v(), v())


def spec(c: StarCoef):
    return (c.c0, c.cn, c.cs, c.cw, c.ce)


SHAPES = [(9, 9), (10, 13), (64, 64), (257, 1031), (1000, 513), (40, 600)]


@pytest.mark.parametrize("R", [1, 2, 3, 4])
@pytest.mark.parametrize("shape", SHAPES, ids=lambda s: f"{s[0]}x{s[1]}")
def test_star_single_bit_exact(ops, R, shape):
    u = normal_grid(*shape, seed=R * 100 + shape[0])
    c = rand_coef(R, R + shape[1])
    say(f"star R={R} {shape}")
    (got,) = ops.star(to_dev(u), [spec(c)])
    assert np.array_equal(to_host(got), star_apply(u, c))


@pytest.mark.parametrize("R", [1, 2, 4])
@pytest.mark.parametrize("nout", [2, 3, 4])
def test_star_fused_bit_exact(ops, R, nout):
    u = normal_grid(123, 777, seed=R + nout)
    coefs = [rand_coef(R, 10 * R + o) for o in range(nout)]
    say(f"star fused R={R} nout={nout}")
    outs = ops.star(to_dev(u), [spec(c) for c in coefs])
    for o, c in enumerate(coefs):
        assert np.array_equal(to_host(outs[o]), star_apply(u, c)), f"output {o}"


@pytest.mark.parametrize("R", [1, 3])
def test_star_iterate(ops, R):
    u0 = normal_grid(90, 140, seed=R)
    c = rand_coef(R, 77 + R)
    # keep the iteration bounded: scale coefficients to a contraction
    scale = 1.0 / (abs(c.c0) + sum(abs(x) for x in c.cn + c.cs + c.cw + c.ce))
    c = StarCoef(c.c0 * scale, [x * scale for x in c.cn], [x * scale for x in c.cs], [x * scale for x in c.cw],
                 [x * scale for x in c.ce])
    for T in (0, 1, 2, 5):
        say(f"star iterate R={R} T={T}")
        got = to_host(ops.star_iterate(to_dev(u0), T, spec(c)))
        assert np.array_equal(got, star_iterate(u0, T, c)), f"T={T}"


def test_star_jacobi_coefficients_on_exact_data(ops):
    """c*N + c*S + c*W + c*E equals the listing's sweep when every operation is exact."""
    import oracle

    rng = np.random.default_rng(5)
    u0 = rng.integers(-100, 101, (50, 70)).astype(np.float64)
    say("star jacobi exact")
    got = to_host(ops.star_iterate(to_dev(u0), 3, spec(StarCoef.jacobi())))
    assert np.array_equal(got, oracle.jacobi5(u0, 3))


def test_star_full_size_fused(ops):
    u = large_f64(0)
    coefs = [rand_coef(2, 1), rand_coef(2, 2)]
    say("star 4096 fused")
    outs = ops.star(to_dev(u), [spec(c) for c in coefs])
    for o, c in enumerate(coefs):
        assert np.array_equal(to_host(outs[o]), star_apply(u, c))


def test_star_errors(ops):
    import ctypes

    import torch

    from paper_2512_19851_amd import StenError, _lib

    u = to_dev(normal_grid(20, 20))
    say("star errors")
    with pytest.raises(StenError):
        ops.star(u, [spec(rand_coef(1, 0))], outs=[u])  # output aliases the input
    with pytest.raises(StenError):
        ops.star(u, [spec(rand_coef(1, 0)), spec(rand_coef(2, 0))])  # fused radii differ
    with pytest.raises(ValueError):
        ops.star(u, [(0.0, [1.0] * 5, [1.0] * 5, [1.0] * 5, [1.0] * 5)])  # radius 5
    torch.cuda.synchronize()
    assert ctypes is not None and _lib is not None
