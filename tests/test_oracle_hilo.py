"""The hi/lo encoding of the reduced-precision form (CPU, exact checks)."""

import numpy as np
import pytest

import oracle


def test_delta_is_ulp_times_2_pow_minus16():
    hi = np.array([1.0, 1.5, 2.0, 0.75, -3.0, 1e-3, 6e4], dtype=np.float32)
    d = oracle.hilo_delta(hi)
    ulp = np.spacing(np.abs(hi)).astype(np.float64)  # FP32 spacing above |hi|
    assert np.array_equal(d, ulp * 2.0 ** -16)


def test_delta_floor_for_zero_and_subnormal():
    hi = np.array([0.0, 1e-45, -1e-40], dtype=np.float32)
    assert np.all(oracle.hilo_delta(hi) == 2.0 ** -149)


def test_encode_hand_values():
    # 1 + 2^-30: hi = 1, delta = 2^-23 * 2^-16 = 2^-39, q = 2^-30 / 2^-39 = 512
    hi, q = oracle.hilo_encode(np.array([1.0 + 2.0 ** -30]))
    assert hi[0] == np.float32(1.0) and q[0] == 512
    # exact FP32 values have q = 0
    hi, q = oracle.hilo_encode(np.array([0.5, -7.25, 0.0]))
    assert np.all(q == 0)
    # half a quantum rounds to even: 1 + 2^-40 -> q = rint(0.5) = 0; 1 + 3*2^-40 -> rint(1.5) = 2
    _, q = oracle.hilo_encode(np.array([1.0 + 2.0 ** -40, 1.0 + 3 * 2.0 ** -40]))
    assert list(q) == [0, 2]


def test_roundtrip_error_within_one_quantum():
    from workloads import mixed_f64

    x = mixed_f64(seed=0, n=256)
    hi, q = oracle.hilo_encode(x)
    xd = oracle.hilo_decode(hi, q)
    d = oracle.hilo_delta(hi)
    err = np.abs(xd - x)
    assert np.all(err <= d / 2)        # half a quantum, renormalised case included
    assert np.all(err <= 2.0 ** -40 * (1 + 2.0 ** -22) * np.abs(x))
    assert q.dtype == np.int16


def test_decode_is_exact():
    """hi + q*delta is exact in FP64: check with rational arithmetic."""
    from fractions import Fraction

    rng = np.random.default_rng(3)
    hi = (rng.standard_normal(200) * 10.0 ** rng.uniform(-3, 3, 200)).astype(np.float32)
    q = rng.integers(-32768, 32768, 200).astype(np.int16)
    xd = oracle.hilo_decode(hi, q)
    d = oracle.hilo_delta(hi)
    for k in range(200):
        assert Fraction(float(xd[k])) == Fraction(float(hi[k])) + int(q[k]) * Fraction(float(d[k]))


def test_bound_hilo_is_below_target_at_T100():
    """The analytic bound meets the 1e-10 componentwise target up to T = 100."""
    u0 = np.ones((5, 5))
    b = oracle.bound_hilo(u0, 100) / oracle.abs_reference(u0, 100)
    assert b.max() < 1e-10


def test_encode_renormalises_top_of_range():
    """A remainder of exactly +ulp/2 gives q = +32768, which int16 cannot hold.

    x = 1 + 2^-24 (half an FP32 ulp above 1, ties to even so hi = 1) needs
    q = 2^-24 / 2^-39 = 32768; hi must step to 1 + 2^-23 and q become -32768.
    Just below a power of two, x = 2 - 2^-24 - 2^-41 rounds to hi = 2 - 2^-23 with
    remainder 2^-24 - 2^-41 -> q = rint(32767.75) = 32768, so hi steps to 2 and
    q = rint((-2^-24 - 2^-41) / 2^-38) = rint(-16384.125) = -16384.
    """
    from fractions import Fraction

    x = np.array([1.0 + 2.0 ** -24, 2.0 - 2.0 ** -24 - 2.0 ** -41])
    hi, q = oracle.hilo_encode(x)
    assert hi[0] == np.float32(1.0 + 2.0 ** -23) and q[0] == -32768
    assert hi[1] == np.float32(2.0) and q[1] == -16384
    xd = oracle.hilo_decode(hi, q)
    assert xd[0] == x[0]
    assert abs(Fraction(float(xd[1])) - Fraction(float(x[1]))) <= Fraction(2.0 ** -39)


def test_encode_rejects_out_of_range():
    with pytest.raises(ValueError):
        oracle.hilo_encode(np.array([1e300]))


# ---------------------------------------------------------------------------
# The bit-level model of the hi/lo sweep
# ---------------------------------------------------------------------------

def test_two_sum_is_error_free():
    """s + e == a + b exactly (rational check) for FP32 inputs of mixed magnitude."""
    from fractions import Fraction

    from oracle.jacobi import _two_sum

    rng = np.random.default_rng(21)
    a = (rng.standard_normal(300) * 10.0 ** rng.uniform(-8, 8, 300)).astype(np.float32)
    b = (rng.standard_normal(300) * 10.0 ** rng.uniform(-8, 8, 300)).astype(np.float32)
    s, e = _two_sum(a, b)
    assert s.dtype == np.float32 and e.dtype == np.float32
    for k in range(300):
        assert Fraction(float(s[k])) + Fraction(float(e[k])) == Fraction(float(a[k])) + Fraction(float(b[k]))
        assert s[k] == np.float32(float(a[k]) + float(b[k]))  # s is the rounded sum


def test_model_reproduces_worked_examples_exactly():
    """Dyadic grids with few bits are exact in hi/lo, so the model gives the hand-derived values."""
    from tests.pins import read_golden

    for name in ("worked_example_5x5.txt", "worked_example_3x4.txt"):
        c, grids = read_golden(name)
        for T in range(len(grids)):
            assert np.array_equal(oracle.jacobi5_hilo_model(grids[0], T, c), grids[T])


def test_model_keeps_harmonic_fixed_points():
    H, W = 9, 13
    i = np.arange(H, dtype=np.float64)[:, None]
    j = np.arange(W, dtype=np.float64)[None, :]
    u = 1 + 2 * i + 3 * j - i * j + (i * i - j * j)
    assert np.array_equal(oracle.jacobi5_hilo_model(u, 5), u)


@pytest.mark.parametrize("T,c", [(1, 0.25), (3, 0.25), (25, 0.25), (4, 0.3), (2, -0.5)])
def test_model_within_bound_of_fp64(T, c):
    from workloads import mixed_f64

    u0 = mixed_f64(seed=T, n=96)
    y = oracle.jacobi5_hilo_model(u0, T, c)
    ref = oracle.jacobi5(u0, T, c)
    assert np.all(np.abs(y - ref) <= oracle.bound_hilo(u0, T, c))
    assert np.array_equal(y[0, :], u0[0, :]) and np.array_equal(y[:, -1], u0[:, -1])
    assert np.max(np.abs(y - ref)) > 0  # not vacuous: the form is not FP64


def test_model_much_better_than_fp32():
    from workloads import mixed_f64

    u0 = mixed_f64(seed=4, n=64)
    T = 20
    ref = oracle.jacobi5(u0, T)
    e_hilo = np.max(np.abs(oracle.jacobi5_hilo_model(u0, T) - ref))
    e_f32 = np.max(np.abs(oracle.jacobi5(u0.astype(np.float32), T, dtype=np.float32).astype(np.float64) - ref))
    assert e_hilo * 1e4 < e_f32


def test_requantise_renormalises():
    from oracle.jacobi import _hilo_requantise

    # L = +ulp(1)/2 = 2^-24 with H = 1: q would be 32768 -> hi = 1 + 2^-23, q = -32768
    H = np.array([1.0, -3.0], dtype=np.float32)
    L = np.array([2.0 ** -24, 2.0 ** -23], dtype=np.float32)  # -3 has ulp 2^-22; +2^-23 is half an ulp
    hi, q = _hilo_requantise(H, L)
    assert hi[0] == np.float32(1.0 + 2.0 ** -23) and q[0] == -32768
    assert hi[1] == np.float32(-3.0 + 2.0 ** -22) and q[1] == -32768
    dec = oracle.hilo_decode(hi, q)
    assert dec[0] == 1.0 + 2.0 ** -24 and dec[1] == -3.0 + 2.0 ** -23
