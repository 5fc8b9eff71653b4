"""Pins of the oracle's binary32 elementary functions, fitness functions and
(fitness, index) keys against closed forms, library routines and brute force.

The paper evaluates Sphere, Rosenbrock and its Cubic function (Sec. 5.1,
Eq. 3); Rastrigin and Ackley are the benchmark's other two functions.
"""
import math

import numpy as np
import pytest
import scipy.optimize

import oracle
from oracle import derive_constants as dc

F32 = np.float32


def ulp_err(got, exact):
    """|got - exact| in units of the binary32 ulp at the exact value."""
    got = np.asarray(got, np.float64)
    exact = np.asarray(exact, np.float64)
    e = np.abs(exact)
    ex = np.floor(np.log2(np.maximum(e, 2.0 ** -126)))
    ulp = 2.0 ** (ex - 23)
    return np.abs(got - exact) / ulp


# ---------------------------------------------------------------- constants
def test_constants_are_rounded_series_coefficients():
    c = oracle.constants()
    assert c["cos"] == dc.cos_pi_coeffs()
    assert c["sin"] == dc.sin_pi_coeffs()
    assert c["exp"] == dc.exp_coeffs()
    hi, lo, l2e = dc.ln2_split()
    assert (c["ln2_hi"], c["ln2_lo"], c["log2e"]) == (hi, lo, l2e)


def test_round_f32_matches_numpy_on_doubles():
    rng = np.random.default_rng(0)
    from fractions import Fraction
    for v in rng.standard_normal(500) * 10.0 ** rng.integers(-20, 20, 500):
        assert dc.round_f32(Fraction(float(v))) == float(F32(v))


# ---------------------------------------------------------------- cospi / exp
def test_cospi_exact_values():
    ks = np.arange(-64, 65, dtype=np.float32)
    c = oracle.cospi_f32(ks)
    assert np.array_equal(c, np.where(ks.astype(np.int64) % 2 == 0, 1.0, -1.0).astype(F32))
    half = oracle.cospi_f32(ks + F32(0.5))
    assert np.all(half == 0.0)
    big = oracle.cospi_f32(np.array([2.0 ** 24, 2.0 ** 25 + 2, 3.0e9, -2.0 ** 30], F32))
    assert np.all(big == 1.0)


def test_cospi_within_2_ulp_of_libm():
    y = np.linspace(-12.0, 12.0, 2_000_001, dtype=np.float64).astype(F32)
    y = np.concatenate([y, (np.random.default_rng(2).random(200_000) - 0.5).astype(F32) * F32(1e-3)])
    got = oracle.cospi_f32(y)
    r = y.astype(np.float64) - np.rint(y.astype(np.float64))
    exact = np.cos(np.pi * r) * np.where(np.rint(y.astype(np.float64)) % 2 == 0, 1.0, -1.0)
    # at |r| = 1/2 the exact value is 0 (libm's cos(pi/2) is not): checked above
    nz = np.abs(r) != 0.5
    err = ulp_err(got[nz], exact[nz])
    assert np.max(err) <= 2.0


def test_exp_exact_and_within_2_ulp():
    assert oracle.exp_f32(np.array([0.0], F32))[0] == 1.0
    x = np.linspace(-87.0, 88.0, 2_000_001).astype(F32)
    got = oracle.exp_f32(x)
    err = ulp_err(got, np.exp(x.astype(np.float64)))
    assert np.max(err) <= 2.0
    assert oracle.exp_f32(np.array([200.0], F32))[0] == np.inf
    assert oracle.exp_f32(np.array([-200.0], F32))[0] == 0.0


# ---------------------------------------------------------------- fitness
def swarm(fit, D, shift=None, lo=-100.0, hi=100.0):
    return oracle.Swarm(fit, 1, D, lo, hi, 0.729, 1.49445, 1.49445, 1.0, 0, shift=shift, nthreads=1)


@pytest.mark.parametrize("fit", ["sphere", "rastrigin", "ackley"])
@pytest.mark.parametrize("D", [1, 2, 7, 32, 128])
def test_zero_at_shift(fit, D):
    s = np.random.default_rng(D).uniform(-5, 5, D).astype(F32)
    sw = swarm(fit, D, s)
    assert sw.fitness_f32(s[None, :])[0] == 0.0
    assert sw.fitness_f64(s[None, :].astype(np.float64))[0] == pytest.approx(0.0, abs=1e-12)


@pytest.mark.parametrize("D", [2, 3, 32, 128])
def test_rosenbrock_zero_at_shift_plus_one_and_d_minus_1_at_shift(D):
    s = np.random.default_rng(D).uniform(-5, 5, D).astype(F32)
    sw = swarm("rosenbrock", D, s)
    # z = 1 exactly requires x - s == 1 in binary32: use integer shifts
    si = np.round(s).astype(F32)
    sw = swarm("rosenbrock", D, si)
    assert sw.fitness_f32((si + 1)[None, :])[0] == 0.0
    assert sw.fitness_f32(si[None, :])[0] == D - 1


def test_integer_points_closed_forms():
    rng = np.random.default_rng(5)
    for D in (1, 3, 16):
        z = rng.integers(-5, 6, (50, D)).astype(F32)
        sq = (z.astype(np.float64) ** 2).sum(1)
        assert np.array_equal(swarm("sphere", D).fitness_f32(z), sq.astype(F32))
        # cos(2 pi k) = 1: Rastrigin reduces to sum z^2
        assert np.array_equal(swarm("rastrigin", D).fitness_f32(z), sq.astype(F32))
        # half-integers: cos(2 pi (k + 1/2)) = -1, f = 20 D + sum z^2
        zh = z + F32(0.5)
        want = 20 * D + (zh.astype(np.float64) ** 2).sum(1)
        assert np.array_equal(swarm("rastrigin", D).fitness_f32(zh), want.astype(F32))
        # Ackley on a constant integer vector a: 20 - 20 exp(-0.2 |a|)
        a = rng.integers(-5, 6, 50)
        pts = np.repeat(a[:, None], D, 1).astype(F32)
        want = 20.0 - 20.0 * np.exp(-0.2 * np.abs(a))
        np.testing.assert_allclose(swarm("ackley", D).fitness_f32(pts), want, rtol=0, atol=4e-6)
        # Cubic at 0: -(8000 D)
        assert swarm("cubic", D).fitness_f32(np.zeros((1, D), F32))[0] == -8000.0 * D


def test_rosenbrock_matches_scipy():
    rng = np.random.default_rng(7)
    for D in (2, 5, 32, 128):
        pts = rng.uniform(-3, 3, (200, D))
        f64 = swarm("rosenbrock", D).fitness_f64(pts)
        np.testing.assert_allclose(f64, [scipy.optimize.rosen(p) for p in pts], rtol=1e-13)


def test_cubic_matches_polynomial_of_eq3():
    rng = np.random.default_rng(8)
    D = 4
    pts = rng.uniform(-100, 100, (300, D))
    poly = np.polynomial.Polynomial([8000.0, -1000.0, -0.8, 1.0])
    want = -poly(pts).sum(1)
    np.testing.assert_allclose(swarm("cubic", D).fitness_f64(pts), want, rtol=1e-12, atol=1e-6)


def test_ackley_rastrigin_f64_match_textbook_formula():
    rng = np.random.default_rng(9)
    for D in (2, 10, 128):
        s = rng.uniform(-5, 5, D).astype(F32)
        pts = rng.uniform(-30, 30, (100, D))
        z = pts - s.astype(np.float64)
        rast = 10 * D + (z ** 2 - 10 * np.cos(2 * np.pi * z)).sum(1)
        ack = (-20 * np.exp(-0.2 * np.sqrt((z ** 2).mean(1))) - np.exp(np.cos(2 * np.pi * z).mean(1))
               + 20 + np.e)
        np.testing.assert_allclose(swarm("rastrigin", D, s).fitness_f64(pts), rast, rtol=1e-12, atol=1e-9)
        np.testing.assert_allclose(swarm("ackley", D, s).fitness_f64(pts), ack, rtol=1e-12, atol=1e-12)


@pytest.mark.parametrize("fit", ["sphere", "rastrigin", "rosenbrock", "ackley", "cubic"])
def test_f32_within_summation_bound_of_f64(fit):
    """binary32 fitness vs binary64 fitness of the same binary32 point: the
    recursive-summation bound gamma_D * sum|terms| (Higham, Thm 4.4) with a
    few ulps per term for the elementary functions and products."""
    rng = np.random.default_rng(11)
    u = 2.0 ** -24
    for D in (2, 32, 128):
        s = rng.uniform(-5, 5, D).astype(F32)
        lo, hi = {"sphere": (-100, 100), "rastrigin": (-5.12, 5.12), "rosenbrock": (-30, 30),
                  "ackley": (-32.768, 32.768), "cubic": (-100, 100)}[fit]
        pts = rng.uniform(lo, hi, (500, D)).astype(F32)
        sw = swarm(fit, D, s)
        f32 = sw.fitness_f32(pts).astype(np.float64)
        f64 = sw.fitness_f64(pts.astype(np.float64))
        z = pts.astype(np.float64) - s
        if fit == "sphere":
            mag = (z ** 2).sum(1)
        elif fit == "rastrigin":
            mag = (z ** 2 + 10).sum(1) + 10 * D
        elif fit == "rosenbrock":
            mag = (100 * (z[:, 1:] - z[:, :-1] ** 2) ** 2 + 100 * z[:, :-1] ** 4 + (1 - z[:, :-1]) ** 2 + 1).sum(1)
        elif fit == "cubic":
            mag = (np.abs(z) ** 3 + 0.8 * z ** 2 + 1000 * np.abs(z) + 8000).sum(1)
        else:
            mag = np.full(len(pts), 50.0)
        gamma = (D + 8) * u / (1 - (D + 8) * u)
        assert np.all(np.abs(f32 - f64) <= gamma * mag * 4 + 1e-30), fit


# ---------------------------------------------------------------- keys
def test_key_order_is_lexicographic_fitness_then_index():
    rng = np.random.default_rng(13)
    specials = np.array([0.0, -0.0, np.inf, -np.inf, np.nan, 1e-45, -1e-45, 1.17549435e-38,
                         -3.4028235e38, 3.4028235e38, 1.0, -1.0], F32)
    vals = np.concatenate([specials, rng.standard_normal(300).astype(F32) * F32(10.0) ** rng.integers(-40, 38, 300).astype(F32),
                           np.repeat(F32(2.5), 5)])
    idx = rng.permutation(len(vals)).astype(np.uint32)
    k = oracle.keys(vals, idx)

    def rank(v):  # NaN after everything, -0 == +0
        return (1, 0.0) if np.isnan(v) else (0, float(v) + 0.0)
    want = sorted(range(len(vals)), key=lambda j: (rank(vals[j]), int(idx[j])))
    got = sorted(range(len(vals)), key=lambda j: int(k[j]))
    assert got == want
    assert oracle.key(-0.0, 3) == oracle.key(0.0, 3)
    for v in [1.5, -2.25, 0.0, 1e-40, 3e38]:
        assert oracle.key_value(oracle.key(v, 9)) == F32(v)
