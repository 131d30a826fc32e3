"""Pins of the oracle's primitives (Listing 2, Listing 3) to closed forms and
to 50-digit mpmath evaluations of their definitions."""

import math

import mpmath as mp
import numpy as np
import pytest

from oracle import model

EPS = np.finfo(np.float64).eps
mp.mp.dps = 50


def _mp_prim(kind, t, args):
    t = mp.mpf(t)
    a = [mp.mpf(x) for x in args]
    if kind == "se":
        return mp.exp(-a[0] * t)
    if kind == "ge":
        return mp.exp(-((a[0] * t) ** a[1]))
    if kind == "sg":
        return mp.exp(-(a[0] * t) ** 2 / 2)
    if kind == "stg":
        s2 = (a[0] * t) ** 2
        return mp.mpf(1) / 3 + mp.mpf(2) / 3 * (1 - s2) * mp.exp(-s2 / 2)
    if kind == "tf":
        return mp.cos(2 * mp.pi * a[1] * t + a[0])
    raise ValueError(kind)


def test_se_half_life():
    lam = 0.5
    t = np.array([math.log(2.0) / lam])
    assert model.prim("se", t, [lam])[0] == pytest.approx(0.5, rel=4 * EPS)


def test_sg_half_point():
    sig = 0.3
    t = np.array([math.sqrt(2.0 * math.log(2.0)) / sig])
    assert model.prim("sg", t, [sig])[0] == pytest.approx(0.5, rel=8 * EPS)


def test_ge_reduces_to_se_and_sg():
    t = np.linspace(0.0, 10.0, 1001)
    lam = 0.7
    np.testing.assert_allclose(model.prim("ge", t, [lam, 1.0]), model.prim("se", t, [lam]), rtol=8 * EPS, atol=0)
    # exp(-(l t)^2) = exp(-(sigma t)^2 / 2) with sigma = sqrt(2) l
    np.testing.assert_allclose(model.prim("ge", t, [lam, 2.0]), model.prim("sg", t, [math.sqrt(2.0) * lam]),
                               rtol=1e-13, atol=1e-300)


def test_stg_at_zero_is_one():
    assert model.prim("stg", np.array([0.0]), [0.3])[0] == 1.0


def test_stg_minimum_value_and_place():
    # d stg / d(sigma t) = 0 at sigma t = sqrt(3); value 1/3 - (4/3) e^(-3/2)
    sig = 0.3
    tmin = math.sqrt(3.0) / sig
    v = model.prim("stg", np.array([tmin]), [sig])[0]
    expect = 1.0 / 3.0 - 4.0 / 3.0 * math.exp(-1.5)
    assert v == pytest.approx(expect, rel=1e-14)
    assert expect == pytest.approx(0.0358264531, abs=1e-10)
    # it is a minimum: neighbours are larger
    tt = np.array([tmin * 0.99, tmin * 1.01])
    assert np.all(model.prim("stg", tt, [sig]) > v)
    # and the analytic derivative vanishes there
    assert abs(model.prim_grad("stg", np.array([tmin]), [sig])[0][0]) < 1e-14


def test_stg_tail_is_one_third():
    # the 1/3 tail of the static Gaussian Kubo-Toyabe: exactly 1/3 in FP64 for sigma t >= 10
    sig = 0.3
    t = np.linspace(10.0 / sig, 100.0 / sig, 50)
    np.testing.assert_array_equal(model.prim("stg", t, [sig]), np.full(t.size, 1.0 / 3.0))


def test_tf_zero_frequency_and_period():
    t = np.linspace(0.0, 5.0, 77)
    phi = 0.4
    np.testing.assert_allclose(model.prim("tf", t, [phi, 0.0]), math.cos(phi), rtol=0, atol=1e-16)
    nu = 1.25  # period 0.8 us
    a = model.prim("tf", t, [phi, nu])
    b = model.prim("tf", t + 0.8, [phi, nu])
    np.testing.assert_allclose(a, b, rtol=0, atol=1e-13)
    # phase shift by pi flips the sign
    np.testing.assert_allclose(model.prim("tf", t, [phi + math.pi, nu]), -a, rtol=0, atol=1e-14)


@pytest.mark.parametrize("kind,args", [
    ("se", [0.5]), ("se", [4.9]), ("ge", [0.8, 0.5]), ("ge", [1.3, 1.7]),
    ("sg", [0.3]), ("sg", [1.1]), ("stg", [0.3]), ("stg", [0.95]),
    ("tf", [0.0, 1.355]), ("tf", [2.1, 47.0]),
])
def test_primitives_against_mpmath(kind, args):
    t = np.linspace(0.0, 10.0, 97)
    got = model.prim(kind, t, args)
    for ti, g in zip(t, got):
        ref = _mp_prim(kind, ti, args)
        # an FP64 argument computed with one or two roundings: error ~ |arg| eps
        # propagated through the primitive, plus the last-place error of libm
        if kind == "tf":
            arg = abs(2 * math.pi * args[1] * ti) + abs(args[0])
            assert abs(g - float(ref)) <= 4 * EPS * (1.0 + arg)
        else:
            scale = 1.0 + (args[0] * ti) ** 2 + abs(args[0] * ti)
            assert abs(g - float(ref)) <= 4 * EPS * scale * max(abs(float(ref)), 1e-300) + 1e-300


@pytest.mark.parametrize("kind,args", [
    ("se", [0.5]), ("ge", [0.8, 0.5]), ("ge", [1.3, 1.7]), ("sg", [0.3]), ("stg", [0.6]), ("tf", [0.3, 2.2]),
])
def test_primitive_derivatives_against_mpmath(kind, args):
    t = np.linspace(0.05, 6.0, 23)
    got = model.prim_grad(kind, t, args)
    for a in range(len(args)):
        for ti, g in zip(t, got[a]):
            def f(x, a=a, ti=ti):
                aa = list(args)
                aa[a] = x
                return _mp_prim(kind, ti, aa)
            ref = mp.diff(f, mp.mpf(args[a]))
            assert abs(g - float(ref)) <= 1e-13 * (1.0 + abs(float(ref)))
