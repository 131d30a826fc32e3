"""Pins of the seeder oracle: BF16 rounding against torch's conversion, the
network's backward pass against finite differences, Adam's first step, the
generator's parameter quantiles, and the expected counts against the
closed-form geometric series of a pure decay."""

import math

import numpy as np
import pytest
import torch

import synth
from oracle import seeder


def test_bf16_matches_torch():
    rng = np.random.default_rng(0)
    x = np.concatenate([rng.normal(0, 1, 20000), rng.normal(0, 1e-30, 1000), rng.normal(0, 1e30, 1000),
                        [0.0, -0.0, 1.0, -1.0, 3.14159, 65504.0, 1e-40, np.inf, -np.inf]]).astype(np.float32)
    ref = torch.from_numpy(x).to(torch.bfloat16).to(torch.float32).numpy()
    np.testing.assert_array_equal(seeder.bf16(x), ref)
    bits = seeder.bf16_bits(x)
    np.testing.assert_array_equal(seeder.from_bf16_bits(bits), ref)


def test_backward_matches_finite_differences():
    """Without rounding the backward pass is the exact gradient of the loss."""
    rng = np.random.default_rng(1)
    Ws, bs = seeder.init_params(3)
    # a small random network of the same structure (dims scaled down)
    dims = (12, 10, 8, 6, 8)
    Ws = [rng.normal(0, 0.5, (dims[l + 1], dims[l])) for l in range(4)]
    bs = [rng.normal(0, 0.1, dims[l + 1]) for l in range(4)]
    X = rng.normal(0, 1, (5, dims[0]))
    T = rng.normal(0, 1, (5, 8))
    Y, cache = seeder.forward(Ws, bs, X, rounding=False)
    loss, dY = seeder.loss_and_grad(Y, T)
    dWs, dbs = seeder.backward(cache, dY, rounding=False)
    h = 1e-6
    for l in range(4):
        for (i, k) in [(0, 0), (1, 2), (dims[l + 1] - 1, dims[l] - 1)]:
            Wp = [w.copy() for w in Ws]
            Wm = [w.copy() for w in Ws]
            Wp[l][i, k] += h
            Wm[l][i, k] -= h
            fp = seeder.loss_and_grad(seeder.forward(Wp, bs, X, rounding=False)[0], T)[0]
            fm = seeder.loss_and_grad(seeder.forward(Wm, bs, X, rounding=False)[0], T)[0]
            assert dWs[l][i, k] == pytest.approx((fp - fm) / (2 * h), rel=1e-6, abs=1e-9)
        j = 1
        bp = [b.copy() for b in bs]
        bm = [b.copy() for b in bs]
        bp[l][j] += h
        bm[l][j] -= h
        fp = seeder.loss_and_grad(seeder.forward(Ws, bp, X, rounding=False)[0], T)[0]
        fm = seeder.loss_and_grad(seeder.forward(Ws, bm, X, rounding=False)[0], T)[0]
        assert dbs[l][j] == pytest.approx((fp - fm) / (2 * h), rel=1e-6, abs=1e-9)


def test_adam_first_step_is_a_signed_lr_step():
    """At t = 1 the bias-corrected moments are g and g^2, so every weight
    moves by -lr sign(g) (up to eps)."""
    rng = np.random.default_rng(2)
    p = [rng.normal(0, 1, 100)]
    g = [rng.normal(0, 1, 100)]
    m = [np.zeros(100)]
    v = [np.zeros(100)]
    out = seeder.adam(p, g, m, v, 1, lr=1e-3)
    np.testing.assert_allclose(out[0] - p[0], -1e-3 * np.sign(g[0]), rtol=1e-6)


def test_theta_quantiles_and_range():
    th = seeder.draw_theta(1234, np.arange(20000))
    lo = np.array([v[0] for v in seeder.RANGES.values()])
    hi = np.array([v[1] for v in seeder.RANGES.values()])
    assert np.all(th >= lo) and np.all(th <= hi)
    # log-uniform N0: its median is the geometric mean of the range
    assert np.median(th[:, 0]) == pytest.approx(math.sqrt(100.0 * 1e5), rel=0.05)
    assert np.mean(th[:, 5]) == pytest.approx(math.pi, rel=0.02)
    # deterministic and counter-addressable
    np.testing.assert_array_equal(seeder.draw_theta(1234, [7, 19999]), th[[7, 19999]])


def test_expected_counts_closed_form():
    """A = 0: the 8-bin sums are N0 sum_s e^(-t_s/tau) + 8 Nbkg, a geometric series."""
    th = synth.theory_exp_cos()
    row = np.array([5000.0, 3.0, 0.0, 0.7, 1.1, 0.2])
    mu = seeder.expected_coarse(row, th)
    r = math.exp(-seeder.DT_FINE / seeder.TAU_MU)
    b = np.arange(seeder.N_COARSE)
    closed = 5000.0 * np.exp(-8 * b * seeder.DT_FINE / seeder.TAU_MU) * (1 - r ** 8) / (1 - r) + 8 * 3.0
    np.testing.assert_allclose(mu, closed, rtol=1e-12)


def test_encode_decode_round_trip():
    th = seeder.draw_theta(9, np.arange(50))
    T = seeder.encode(th)
    for i in range(50):
        d = np.full(seeder.N_FINE, 100.0)
        d[:1000] = 5000.0
        start, ok = seeder.decode(T[i], d)
        assert ok
        np.testing.assert_allclose(start[2:5], th[i, 2:5], rtol=1e-12)
        assert math.cos(start[5] - th[i, 5]) == pytest.approx(1.0, abs=1e-12)
    bad = T[0].copy()
    bad[2] = 9.0  # nu far outside the trained range
    assert not seeder.decode(bad, d)[1]


def test_network_input_of_noiseless_histogram_is_the_asymmetry():
    """Noiseless data: zero for A = 0; otherwise the rebin-averaged A(t) up to
    the offset and scale that the window estimates of N0 and Nbkg introduce."""
    th = synth.theory_exp_cos()
    for A in (0.0, 0.2):
        row = np.array([20000.0, 3.0, A, 0.3, 0.7, 0.4])
        mu = seeder.expected_coarse(row, th)
        x = seeder.network_input(mu)
        t = (np.arange(seeder.N_FINE) * seeder.DT_FINE).reshape(seeder.N_COARSE, seeder.REBIN)
        e = np.exp(-t / seeder.TAU_MU)
        asym = (e * A * np.exp(-0.3 * t) * np.cos(2 * np.pi * 0.7 * t + 0.4)).sum(axis=1) / e.sum(axis=1)
        if A == 0.0:
            assert np.max(np.abs(x)) < 1e-9
        else:
            # the windows see part of the oscillation: equal up to offset and scale
            assert np.corrcoef(x, asym)[0, 1] > 0.999
    n0, nb = seeder.window_estimates(seeder.expected_coarse(np.array([5000.0, 7.0, 0.0, 0.3, 0.7, 0.4]), th))
    assert n0 == pytest.approx(5000.0, rel=1e-9) and nb == pytest.approx(7.0, rel=1e-9)
