"""Pins of the oracle's analytic gradient and reference minimiser:
Richardson finite differences, closed-form partial derivatives, the exact
weighted least-squares minimum over (N0, Nbkg), and brute-force scans."""

import json
import math
import os

import numpy as np
import pytest

import synth
from oracle import fit, model, philox

HERE = os.path.dirname(os.path.abspath(__file__))


def _data(cfg_theory, histos, p, seed):
    rng = np.random.default_rng(seed)
    return [synth.draw_counts(model.model_full(cfg_theory, h, p), rng) for h in histos]


def _cases():
    c1 = synth.config_c1()
    h1 = [dict(c1["histos"][0], n_bins=300, last=299, dt=0.02)]
    yield "exp_cos", c1["theory"], h1, c1["p_true"]
    c2 = synth.config_c2()
    h2 = [dict(h, n_bins=120, last=119, dt=0.08) for h in c2["histos"][:3]]
    yield "c2_3det", c2["theory"], h2, c2["p_true"]
    ps = synth.config_paper_shape()
    h3 = [dict(h, n_bins=100, last=99, dt=0.05) for h in ps["histos"][:2]]
    p3 = ps["p_true"].copy()
    p3[1] = 0.3  # nu = 4.07 MHz via the function array
    yield "eq4_fnarray", ps["theory"], h3, p3
    g = synth.theory_exp_cos()
    g["terms"][0]["factors"][0] = {"prim": "ge", "args": [synth.ref_p(3), synth.ref_lit(1.6)]}
    yield "ge_lit_beta", g, h1, c1["p_true"]
    gk = synth.theory_exp_gkt()
    yield "exp_gkt", gk, h1, np.array([900.0, 4.0, 0.15, 0.8, 0.12, 0.4])


@pytest.mark.parametrize("kind", ["chi2", "poisson"])
@pytest.mark.parametrize("case", list(range(5)))
def test_gradient_matches_richardson_fd(case, kind):
    name, th, histos, p = list(_cases())[case]
    counts = _data(th, histos, p, 11 + case)
    # away from the minimum, where the gradient is not round-off
    q = p * (1.0 + 1e-2 * np.cos(np.arange(p.size)))
    g = model.grad(th, histos, counts, q, kind)
    fd = model.grad_fd(th, histos, counts, q, kind)
    scale = np.maximum(np.abs(fd), np.max(np.abs(fd)) * 1e-3)
    assert np.all(np.abs(g - fd) <= 1e-6 * scale), (name, g, fd)


def test_gradient_closed_forms():
    name, th, histos, p = list(_cases())[0]
    counts = _data(th, histos, p, 3)
    q = p * 1.01
    g = model.grad(th, histos, counts, q, "chi2")
    d = counts[0]
    N = model.model(th, histos[0], q)
    v = np.where(d > 0, d, 1.0)
    t = model.time_grid(histos[0])
    res = model.resolve(th, q, 0)
    A = model.asymmetry(th, t, res)
    assert g[1] == pytest.approx(math.fsum(-2.0 * (d - N) / v), rel=1e-12)
    assert g[0] == pytest.approx(math.fsum(-2.0 * (d - N) * np.exp(-t / th["tau_mu"]) * (1 + A) / v), rel=1e-12)


def test_fit_matches_linear_least_squares():
    """With every parameter but N0 and Nbkg fixed, chi^2 is exactly quadratic
    in the two; the weighted normal equations give the minimum."""
    c1 = synth.config_c1()
    th = c1["theory"]
    h = [dict(c1["histos"][0], n_bins=2048, last=2047, dt=0.004)]
    counts = _data(th, h, c1["p_true"], 21)
    start = c1["p_true"].copy()
    start[0] *= 1.1
    start[1] *= 0.7
    fixed = np.array([False, False, True, True, True, True])
    r = fit.fit(th, h, counts, start, "chi2", fixed=fixed)
    exact = fit.linear_n0_nbkg(th, h[0], counts[0], start)
    np.testing.assert_allclose(r["p"][:2], exact, rtol=1e-10)


def test_fit_brute_force_grid():
    """Tiny histogram, lambda and nu free: the fitted minimum is no larger than
    any point of a fine grid and lies within one cell of the grid's best."""
    th = synth.theory_exp_cos()
    h = [{"n_bins": 48, "dt": 0.1, "t0_bin": 0.0, "first": 0, "last": 47, "map_row": 0}]
    truth = np.array([2000.0, 5.0, 0.25, 0.6, 1.1, 0.0])
    counts = _data(th, h, truth, 31)
    lam = np.linspace(0.2, 1.2, 101)
    nu = np.linspace(0.8, 1.4, 121)
    grid = np.empty((lam.size, nu.size))
    for i, l in enumerate(lam):
        for j, n in enumerate(nu):
            q = truth.copy()
            q[3], q[4] = l, n
            grid[i, j] = model.cost(th, h, counts, q)
    i, j = np.unravel_index(np.argmin(grid), grid.shape)
    start = truth.copy()
    start[3], start[4] = lam[i], nu[j]
    r = fit.fit(th, h, counts, start, fixed=np.array([True, True, True, False, False, True]))
    assert r["cost"] <= grid.min() + 1e-9
    assert abs(r["p"][3] - lam[i]) <= lam[1] - lam[0]
    assert abs(r["p"][4] - nu[j]) <= nu[1] - nu[0]


def test_philox_known_answers():
    with open(os.path.join(HERE, "golden", "philox4x32_10_kat.json")) as fh:
        kat = json.load(fh)
    for v in kat["vectors"]:
        ctr = np.array([int(x, 16) for x in v["ctr"]], dtype=np.uint32)
        key = np.array([int(x, 16) for x in v["key"]], dtype=np.uint32)
        out = philox.philox4x32_10(ctr, key)
        assert [int(x) for x in out] == [int(x, 16) for x in v["out"]]
