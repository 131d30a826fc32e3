"""Pins of the oracle's model and cost (Eqs. 1-3) to a hand-worked example,
to high-precision noiseless data, and to invariants of the definitions."""

import json
import math
import os

import mpmath as mp
import numpy as np
import pytest

import synth
from oracle import model, scalar

HERE = os.path.dirname(os.path.abspath(__file__))
EPS = np.finfo(np.float64).eps
mp.mp.dps = 50


def _hand_case():
    with open(os.path.join(HERE, "golden", "hand_3bin.json")) as fh:
        g = json.load(fh)
    th = synth.theory_exp_cos()
    pr = g["params"]
    p = np.array([pr["N0"], pr["Nbkg"], pr["A"], pr["lambda"], pr["nu"], pr["phi"]])
    h = {"n_bins": 3, "dt": th["tau_mu"] * math.log(2.0), "t0_bin": 0.0, "first": 0, "last": 2, "map_row": 0}
    return g, th, h, p


def test_hand_worked_model_values():
    g, th, h, p = _hand_case()
    N = model.model(th, h, p)
    np.testing.assert_allclose(N, [130.0, 67.5, 36.25], rtol=4 * EPS)


@pytest.mark.parametrize("kind,key", [("chi2", "chi2_closed_form"), ("poisson", "poisson_closed_form")])
def test_hand_worked_cost(kind, key):
    g, th, h, p = _hand_case()
    expect = float(eval(g[key], {"log": mp.log}, {}))  # closed form written in the fixture
    got = model.cost(th, [h], [np.array(g["counts"])], p, kind)
    assert got == pytest.approx(expect, rel=1e-13)
    assert scalar.cost(th, [h], [np.array(g["counts"])], p, kind) == pytest.approx(expect, rel=1e-13)


def _mp_model(theory, h, p, n):
    """Eq. 1 at 50 digits for the single-row exp*cos / c2 style theories."""
    row = h["map_row"]
    P = [mp.mpf(x) for x in p]
    m = theory["map"][row]

    def ref(r):
        kind, x = r
        if kind == "p":
            return P[m[x]]
        if kind == "f":
            Fi = theory["F"][m[x]]
            return sum(mp.mpf(Fi[k]) * P[k] for k in range(len(P))) + mp.mpf(theory["f0"][m[x]])
        return mp.mpf(x)

    t = (mp.mpf(n) - mp.mpf(h["t0_bin"])) * mp.mpf(h["dt"])
    A = mp.mpf(0)
    for term in theory["terms"]:
        v = mp.mpf(term["coef"]) * ref(term["amp"])
        for fac in term["factors"]:
            a = [ref(r) for r in fac["args"]]
            k = fac["prim"]
            if k == "se":
                v *= mp.exp(-a[0] * t)
            elif k == "ge":
                v *= mp.exp(-((a[0] * t) ** a[1]))
            elif k == "sg":
                v *= mp.exp(-(a[0] * t) ** 2 / 2)
            elif k == "stg":
                s2 = (a[0] * t) ** 2
                v *= mp.mpf(1) / 3 + mp.mpf(2) / 3 * (1 - s2) * mp.exp(-s2 / 2)
            elif k == "tf":
                v *= mp.cos(2 * mp.pi * a[1] * t + a[0])
        A += v
    return ref(theory["n0"]) * mp.exp(-t / mp.mpf(theory["tau_mu"])) * (1 + A) + ref(theory["nbkg"])


@pytest.mark.parametrize("which", ["c1", "c2", "eq4"])
def test_noiseless_at_truth_is_zero(which):
    """Noiseless non-integer data at the true parameters: the cost is zero up
    to rounding.  chi^2: bound sum (4 eps N)^2 / v from the rounding of N.
    Likelihood: its two halves (N - d) and d ln(d/N) cancel, and the rounding
    of d/N alone leaves up to about eps d per bin, so the bound is sum 4 eps d."""
    if which == "c1":
        cfg = synth.config_c1()
        histos = [dict(cfg["histos"][0], n_bins=96, last=95)]
    elif which == "c2":
        cfg = synth.config_c2()
        histos = [dict(h, n_bins=48, last=47, dt=0.05) for h in cfg["histos"][:3]]
    else:
        cfg = synth.config_paper_shape()
        histos = [dict(h, n_bins=40, last=39, dt=0.2) for h in cfg["histos"][:2]]
    th, p = cfg["theory"], cfg["p_true"]
    counts = [np.array([float(_mp_model(th, h, p, n)) for n in range(h["n_bins"])]) for h in histos]
    # FP64 arguments of exp / cos are rounded once or twice: the error they
    # carry grows with the size of the argument, theta_n <= 100 t_n + 10 here
    thetas = [100.0 * model.time_grid(h) + 10.0 for h in histos]
    for h, d, th_n in zip(histos, counts, thetas):
        assert np.all(np.abs(model.model(th, h, p) - d) <= 4 * EPS * d * th_n)
    for kind in ("chi2", "poisson"):
        c = model.cost(th, histos, counts, p, kind)
        if kind == "chi2":
            bound = sum(float(np.sum((4 * EPS * d * th_n) ** 2 / d)) for d, th_n in zip(counts, thetas))
            assert 0.0 <= c <= bound, (kind, c, bound)
        else:
            bound = sum(float(np.sum(4 * EPS * d)) for d in counts)
            assert abs(c) <= bound, (kind, c, bound)


def _small_c1(n=200, seed=5):
    cfg = synth.config_c1()
    h = dict(cfg["histos"][0], n_bins=n, last=n - 1, dt=0.02)
    rng = np.random.default_rng(seed)
    d = synth.draw_counts(model.model_full(cfg["theory"], h, cfg["p_true"]), rng)
    return cfg["theory"], h, d, cfg["p_true"]


@pytest.mark.parametrize("kind", ["chi2", "poisson"])
def test_scalar_and_vector_agree(kind):
    th, h, d, p = _small_c1()
    p2 = p * (1 + 0.01)
    a = model.cost(th, [h], [d], p2, kind)
    b = scalar.cost(th, [h], [d], p2, kind)
    assert a == pytest.approx(b, rel=1e-13)


@pytest.mark.parametrize("kind", ["chi2", "poisson"])
def test_concatenation_adds_and_permutation_preserves(kind):
    th, h, d, p = _small_c1()
    h1 = dict(h, first=0, last=99)
    h2 = dict(h, first=100, last=199)
    whole = model.cost(th, [h], [d], p, kind)
    parts = model.cost(th, [h1], [d], p, kind) + model.cost(th, [h2], [d], p, kind)
    assert whole == pytest.approx(parts, rel=1e-15)
    # per-bin terms do not depend on the order of the bins
    N = model.model(th, h, p)
    terms = model.cost_terms(d, N, kind)
    perm = np.random.default_rng(1).permutation(d.size)
    assert math.fsum(model.cost_terms(d[perm], N[perm], kind)) == math.fsum(terms)


def test_amplitude_phase_symmetry():
    # A cos(x + phi) = (-A) cos(x + phi + pi)
    th, h, d, p = _small_c1()
    q = p.copy()
    q[2] = -p[2]
    q[5] = p[5] + math.pi
    for kind in ("chi2", "poisson"):
        assert model.cost(th, [h], [d], p, kind) == pytest.approx(model.cost(th, [h], [d], q, kind), rel=1e-13)


def test_zero_background_amplitude_model():
    # A = 0 reduces Eq. 1 to N0 e^(-t/tau) + Nbkg
    th, h, d, p = _small_c1()
    q = p.copy()
    q[2] = 0.0
    t = model.time_grid(h)
    np.testing.assert_allclose(model.model(th, h, q), q[0] * np.exp(-t / th["tau_mu"]) + q[1], rtol=2 * EPS)


def test_poisson_terms_nonnegative_and_edge_cases():
    d = np.array([0.0, 0.0, 3.0, 5.0, 7.0])
    N = np.array([2.5, 0.0, 3.0, 4.0, -1.0])
    t = model.cost_terms(d, N, "poisson")
    assert t[0] == 5.0           # d = 0: 2N
    assert t[1] == 0.0
    assert t[2] == 0.0           # N = d: zero
    assert t[3] > 0.0
    assert t[4] == math.inf      # N <= 0 < d
    rng = np.random.default_rng(3)
    dd = rng.poisson(20.0, 1000).astype(float)
    NN = rng.uniform(1.0, 40.0, 1000)
    assert np.all(model.cost_terms(dd, NN, "poisson") >= 0)


def test_chi2_empty_bin_weight_one():
    t = model.cost_terms(np.array([0.0, 4.0]), np.array([3.0, 6.0]), "chi2")
    assert t[0] == 9.0 and t[1] == 1.0


def test_function_array_route():
    """Eq. 4 with nu taken from f = F p: moving B moves nu = 13.553879 B."""
    cfg = synth.config_paper_shape()
    th, p = cfg["theory"], cfg["p_true"]
    f = model.function_array(th, p)
    assert f[0] == pytest.approx(13.553879 * p[1], rel=1e-15)
    res = dict((n, v) for n, v, _ in model.resolve(th, p, 3))
    assert res["arg0.1.1"] == pytest.approx(f[0], rel=0)
    assert res["arg0.1.0"] == p[2 + 4 * 3 + 3]
