"""Pins of the oracle parts that set the scale of GPU tolerances: the
gradient's absolute scale (sum over bins of |r_n dN_n/dp_k|, Eq. 2 and its
derivative), the per-histogram costs (the double sum of Eq. 2 / Eq. 3 split
by histogram), and the reference minimiser's covariance (2 H^-1 of the cost,
which for the (N0, Nbkg) least-squares case has a closed form)."""

import math

import numpy as np
import pytest

import synth
from oracle import fit, model


def _data(theory, histos, p, seed):
    rng = np.random.default_rng(seed)
    return [synth.draw_counts(model.model_full(theory, h, p), rng) for h in histos]


def _jac_by_model_differences(theory, h, p, k):
    """dN_n/dp_k per bin from central differences of the model itself with one
    Richardson step: a route that shares nothing with the oracle's closed-form
    derivatives."""
    hk = 1e-4 * max(abs(p[k]), 1.0)

    def cd(step):
        pp, pm = p.copy(), p.copy()
        pp[k] += step
        pm[k] -= step
        return (model.model(theory, h, pp) - model.model(theory, h, pm)) / (2.0 * step)

    return (4.0 * cd(hk / 2) - cd(hk)) / 3.0


def _cases():
    c1 = synth.config_c1()
    yield c1["theory"], [dict(c1["histos"][0], n_bins=400, last=399, dt=0.015)], c1["p_true"]
    c2 = synth.config_c2()
    yield c2["theory"], [dict(h, n_bins=150, last=149, dt=0.06) for h in c2["histos"][:3]], c2["p_true"]
    gk = synth.theory_exp_gkt()
    yield gk, [{"n_bins": 300, "dt": 0.03, "t0_bin": 0.0, "first": 5, "last": 290, "map_row": 0}], \
        np.array([900.0, 4.0, 0.15, 0.8, 0.12, 0.4])


def _split_references(theory, p):
    """The same model with every parameter reference of every map row given a
    parameter of its own (value copied from p): returns the rewritten theory,
    its parameter vector and, per new parameter, the original index. A
    parameter that feeds several references of one histogram (C2's shared
    amplitude feeds both terms) is then one new parameter per reference."""
    refs = [("n0", None, None), ("nbkg", None, None)]
    for k, term in enumerate(theory["terms"]):
        refs.append(("amp", k, None))
        for i, fac in enumerate(term["factors"]):
            for a in range(len(fac["args"])):
                refs.append(("arg", k, (i, a)))
    R = len(refs)
    new = {key: theory[key] for key in theory}
    new["terms"] = [{"coef": t["coef"], "amp": t["amp"],
                     "factors": [{"prim": f["prim"], "args": list(f["args"])} for f in t["factors"]]}
                    for t in theory["terms"]]

    def get(r):
        kind, k, ia = r
        if kind in ("n0", "nbkg"):
            return new[kind]
        if kind == "amp":
            return new["terms"][k]["amp"]
        return new["terms"][k]["factors"][ia[0]]["args"][ia[1]]

    def put(r, ref):
        kind, k, ia = r
        if kind in ("n0", "nbkg"):
            new[kind] = ref
        elif kind == "amp":
            new["terms"][k]["amp"] = ref
        else:
            new["terms"][k]["factors"][ia[0]]["args"][ia[1]] = ref

    orig_slots = [get(r) for r in refs]
    rows = theory["map"]
    back, vals, new_map = [], [], []
    for j, row in enumerate(rows):
        new_map.append([j * R + r for r in range(R)])
        for r in range(R):
            kind, x = orig_slots[r]
            k = row[x] if kind == "p" else -1
            back.append(k)
            vals.append(p[k] if k >= 0 else 0.0)
    for r in range(R):
        if orig_slots[r][0] == "p":
            put(refs[r], ("p", r))
    new["map"] = new_map
    new["n_par"] = len(rows) * R
    return new, np.array(vals), np.array(back)


@pytest.mark.parametrize("kind", ["chi2", "poisson"])
@pytest.mark.parametrize("case", [0, 1, 2])
def test_grad_abs_scale_against_model_differences(case, kind):
    """sum over bins and over the references a parameter feeds of
    |r_n dN_n/dR| with r_n = d(term)/dN (Eq. 2: -2 (d - N)/v; Eq. 3:
    2 (1 - d/N)) written out bin by bin, dN/dR from differences of the model
    with every reference given its own parameter."""
    theory, histos, p = list(_cases())[case]
    counts = _data(theory, histos, p, 70 + case)
    q = p * (1.0 + 1e-2 * np.sin(np.arange(p.size) + 1.0))
    got = model.grad_abs_scale(theory, histos, counts, q, kind)
    split, qs, back = _split_references(theory, q)
    want = np.zeros(q.size)
    for h, c in zip(histos, counts):
        N = model.model(theory, h, q)
        np.testing.assert_array_equal(model.model(split, h, qs), N)
        d = np.asarray(c, dtype=np.float64)[h["first"]:h["last"] + 1]
        if kind == "chi2":
            r = -2.0 * (d - N) / np.where(d > 0, d, 1.0)
        else:
            r = np.where(d > 0, 2.0 * (1.0 - d / N), 2.0)
        R = len(split["map"][0])
        for m in range(h["map_row"] * R, (h["map_row"] + 1) * R):
            if back[m] >= 0:
                want[back[m]] += math.fsum(np.abs(r * _jac_by_model_differences(split, h, qs, m)))
    np.testing.assert_allclose(got, want, rtol=1e-6, atol=0)
    # a sum of absolute values bounds the sum itself (triangle inequality)
    g = model.grad(theory, histos, counts, q, kind)
    assert np.all(np.abs(g) <= got * (1.0 + 1e-12))


def test_grad_abs_scale_background_is_sum_of_abs_residual_weights():
    """dN/dNbkg = 1 (Eq. 1), so the background component is sum_n |r_n|."""
    theory, histos, p = list(_cases())[0]
    counts = _data(theory, histos, p, 81)
    h, c = histos[0], counts[0]
    N = model.model(theory, h, p)
    d = np.asarray(c, dtype=np.float64)
    want = math.fsum(np.abs(2.0 * (d - N) / np.where(d > 0, d, 1.0)))
    got = model.grad_abs_scale(theory, histos, counts, p, "chi2")[1]
    assert got == pytest.approx(want, rel=1e-13)


@pytest.mark.parametrize("kind", ["chi2", "poisson"])
def test_cost_per_histo_adds_up_to_cost(kind):
    """The double sum over j and n (Eq. 2 / Eq. 3) split by histogram: each
    part is an exactly rounded sum, so their sum is within a few ulps of the
    exactly rounded total; one histogram alone is the total."""
    theory, histos, p = list(_cases())[1]
    counts = _data(theory, histos, p, 91)
    q = p * 1.003
    parts = model.cost_per_histo(theory, histos, counts, q, kind)
    total = model.cost(theory, histos, counts, q, kind)
    assert len(parts) == len(histos)
    assert abs(math.fsum(parts) - total) <= 4 * np.finfo(float).eps * total
    for j in range(len(histos)):
        alone = model.cost(theory, [histos[j]], [counts[j]], q, kind)
        assert parts[j] == alone


def _linear_case(seed=101):
    c1 = synth.config_c1()
    th = c1["theory"]
    h = [dict(c1["histos"][0], n_bins=1500, last=1499, dt=0.005)]
    counts = _data(th, h, c1["p_true"], seed)
    return th, h, counts, c1["p_true"]


def _normal_matrix(th, h, counts, p):
    """Weighted normal matrix of the (N0, Nbkg) least-squares problem: N = N0 u
    + Nbkg with u = e^(-t/tau) (1 + A) (Eq. 1) and weights 1/v (Eq. 2)."""
    t = model.time_grid(h)
    res = model.resolve(th, p, h["map_row"])
    u = np.exp(-t / th["tau_mu"]) * (1.0 + model.asymmetry(th, t, res))
    d = np.asarray(counts, dtype=np.float64)[h["first"]:h["last"] + 1]
    w = 1.0 / np.where(d > 0, d, 1.0)
    return np.array([[np.sum(w * u * u), np.sum(w * u)], [np.sum(w * u), np.sum(w)]])


def test_fit_covariance_linear_closed_form():
    """chi^2 = sum w (d - N0 u - Nbkg)^2 has the Hessian 2 M (M the weighted
    normal matrix), so the covariance 2 H^-1 the oracle returns is M^-1
    exactly; its condition number is that of M."""
    th, h, counts, truth = _linear_case()
    start = truth.copy()
    start[0] *= 1.1
    start[1] *= 0.6
    fixed = np.array([False, False, True, True, True, True])
    r = fit.fit(th, h, counts, start, "chi2", fixed=fixed)
    M = _normal_matrix(th, h[0], counts[0], start)
    np.testing.assert_allclose(r["cov"], np.linalg.inv(M), rtol=1e-7)
    np.testing.assert_allclose(r["sigma"], np.sqrt(np.diag(np.linalg.inv(M))), rtol=1e-7)
    assert r["cond"] == pytest.approx(np.linalg.cond(M), rel=1e-6)


@pytest.mark.parametrize("k", [0, 1])
def test_fit_sigma_is_unit_cost_change_for_one_linear_parameter(k):
    """With one linear parameter free the cost is an exact parabola: moving it
    by +-sigma from the minimum raises chi^2 by exactly 1 (Eq. 2 read as
    -2 ln L up to a constant)."""
    th, h, counts, truth = _linear_case(seed=102 + k)
    fixed = np.ones(6, bool)
    fixed[k] = False
    start = truth.copy()
    start[k] *= 1.05
    r = fit.fit(th, h, counts, start, "chi2", fixed=fixed)
    s = r["sigma"][0]
    c0 = model.cost(th, h, counts, r["p"])
    for sgn in (1.0, -1.0):
        q = r["p"].copy()
        q[k] += sgn * s
        assert model.cost(th, h, counts, q) - c0 == pytest.approx(1.0, abs=1e-6)
