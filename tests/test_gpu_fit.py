"""GPU fits (mu_fit_batch) against the oracle's reference minimiser and the
closed-form least-squares minimum.  Bar: parameters within 1e-6 of
max(|p_k|, sigma_k) of the reference; the (N0, Nbkg) least-squares special
case within 1e-10 relative."""

import numpy as np
import pytest

import synth
from oracle import fit as ofit
from oracle import model
from paper_1604_02334_amd import api

from _workloads import counts_for

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    c = api.Context(0)
    yield c
    c.close()


def _say(*a):
    print("[case]", *a, flush=True)


def _agree(p, ref, sigma, tol=1e-6):
    scale = np.maximum(np.abs(ref), sigma)
    return np.all(np.abs(p - ref) <= tol * scale), np.max(np.abs(p - ref) / scale)


def _small_c1(n_bins=2048, dt=0.004, seed=41):
    cfg = synth.config_c1()
    h = [dict(cfg["histos"][0], n_bins=n_bins, last=n_bins - 1, dt=dt)]
    counts = counts_for(cfg["theory"], h, cfg["p_true"], np.random.default_rng(seed))
    return cfg["theory"], h, counts, cfg["p_true"]


@pytest.mark.parametrize("kind", ["chi2", "poisson"])
def test_fit_matches_oracle_fit(ctx, kind):
    _say("fit vs oracle", kind)
    th_d, h, counts, truth = _small_c1()
    start = truth * np.array([1.04, 0.95, 1.05, 0.96, 1.01, 1.0]) + np.array([0, 0, 0, 0, 0, 0.03])
    ref = ofit.fit(th_d, h, counts, start, kind)
    th, d = api.Theory(ctx, th_d), api.Data(ctx, h, counts)
    p, cov, res = api.fit_batch(ctx, [d], [th], start[None], kind)
    assert res[0]["status"] == 0, res
    ok, worst = _agree(p[0], ref["p"], ref["sigma"])
    assert ok, (worst, p[0], ref["p"])
    assert abs(res[0]["cost"] - ref["cost"]) <= 1e-10 * ref["cost"]
    # covariance from the final Hessian agrees with the oracle's to a few percent
    np.testing.assert_allclose(np.sqrt(np.diag(cov[0])), ref["sigma"], rtol=2e-2)


def test_fit_matches_linear_least_squares(ctx):
    _say("fit linear lsq")
    th_d, h, counts, truth = _small_c1(seed=42)
    start = truth.copy()
    start[0] *= 1.2
    start[1] *= 0.5
    fixed = np.array([0, 0, 1, 1, 1, 1], dtype=np.uint8)
    th, d = api.Theory(ctx, th_d), api.Data(ctx, h, counts)
    p, _, res = api.fit_batch(ctx, [d], [th], start[None], fixed=fixed)
    exact = ofit.linear_n0_nbkg(th_d, h[0], counts[0], start)
    np.testing.assert_allclose(p[0][:2], exact, rtol=1e-10)
    np.testing.assert_array_equal(p[0][2:], start[2:])


def _same_minimum(pa, pb, cov, tol=1e-6):
    """Two fits of one dataset agree when every parameter differs by at most
    tol * max(|p_k|, sigma_k) (sigma from the covariance 2V).  Where the
    correlation matrix has condition above 1e6 (a parameter combination the
    data barely determine) the test is made along the eigen-directions of
    the covariance in those scaled units: each direction whose standard
    deviation is at most 1 (determined to better than the parameter scale)
    must agree to tol; looser directions are not compared.  Returns (ok,
    worst ratio, ill-conditioned)."""
    sig = np.sqrt(np.abs(np.diag(cov)))
    scale = np.maximum(np.abs(pa), sig)
    d = (pa - pb) / scale
    corr = cov / np.outer(np.where(sig > 0, sig, 1.0), np.where(sig > 0, sig, 1.0))
    ill = not np.all(np.isfinite(corr)) or np.linalg.cond(corr) > 1e6
    if not ill:
        return bool(np.all(np.abs(d) <= tol)), float(np.max(np.abs(d))), False
    w, Q = np.linalg.eigh(cov / np.outer(scale, scale))
    y = Q.T @ d
    sel = np.sqrt(np.maximum(w, 0.0)) <= 1.0
    worst = float(np.max(np.abs(y[sel]))) if np.any(sel) else 0.0
    return worst <= tol, worst, True


def test_batched_and_plain_paths_agree(ctx):
    """Uneven independent datasets: the batched path (one launch per round,
    analytic gradients) and the plain path (one launch per cost evaluation,
    central differences) reach the same minimum within 1e-6 of
    max(|p|, sigma) (along the determined directions where the covariance is
    nearly degenerate); the plain one needs many more evaluations.  Every
    fit must converge (EDM below tolerance) unless its covariance is
    degenerate; the exceptions are counted by cause."""
    _say("batched vs plain")
    cfg = synth.config_c4(n_sets=12, lo_exp=11, hi_exp=13)
    rng = cfg["rng"]
    sets = cfg["sets"]
    ths = [api.Theory(ctx, s["theory"]) for s in sets]
    cnts = [counts_for(s["theory"], s["histos"], s["p_true"], rng) for s in sets]
    ds = [api.Data(ctx, s["histos"], c) for s, c in zip(sets, cnts)]
    ld = 6
    start = np.zeros((len(sets), ld))
    for j, s in enumerate(sets):
        start[j, :s["start"].size] = s["start"]
    pb, covb, rb = api.fit_batch(ctx, ds, ths, start)
    pp, covp, rp = api.fit_batch(ctx, ds, ths, start, analytic_grad=False, batched=False)
    causes = {"compared": 0, "compared_degenerate": 0, "unconverged_degenerate": 0}
    for j, s in enumerate(sets):
        n = s["start"].size
        ok, worst, ill = _same_minimum(pb[j, :n], pp[j, :n], covb[j][:n, :n])
        if rb[j]["status"] != 0 or rp[j]["status"] != 0:
            # only a fit in a degenerate valley may stay unconverged
            assert ill, (j, s["family"], rb[j], rp[j])
            causes["unconverged_degenerate"] += 1
            continue
        causes["compared_degenerate" if ill else "compared"] += 1
        assert ok, (j, s["family"], worst, pb[j, :n], pp[j, :n])
    print("[fits]", causes, flush=True)
    assert causes["compared"] >= len(sets) - 2
    assert sum(r["n_fcn"] for r in rp) > sum(r["n_fcn"] for r in rb)


def test_fit_c2_shape_reduced(ctx):
    """The 16-detector, 52-parameter theory on a reduced grid against the
    oracle's minimiser."""
    _say("fit c2 reduced")
    cfg = synth.config_c2()
    hs = [dict(h, n_bins=1024, last=1023, dt=0.0128) for h in cfg["histos"]]
    counts = counts_for(cfg["theory"], hs, cfg["p_true"], np.random.default_rng(43))
    start = cfg["p_true"] * (1.0 + 0.02 * np.cos(np.arange(cfg["p_true"].size)))
    ref = ofit.fit(cfg["theory"], hs, counts, start)
    th, d = api.Theory(ctx, cfg["theory"]), api.Data(ctx, hs, counts)
    p, cov, res = api.fit_batch(ctx, [d], [th], start[None])
    assert res[0]["status"] == 0, res
    ok, worst = _agree(p[0], ref["p"], ref["sigma"])
    assert ok, worst


def test_fit_edge_cases(ctx):
    _say("fit edges")
    th_d, h, counts, truth = _small_c1(n_bins=512, seed=44)
    th, d = api.Theory(ctx, th_d), api.Data(ctx, h, counts)
    bad = truth.copy()
    bad[2] = np.nan
    with pytest.raises(api.A.MuError):
        api.fit_batch(ctx, [d], [th], bad[None])
    p, _, res = api.fit_batch(ctx, [d], [th], (truth * 1.1)[None], max_fcn=3, polish=False)
    assert res[0]["status"] == 1
    neg = truth.copy()
    neg[0], neg[1] = -1e3, 0.0
    p, _, res = api.fit_batch(ctx, [d], [th], neg[None], cost="poisson")
    assert res[0]["status"] == 2
    # all parameters fixed: nothing moves
    p, _, res = api.fit_batch(ctx, [d], [th], truth[None], fixed=np.ones(6, np.uint8))
    np.testing.assert_array_equal(p[0], truth)


def test_multi_run_fit(ctx):
    """Two runs of different binning and time origin fitted together: lambda
    shared, amplitude and frequency per run, N0, Nbkg and phase per
    histogram (one dataset holding both runs' histograms, one map row per
    histogram).  Against the oracle's minimiser at 1e-6 of max(|p|, sigma)."""
    _say("multi-run fit")
    cfg = synth.config_multi_run()
    th_d, hs = cfg["theory"], cfg["histos"]
    counts = counts_for(th_d, hs, cfg["p_true"], cfg["rng"])
    start = cfg["p_true"] * (1.0 + 0.02 * np.cos(np.arange(cfg["p_true"].size)))
    ref = ofit.fit(th_d, hs, counts, start)
    th, d = api.Theory(ctx, th_d), api.Data(ctx, hs, counts)
    p, cov, res = api.fit_batch(ctx, [d], [th], start[None])
    assert res[0]["status"] == 0, res
    ok, worst = _agree(p[0], ref["p"], ref["sigma"])
    assert ok, worst
    H, c = api.hesse(ctx, d, th, p[0], method="diff")
    np.testing.assert_allclose(np.sqrt(np.diag(c)), ref["sigma"], rtol=1e-4)
