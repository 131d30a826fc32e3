"""Parameter errors after the minimum against the oracle (oracle/errors.py):

* mu_hesse Gauss-Newton (Jacobian rows + FP64 matrix-core Gram kernel + host
  chain rule): every element within 1e-10 sqrt(H_kk H_ll) of the oracle's
  exactly summed Gauss-Newton Hessian (Cauchy-Schwarz bounds the sum of
  |c J_k J_l| by that scale), for both costs, on single-histogram theories,
  the 16-detector 52-parameter theory, the paper's Eq. 4 with its function
  array, and a three-term theory whose resolved scalars fill all four 16 x 16
  blocks of the Gram matrix; in the linear (N0, Nbkg) block, twice the
  weighted normal matrix (closed form).
* mu_hesse by differences of the analytic gradient: on noiseless data at the
  true parameters (no residuals) it equals the Gauss-Newton Hessian to 1e-6.
* The covariance 2 H^-1 of the free block against the oracle's.
* mu_profile and mu_minos: in the linear case the profile is the exact
  parabola f_min + ((x - x*) / sigma)^2 and the crossings are -sigma, +sigma;
  on a nonlinear parameter the crossings match the oracle's bisection of its
  own profile to 1e-6 sigma.
"""

import math

import numpy as np
import pytest

import synth
from oracle import errors, fit as ofit, model
from paper_1604_02334_amd import api

from _workloads import counts_for, perturbed

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    c = api.Context(0)
    yield c
    c.close()


def _say(*a):
    print("[case]", *a, flush=True)


def _three_term():
    """A = A1 se(l1) tf(phi, nu) + A2 sg(s) tf(phi2, nu) + A3 stg(s3) se(l3):
    resolved scalars up to index 23 (beyond the first 16 x 16 block)."""
    th = synth.theory_exp_cos()
    th["terms"] = [
        {"coef": 1.0, "amp": ("p", 2), "factors": [{"prim": "se", "args": [("p", 3)]},
                                                   {"prim": "tf", "args": [("p", 5), ("p", 4)]}]},
        {"coef": 1.0, "amp": ("p", 6), "factors": [{"prim": "sg", "args": [("p", 7)]},
                                                   {"prim": "tf", "args": [("p", 8), ("p", 4)]}]},
        {"coef": 1.0, "amp": ("p", 9), "factors": [{"prim": "stg", "args": [("p", 10)]},
                                                   {"prim": "se", "args": [("p", 11)]}]},
    ]
    th["map"] = [list(range(12))]
    th["n_par"] = 12
    th["names"] = [f"p{i}" for i in range(12)]
    p = np.array([900.0, 3.0, 0.15, 0.6, 1.7, 0.3, 0.08, 0.5, 1.1, 0.05, 0.4, 0.2])
    return th, p


def _cases():
    rng = np.random.default_rng(61)
    h1 = [{"n_bins": 3000, "dt": 0.003, "t0_bin": 0.0, "first": 4, "last": 2990, "map_row": 0}]
    out = []
    for th, p in ((synth.theory_exp_cos(), np.array([900.0, 3.0, 0.2, 0.8, 1.7, 0.3])),
                  (synth.theory_exp_gkt(), np.array([900.0, 3.0, 0.15, 0.8, 0.12, 0.4])),
                  _three_term()):
        out.append((th, h1, counts_for(th, h1, p, rng), perturbed(p, 1e-2, 62)))
    c2 = synth.config_c2()
    hs = [dict(h, n_bins=2048, last=2047, dt=0.0064) for h in c2["histos"]]
    out.append((c2["theory"], hs, counts_for(c2["theory"], hs, c2["p_true"], rng), perturbed(c2["p_true"], 1e-2, 63)))
    ps = synth.config_paper_shape(n_bins=1500)
    hs = ps["histos"]
    out.append((ps["theory"], hs, counts_for(ps["theory"], hs, ps["p_true"], rng), perturbed(ps["p_true"], 1e-3, 64)))
    return out


@pytest.mark.parametrize("kind", ["chi2", "poisson"])
def test_gauss_newton_hessian_against_oracle(ctx, kind):
    _say("hesse gauss-newton", kind)
    for th_d, hs, cnt, p in _cases():
        th, d = api.Theory(ctx, th_d), api.Data(ctx, hs, cnt)
        H, cov = api.hesse(ctx, d, th, p, kind)
        ref = errors.gauss_newton_hessian(th_d, hs, cnt, p, kind)
        dg = np.sqrt(np.abs(np.diag(ref)))
        scale = np.outer(dg, dg)
        assert np.all(np.abs(H - ref) <= 1e-10 * scale), (th_d["n_par"], np.max(np.abs(H - ref) / np.maximum(scale, 1e-300)))
        assert cov is not None
        cref = errors.covariance(ref)
        sg = np.sqrt(np.abs(np.diag(cref)))
        assert np.all(np.abs(cov - cref) <= 1e-6 * np.outer(sg, sg))
        th.close()
        d.close()


def test_gauss_newton_linear_block_closed_form(ctx):
    _say("hesse linear block")
    th_d, hs, cnt, p = _cases()[0]
    th, d = api.Theory(ctx, th_d), api.Data(ctx, hs, cnt)
    H, _ = api.hesse(ctx, d, th, p)
    res = model.resolve(th_d, p, 0)
    t = model.time_grid(hs[0])
    u = np.exp(-t / th_d["tau_mu"]) * (1.0 + model.asymmetry(th_d, t, res))
    dd = np.asarray(cnt[0], dtype=np.float64)[hs[0]["first"]:hs[0]["last"] + 1]
    w = 1.0 / np.where(dd > 0, dd, 1.0)
    M = np.array([[math.fsum(w * u * u), math.fsum(w * u)], [math.fsum(w * u), math.fsum(w)]])
    np.testing.assert_allclose(H[:2, :2], 2.0 * M, rtol=1e-11)
    # fixed parameters: zero rows and columns, covariance of the free block
    fixed = np.array([0, 0, 1, 1, 1, 1], np.uint8)
    Hf, cov = api.hesse(ctx, d, th, p, fixed=fixed)
    assert np.all(Hf[2:] == 0) and np.all(Hf[:, 2:] == 0)
    np.testing.assert_allclose(cov[:2, :2], np.linalg.inv(M), rtol=1e-10)
    th.close()
    d.close()


def test_difference_hessian_equals_gauss_newton_without_residuals(ctx):
    _say("hesse diff vs gn, noiseless")
    for th_d, p in ((synth.theory_exp_cos(), np.array([900.0, 3.0, 0.2, 0.8, 1.7, 0.3])),
                    (synth.theory_exp_gkt(), np.array([900.0, 3.0, 0.15, 0.8, 0.12, 0.4]))):
        hs = [{"n_bins": 3000, "dt": 0.003, "t0_bin": 0.0, "first": 0, "last": 2999, "map_row": 0}]
        cnt = counts_for(th_d, hs, p, None, noiseless=True)
        th, d = api.Theory(ctx, th_d), api.Data(ctx, hs, cnt)
        for kind in ("chi2", "poisson"):
            Hg, _ = api.hesse(ctx, d, th, p, kind)
            Hd, _ = api.hesse(ctx, d, th, p, kind, method="diff")
            dg = np.sqrt(np.abs(np.diag(Hg)))
            assert np.all(np.abs(Hd - Hg) <= 1e-6 * np.outer(dg, dg)), kind
        th.close()
        d.close()


def test_profile_and_minos_linear_case(ctx):
    _say("profile / minos, linear")
    th_d, hs, cnt, p = _cases()[0]
    th, d = api.Theory(ctx, th_d), api.Data(ctx, hs, cnt)
    fixed = np.array([0, 0, 1, 1, 1, 1], np.uint8)
    pm, _, r = api.fit_batch(ctx, [d], [th], (p * np.array([1.1, 0.7, 1, 1, 1, 1]))[None], fixed=fixed)
    pm = pm[0]
    H, cov = api.hesse(ctx, d, th, pm, fixed=fixed)
    sig = math.sqrt(cov[0, 0])
    fmin = r[0]["cost"]
    xs = pm[0] + sig * np.array([-1.5, -0.5, 0.7, 2.0])
    pc, pp, st = api.profile(ctx, d, th, pm, 0, xs, fixed=fixed)
    np.testing.assert_allclose(pc, fmin + ((xs - pm[0]) / sig) ** 2, rtol=1e-11)
    ref = errors.profile(th_d, hs, cnt, pm, 0, xs, fixed=fixed.astype(bool))
    np.testing.assert_allclose(pc, ref, rtol=1e-11)
    lo, hi, rounds = api.minos(ctx, d, th, pm, 0, fixed=fixed)
    assert abs(lo + sig) <= 1e-7 * sig and abs(hi - sig) <= 1e-7 * sig, (lo, hi, sig, rounds)
    th.close()
    d.close()


def test_minos_nonlinear_parameter_against_oracle(ctx):
    _say("minos nonlinear")
    th_d = synth.theory_exp_cos()
    p = np.array([900.0, 4.0, 0.21, 0.6, 1.3, 0.4])
    hs = [{"n_bins": 600, "dt": 0.012, "t0_bin": 0.0, "first": 0, "last": 599, "map_row": 0}]
    cnt = counts_for(th_d, hs, p, np.random.default_rng(65))
    th, d = api.Theory(ctx, th_d), api.Data(ctx, hs, cnt)
    pm, _, r = api.fit_batch(ctx, [d], [th], p[None])
    pm = pm[0]
    assert r[0]["status"] == 0
    for k in (3, 4):  # lambda, nu
        lo, hi, rounds = api.minos(ctx, d, th, pm, k)
        rlo, rhi = errors.minos(th_d, hs, cnt, pm, k)
        sig = 0.5 * (rhi - rlo)
        assert abs(lo - rlo) <= 1e-6 * sig and abs(hi - rhi) <= 1e-6 * sig, (k, lo, rlo, hi, rhi, rounds)
        assert lo < 0 < hi
    th.close()
    d.close()
