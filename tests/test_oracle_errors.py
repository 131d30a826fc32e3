"""Pins of the oracle's parameter-error functions (oracle/errors.py) against
closed forms and an independent route.

* Gauss-Newton Hessian: (a) in the (N0, Nbkg) block, where N is linear in the
  two parameters, it equals exactly twice the weighted normal matrix of the
  least-squares problem (Eq. 2 with weights 1/v); (b) on noiseless
  non-integer data at the true parameters every residual vanishes, so it
  equals the full Hessian of the cost, here from Richardson central
  differences of the oracle's analytic gradient (every parameter, both
  costs).
* Profile and MINOS errors: with only N0 and Nbkg free, chi^2 is exactly
  quadratic, so the profile in N0 is the parabola f_min + (N0 - N0*)^2 /
  sigma^2 with sigma^2 from the covariance 2 H^-1, and the two crossings of
  f_min + 1 sit at -sigma and +sigma.
"""

import math

import numpy as np

import synth
from oracle import errors, fit as ofit, model

from _workloads import counts_for


def _small(n_bins=600, dt=0.012, seed=7, noiseless=False, theory=None, p=None):
    th = theory or synth.theory_exp_cos()
    p = p if p is not None else np.array([900.0, 4.0, 0.21, 0.6, 1.3, 0.4])
    h = [{"n_bins": n_bins, "dt": dt, "t0_bin": 0.0, "first": 0, "last": n_bins - 1, "map_row": 0}]
    c = counts_for(th, h, p, np.random.default_rng(seed), noiseless=noiseless)
    return th, h, c, p


def _normal_matrix(th, h, counts, p):
    res = model.resolve(th, p, 0)
    t = model.time_grid(h)
    u = np.exp(-t / th["tau_mu"]) * (1.0 + model.asymmetry(th, t, res))
    d = np.asarray(counts, dtype=np.float64)[h["first"]:h["last"] + 1]
    w = 1.0 / np.where(d > 0, d, 1.0)
    return np.array([[math.fsum(w * u * u), math.fsum(w * u)], [math.fsum(w * u), math.fsum(w)]])


def test_gauss_newton_linear_block_is_twice_the_normal_matrix():
    th, h, c, p = _small()
    q = p * 1.01
    H = errors.gauss_newton_hessian(th, h, c, q)
    M = _normal_matrix(th, h[0], c[0], q)
    np.testing.assert_allclose(H[:2, :2], 2.0 * M, rtol=1e-14)


def _hess_fd(th, h, c, p, kind, rel=1e-4):
    n = p.size
    H = np.zeros((n, n))
    for k in range(n):
        hk = rel * max(abs(p[k]), 1e-2)

        def cd(s):
            pp, pm = p.copy(), p.copy()
            pp[k] += s
            pm[k] -= s
            return (model.grad(th, h, c, pp, kind) - model.grad(th, h, c, pm, kind)) / (2 * s)

        H[:, k] = (4.0 * cd(hk / 2) - cd(hk)) / 3.0
    return 0.5 * (H + H.T)


def test_gauss_newton_equals_full_hessian_without_residuals():
    for th, p in ((synth.theory_exp_cos(), np.array([900.0, 4.0, 0.21, 0.6, 1.3, 0.4])),
                  (synth.theory_exp_gkt(), np.array([900.0, 3.0, 0.15, 0.8, 0.12, 0.4]))):
        th, h, c, p = _small(theory=th, p=p, noiseless=True)
        for kind in ("chi2", "poisson"):
            H = errors.gauss_newton_hessian(th, h, c, p, kind)
            Hfd = _hess_fd(th, h, c, p, kind)
            scale = np.sqrt(np.outer(np.abs(np.diag(H)), np.abs(np.diag(H))))
            assert np.all(np.abs(H - Hfd) <= 1e-6 * scale), (kind, np.max(np.abs(H - Hfd) / scale))


def test_covariance_inverts_the_free_block():
    H = np.array([[4.0, 1.0, 0.5], [1.0, 3.0, 0.2], [0.5, 0.2, 2.0]])
    C = errors.covariance(H, fixed=[False, True, False])
    assert np.all(C[1] == 0) and np.all(C[:, 1] == 0)
    idx = [0, 2]
    np.testing.assert_allclose(C[np.ix_(idx, idx)] @ H[np.ix_(idx, idx)], 2.0 * np.eye(2), atol=1e-15)


def test_profile_and_minos_of_a_quadratic_cost():
    th, h, c, p = _small(seed=8)
    fixed = np.array([False, False, True, True, True, True])
    fmin = ofit.fit(th, h, c, p * np.array([1.1, 0.7, 1, 1, 1, 1]), fixed=fixed)
    pm = fmin["p"]
    H = errors.gauss_newton_hessian(th, h, c, pm)
    sig = math.sqrt(errors.covariance(H, fixed)[0, 0])
    xs = pm[0] + sig * np.array([-1.5, -0.5, 0.7, 2.0])
    prof = errors.profile(th, h, c, pm, 0, xs, fixed=fixed)
    expect = fmin["cost"] + ((xs - pm[0]) / sig) ** 2
    np.testing.assert_allclose(prof, expect, rtol=1e-10)
    lo, hi = errors.minos(th, h, c, pm, 0, fixed=fixed)
    assert abs(lo + sig) <= 1e-7 * sig and abs(hi - sig) <= 1e-7 * sig, (lo, hi, sig)
