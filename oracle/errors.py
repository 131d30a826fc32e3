"""Parameter errors after the minimum (test infrastructure only).

The paper's fits end with Minuit2's minimisation (Sec. 4, Table 1); the usual
next steps are a Hessian-based covariance and likelihood-profile errors.  Both
costs are -2 ln(likelihood) up to a constant (Eqs. 2-3), so the covariance is
2 H^-1 and a change of `up` = 1 in the profiled cost marks one standard
deviation.

* gauss_newton_hessian: H_kl = sum_n c_n (dN_n/dp_k) (dN_n/dp_l), with
  c_n = d^2 term / dN^2 at the bin: 2 / v for chi^2 (v = d, or 1 for d = 0)
  and 2 d / N^2 for the likelihood; the terms with the residual times the
  second derivative of N are dropped.  Each element is an exactly rounded sum.
* profile: the cost minimised over every other free parameter with p_k held
  at each given value (the oracle's own minimiser).
* minos: the two values of p_k where the profile rises by `up` above the
  minimum, found by bracketing and bisection of the profile.
"""

from __future__ import annotations

import math

import numpy as np

from . import fit as ofit
from . import model


def cost_d2N(d, N, kind):
    """Second derivative of the per-bin term in N: 2/v (chi^2), 2 d / N^2 (likelihood)."""
    d = np.asarray(d, dtype=np.float64)
    if kind == "chi2":
        return 2.0 / np.where(d > 0, d, 1.0)
    if kind == "poisson":
        return 2.0 * d / (N * N)
    raise ValueError(f"unknown cost {kind!r}")


def jacobian(theory, h, p):
    """dN_n/dp_k over the fit range of histogram h: [bins][n_par] (chain rule
    through the map and the function array)."""
    p = np.asarray(p, dtype=np.float64)
    res = model.resolve(theory, p, h["map_row"])
    t = model.time_grid(h)
    J = np.zeros((t.size, p.size))
    for (_, _, jac), dN in zip(res, model._dN_dres(theory, t, res)):
        for k in np.nonzero(jac)[0]:
            J[:, k] += dN * jac[k]
    return J


def gauss_newton_hessian(theory, histos, counts, p, kind="chi2"):
    p = np.asarray(p, dtype=np.float64)
    n = p.size
    parts = [[[] for _ in range(n)] for _ in range(n)]
    for h, c in zip(histos, counts):
        d = np.asarray(c, dtype=np.float64)[h["first"]:h["last"] + 1]
        N = model.model(theory, h, p)
        w = cost_d2N(d, N, kind)
        J = jacobian(theory, h, p)
        for k in range(n):
            if not np.any(J[:, k]):
                continue
            for l in range(k, n):
                if np.any(J[:, l]):
                    parts[k][l].append(w * J[:, k] * J[:, l])
    H = np.zeros((n, n))
    for k in range(n):
        for l in range(k, n):
            if parts[k][l]:
                H[k, l] = H[l, k] = math.fsum(np.concatenate(parts[k][l]))
    return H


def covariance(H, fixed=None):
    """2 H^-1 over the free block (zero rows and columns for fixed parameters)."""
    n = H.shape[0]
    free = np.ones(n, bool) if fixed is None else ~np.asarray(fixed, bool)
    C = np.zeros((n, n))
    idx = np.nonzero(free)[0]
    C[np.ix_(idx, idx)] = 2.0 * np.linalg.inv(H[np.ix_(idx, idx)])
    return C


def profile(theory, histos, counts, p_min, k, values, kind="chi2", fixed=None):
    """Profile cost at each value of parameter k (every other free parameter
    minimised), with the minimiser started from p_min."""
    p_min = np.asarray(p_min, dtype=np.float64)
    fx = np.zeros(p_min.size, bool) if fixed is None else np.asarray(fixed, bool).copy()
    fx[k] = True
    out = []
    for v in values:
        s = p_min.copy()
        s[k] = v
        out.append(ofit.fit(theory, histos, counts, s, kind, fixed=fx)["cost"])
    return np.array(out)


def minos(theory, histos, counts, p_min, k, kind="chi2", up=1.0, fixed=None, sigma=None, rtol=1e-9):
    """(lower, upper) errors of parameter k: p_k - p_min_k at the two points
    where the profile equals cost(p_min) + up (bisection on brackets that
    start one Hessian standard deviation out and double until they hold)."""
    p_min = np.asarray(p_min, dtype=np.float64)
    f0 = model.cost(theory, histos, counts, p_min, kind)
    if sigma is None:
        H = gauss_newton_hessian(theory, histos, counts, p_min, kind)
        sigma = math.sqrt(covariance(H, fixed)[k, k])

    def excess(x):
        return profile(theory, histos, counts, p_min, k, [x], kind, fixed)[0] - f0 - up

    errs = []
    for sgn in (-1.0, 1.0):
        a, b = 0.0, sgn * sigma
        while excess(p_min[k] + b) < 0.0:
            a, b = b, 2.0 * b
        for _ in range(200):
            m = 0.5 * (a + b)
            if excess(p_min[k] + m) < 0.0:
                a = m
            else:
                b = m
            if abs(b - a) <= rtol * sigma:
                break
        errs.append(0.5 * (a + b))
    return errs[0], errs[1]
