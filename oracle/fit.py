"""Reference minimiser of the chi^2 / likelihood cost (test infrastructure).

The paper minimises its cost with Minuit2's ``minimize`` (Sec. 4, Table 1).
This oracle reaches the same minimum by a different, plainly checkable route:
scipy's BFGS with the oracle's analytic gradient, then Newton steps with a
Hessian from central differences of that gradient, until every relative step
is below 1e-12.  The covariance is 2 H^-1: both costs are -2 ln(likelihood)
up to a constant, so a change of 1 in the cost is one standard deviation.
"""

from __future__ import annotations

import numpy as np
from scipy.optimize import minimize

from . import model


def _hessian(fun_g, x, scale):
    n = x.size
    H = np.zeros((n, n))
    for k in range(n):
        h = 1e-5 * scale[k]
        xp = x.copy()
        xm = x.copy()
        xp[k] += h
        xm[k] -= h
        H[:, k] = (fun_g(xp) - fun_g(xm)) / (2 * h)
    return 0.5 * (H + H.T)


def fit(theory, histos, counts, start, kind="chi2", fixed=None, polish_iters=20):
    """Minimise the cost from ``start``.  Returns a dict with the parameters,
    cost, covariance (free block), Hessian condition number and counts of
    evaluations."""
    start = np.asarray(start, dtype=np.float64)
    fixed = np.zeros(start.size, bool) if fixed is None else np.asarray(fixed, bool)
    free = np.nonzero(~fixed)[0]
    n_eval = [0]

    def full(x):
        p = start.copy()
        p[free] = x
        return p

    def f(x):
        n_eval[0] += 1
        return model.cost(theory, histos, counts, full(x), kind)

    def g(x):
        return model.grad(theory, histos, counts, full(x), kind)[free]

    x = start[free].copy()
    res = minimize(f, x, jac=g, method="BFGS", options={"gtol": 1e-9, "maxiter": 20000})
    x = res.x
    scale = np.maximum(np.abs(x), 1e-3)
    H = _hessian(g, x, scale)
    for _ in range(polish_iters):
        gx = g(x)
        try:
            step = -np.linalg.solve(H, gx)
        except np.linalg.LinAlgError:
            break
        # accept only steps that do not raise the cost (pure Newton near the minimum)
        cur = f(x)
        xn = x + step
        if f(xn) > cur + 1e-12 * abs(cur):
            break
        x = xn
        sig = np.sqrt(np.abs(np.diag(2.0 * np.linalg.inv(H))))
        if np.all(np.abs(step) <= 1e-12 * np.maximum(np.abs(x), sig)):
            break
        H = _hessian(g, x, np.maximum(np.abs(x), 1e-3))
    H = _hessian(g, x, np.maximum(np.abs(x), 1e-3))
    cov = 2.0 * np.linalg.inv(H)
    return {"p": full(x), "cost": f(x), "cov": cov, "free": free,
            "sigma": np.sqrt(np.abs(np.diag(cov))), "cond": float(np.linalg.cond(H)),
            "n_eval": n_eval[0], "scipy_status": int(res.status)}


def linear_n0_nbkg(theory, h, counts, p):
    """Exact chi^2 minimiser over (N0, Nbkg) with every other parameter held:
    N = N0 u + Nbkg with u = e^(-t/tau) (1 + A) is linear in the two, and
    the weights 1/v do not depend on the parameters, so the weighted normal
    equations give the minimum in closed form.  Requires map slots 0 and 1
    to be plain parameter references for N0 and Nbkg."""
    res = model.resolve(theory, p, h["map_row"])
    t = model.time_grid(h)
    a = model.asymmetry(theory, t, res)
    u = np.exp(-t / theory["tau_mu"]) * (1.0 + a)
    d = np.asarray(counts, dtype=np.float64)[h["first"]:h["last"] + 1]
    w = 1.0 / np.where(d > 0, d, 1.0)
    M = np.array([[np.sum(w * u * u), np.sum(w * u)], [np.sum(w * u), np.sum(w)]])
    r = np.array([np.sum(w * u * d), np.sum(w * d)])
    return np.linalg.solve(M, r)
