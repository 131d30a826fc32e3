"""Pure-Python, one-bin-at-a-time evaluation of the same definitions as
``oracle.model`` (Eqs. 1-3, Listings 2-3), using only the ``math`` module.

It exists to cross-check the vectorised oracle on tiny inputs; it is written
separately so that a vectorisation or indexing slip in one does not hide in
the other.  Test infrastructure only.
"""

from __future__ import annotations

import math


def _ref(theory, ref, p, row):
    kind, x = ref
    if kind == "p":
        return p[theory["map"][row][x]]
    if kind == "f":
        i = theory["map"][row][x]
        F = theory["F"][i]
        return math.fsum(F[k] * p[k] for k in range(len(p))) + theory["f0"][i]
    return x


def prim1(kind, t, a):
    if kind == "se":
        return math.exp(-a[0] * t)
    if kind == "ge":
        return math.exp(-((a[0] * t) ** a[1]))
    if kind == "sg":
        return math.exp(-0.5 * (a[0] * t) ** 2)
    if kind == "stg":
        s2 = (a[0] * t) ** 2
        return 1.0 / 3.0 + (2.0 / 3.0) * (1.0 - s2) * math.exp(-0.5 * s2)
    if kind == "tf":
        return math.cos(2.0 * math.pi * a[1] * t + a[0])
    raise ValueError(kind)


def model_bin(theory, h, p, n):
    """N(t_n) for bin n of histogram h (Eq. 1)."""
    row = h["map_row"]
    t = (n - h["t0_bin"]) * h["dt"]
    A = 0.0
    for term in theory["terms"]:
        v = term["coef"] * _ref(theory, term["amp"], p, row)
        for fac in term["factors"]:
            v *= prim1(fac["prim"], t, [_ref(theory, r, p, row) for r in fac["args"]])
        A += v
    n0 = _ref(theory, theory["n0"], p, row)
    nb = _ref(theory, theory["nbkg"], p, row)
    return n0 * math.exp(-t / theory["tau_mu"]) * (1.0 + A) + nb


def term_bin(d, N, kind):
    """One bin's cost term (Eq. 2 or Eq. 3)."""
    if kind == "chi2":
        v = d if d > 0 else 1.0
        return (d - N) ** 2 / v
    if d == 0:
        return 2.0 * N
    if N <= 0:
        return math.inf
    return 2.0 * ((N - d) + d * math.log(d / N))


def cost(theory, histos, counts, p, kind="chi2"):
    terms = []
    for h, c in zip(histos, counts):
        for n in range(h["first"], h["last"] + 1):
            terms.append(term_bin(float(c[n]), model_bin(theory, h, p, n), kind))
    return math.fsum(terms)
