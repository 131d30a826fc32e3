"""FP64 oracle of the histogram model, the two cost functions and their
analytic gradient (test infrastructure only; see the package docstring).

Definitions followed, in the paper's order:

1. function array f = F p + f0 (Sec. 4.2.1: "precomputed function values";
   affine form is this oracle's reading);
2. per histogram j, N0^j, Nbkg^j and every primitive argument are read through
   the map row of j (parameter set P^j of Sec. 4.1; map array of Listing 3);
3. time of bin n: t = (n - t0_bin) dt (Eq. 1 text);
4. asymmetry A(t) = sum_k coef_k amp_k prod_i prim_ki(t) (Listings 2-3);
5. N = N0 e^(-t/tau_mu) (1 + A) + Nbkg (Eq. 1);
6. per-bin cost: chi^2 term (d - N)^2 / v with v = d, or 1 for d = 0 (Eq. 2);
   likelihood term 2 [(N - d) + d ln(d/N)], 2N for d = 0, +inf for N <= 0 < d
   (Eq. 3, minimised);
7. total = exactly rounded sum (math.fsum) over every bin of every histogram.
"""

from __future__ import annotations

import math

import numpy as np

PRIM_NARGS = {"se": 1, "ge": 2, "sg": 1, "stg": 1, "tf": 2}
COST_KINDS = ("chi2", "poisson")


# ---------------------------------------------------------------------------
# Step 1-2: parameter resolution
# ---------------------------------------------------------------------------

def function_array(theory, p):
    """f = F p + f0 (Sec. 4.2.1, function array)."""
    F = theory.get("F")
    if F is None:
        return np.zeros(0)
    F = np.asarray(F, dtype=np.float64)
    f0 = np.asarray(theory["f0"], dtype=np.float64)
    return np.array([math.fsum(F[i] * p) + f0[i] for i in range(F.shape[0])])


def _ref_value_and_jac(theory, ref, p, f, row):
    """Value of one argument reference and its derivative with respect to p.

    ("p", s) -> p[m[row][s]];  ("f", s) -> f[m[row][s]];  ("lit", x) -> x
    (map array, Listing 3)."""
    n_par = p.size
    kind, x = ref
    jac = np.zeros(n_par)
    if kind == "p":
        k = theory["map"][row][x]
        jac[k] = 1.0
        return float(p[k]), jac
    if kind == "f":
        i = theory["map"][row][x]
        jac[:] = np.asarray(theory["F"][i], dtype=np.float64)
        return float(f[i]), jac
    if kind == "lit":
        return float(x), jac
    raise ValueError(f"unknown reference kind {kind!r}")


def resolve(theory, p, row):
    """Resolved scalars of one (parameter vector, histogram) pair.

    Returns a list of (name, value, d value / d p) in a fixed order:
    N0, Nbkg, then per term its amplitude, then per factor its arguments."""
    p = np.asarray(p, dtype=np.float64)
    f = function_array(theory, p)
    out = [("n0",) + _ref_value_and_jac(theory, theory["n0"], p, f, row),
           ("nbkg",) + _ref_value_and_jac(theory, theory["nbkg"], p, f, row)]
    for k, term in enumerate(theory["terms"]):
        out.append((f"amp{k}",) + _ref_value_and_jac(theory, term["amp"], p, f, row))
        for i, fac in enumerate(term["factors"]):
            for a, ref in enumerate(fac["args"]):
                out.append((f"arg{k}.{i}.{a}",) + _ref_value_and_jac(theory, ref, p, f, row))
    return out


# ---------------------------------------------------------------------------
# Step 3-5: time grid, primitives, model
# ---------------------------------------------------------------------------

def time_grid(h):
    """t_n = (n - t0_bin) dt for n = first..last (Eq. 1 text)."""
    n = np.arange(h["first"], h["last"] + 1, dtype=np.float64)
    return (n - h["t0_bin"]) * h["dt"]


def prim(kind, t, args):
    """The predefined primitives (Listing 2) and the precession tf (Listing 3).

    se  = exp(-lambda t)
    ge  = exp(-(lambda t)^beta)
    sg  = exp(-(sigma t)^2 / 2)
    stg = 1/3 + 2/3 (1 - (sigma t)^2) exp(-(sigma t)^2 / 2)   (real division)
    tf  = cos(2 pi nu t + phi), args (phi, nu)
    """
    if kind == "se":
        (lam,) = args
        return np.exp(-lam * t)
    if kind == "ge":
        lam, beta = args
        return np.exp(-np.power(lam * t, beta))
    if kind == "sg":
        (sig,) = args
        return np.exp(-0.5 * (sig * t) ** 2)
    if kind == "stg":
        (sig,) = args
        s2 = (sig * t) ** 2
        return 1.0 / 3.0 + (2.0 / 3.0) * (1.0 - s2) * np.exp(-0.5 * s2)
    if kind == "tf":
        phi, nu = args
        return np.cos(2.0 * np.pi * nu * t + phi)
    raise ValueError(f"unknown primitive {kind!r}")


def prim_grad(kind, t, args):
    """Derivatives of each primitive with respect to each of its arguments."""
    if kind == "se":
        (lam,) = args
        return [-t * np.exp(-lam * t)]
    if kind == "ge":
        lam, beta = args
        x = lam * t
        xb = np.power(x, beta)
        g = np.exp(-xb)
        with np.errstate(divide="ignore", invalid="ignore"):
            d_lam = np.where(x > 0, -beta * xb / lam * g, (-t if beta == 1.0 else 0.0 * t))
            d_beta = np.where(x > 0, -xb * np.log(np.where(x > 0, x, 1.0)) * g, 0.0)
        return [d_lam, d_beta]
    if kind == "sg":
        (sig,) = args
        return [-sig * t * t * np.exp(-0.5 * (sig * t) ** 2)]
    if kind == "stg":
        (sig,) = args
        s2 = (sig * t) ** 2
        return [(2.0 / 3.0) * sig * t * t * (s2 - 3.0) * np.exp(-0.5 * s2)]
    if kind == "tf":
        phi, nu = args
        s = np.sin(2.0 * np.pi * nu * t + phi)
        return [-s, -2.0 * np.pi * t * s]
    raise ValueError(f"unknown primitive {kind!r}")


def _unpack(theory, res):
    vals = [v for (_, v, _) in res]
    n0, nbkg = vals[0], vals[1]
    pos = 2
    terms = []
    for term in theory["terms"]:
        amp = vals[pos]
        pos += 1
        facs = []
        for fac in term["factors"]:
            na = len(fac["args"])
            facs.append((fac["prim"], vals[pos:pos + na]))
            pos += na
        terms.append((term["coef"], amp, facs))
    return n0, nbkg, terms


def asymmetry(theory, t, res):
    """A(t) = sum_k coef_k amp_k prod_i prim_ki(t) (Listing 3)."""
    _, _, terms = _unpack(theory, res)
    a = np.zeros_like(t)
    for coef, amp, facs in terms:
        prod = np.full_like(t, coef * amp)
        for kind, args in facs:
            prod = prod * prim(kind, t, args)
        a = a + prod
    return a


def model(theory, h, p):
    """Expected counts N(t_n) over the fit range of histogram h (Eq. 1)."""
    res = resolve(theory, p, h["map_row"])
    n0, nbkg, _ = _unpack(theory, res)
    t = time_grid(h)
    a = asymmetry(theory, t, res)
    return n0 * np.exp(-t / theory["tau_mu"]) * (1.0 + a) + nbkg


def model_full(theory, h, p):
    """N over every bin 0..n_bins-1 of h, ignoring its fit range (used to
    draw synthetic counts)."""
    hh = dict(h)
    hh["first"], hh["last"] = 0, h["n_bins"] - 1
    return model(theory, hh, p)


# ---------------------------------------------------------------------------
# Step 6-7: cost
# ---------------------------------------------------------------------------

def cost_terms(d, N, kind):
    """Per-bin cost terms of Eq. 2 (chi2) or Eq. 3 (poisson)."""
    d = np.asarray(d, dtype=np.float64)
    if kind == "chi2":
        v = np.where(d > 0, d, 1.0)
        return (d - N) ** 2 / v
    if kind == "poisson":
        out = np.empty_like(N)
        pos = d > 0
        with np.errstate(divide="ignore", invalid="ignore"):
            lt = 2.0 * ((N - d) + d * np.log(d / N))
        out[pos] = lt[pos]
        out[~pos] = 2.0 * N[~pos]
        out[pos & (N <= 0)] = np.inf
        return out
    raise ValueError(f"unknown cost {kind!r}")


def cost_dN(d, N, kind):
    """d(term)/dN per bin: -2 (d - N) / v for chi2, 2 (1 - d/N) for poisson."""
    d = np.asarray(d, dtype=np.float64)
    if kind == "chi2":
        v = np.where(d > 0, d, 1.0)
        return -2.0 * (d - N) / v
    if kind == "poisson":
        with np.errstate(divide="ignore", invalid="ignore"):
            return np.where(d > 0, 2.0 * (1.0 - d / N), 2.0)
    raise ValueError(f"unknown cost {kind!r}")


def _fit_range(h, counts):
    return np.asarray(counts, dtype=np.float64)[h["first"]:h["last"] + 1]


def cost_per_histo(theory, histos, counts, p, kind="chi2"):
    """Cost of each histogram, each an exactly rounded sum of its terms."""
    out = []
    for h, c in zip(histos, counts):
        N = model(theory, h, p)
        out.append(math.fsum(cost_terms(_fit_range(h, c), N, kind)))
    return out


def cost(theory, histos, counts, p, kind="chi2"):
    """Total cost: exactly rounded sum over every bin of every histogram
    (Eq. 2 / Eq. 3 double sum over j and n)."""
    terms = []
    for h, c in zip(histos, counts):
        N = model(theory, h, p)
        terms.append(cost_terms(_fit_range(h, c), N, kind))
    return math.fsum(np.concatenate(terms)) if terms else 0.0


# ---------------------------------------------------------------------------
# Analytic gradient
# ---------------------------------------------------------------------------

def _dN_dres(theory, t, res):
    """dN/d(resolved scalar) per bin, in resolve()'s order (chain rule through
    Eq. 1 and the product form of A)."""
    n0, nbkg, terms = _unpack(theory, res)
    E = np.exp(-t / theory["tau_mu"])
    out = []
    a = np.zeros_like(t)
    per_term = []
    for coef, amp, facs in terms:
        fv = [prim(kind, t, args) for kind, args in facs]
        prod = np.ones_like(t)
        for v in fv:
            prod = prod * v
        a = a + coef * amp * prod
        per_term.append((coef, amp, facs, fv, prod))
    out.append(E * (1.0 + a))          # dN/dN0
    out.append(np.ones_like(t))        # dN/dNbkg
    for coef, amp, facs, fv, prod in per_term:
        out.append(n0 * E * coef * prod)               # dN/damp
        for i, (kind, args) in enumerate(facs):
            others = np.ones_like(t)
            for j2, v in enumerate(fv):
                if j2 != i:
                    others = others * v
            for dprim in prim_grad(kind, t, args):
                out.append(n0 * E * coef * amp * others * dprim)
    return out


def grad(theory, histos, counts, p, kind="chi2"):
    """Analytic gradient d cost / d p.  Each component is an exactly rounded
    sum over bins and resolved scalars of r_n dN_n/dR * dR/dp."""
    p = np.asarray(p, dtype=np.float64)
    acc = [[] for _ in range(p.size)]
    for h, c in zip(histos, counts):
        res = resolve(theory, p, h["map_row"])
        t = time_grid(h)
        N = model(theory, h, p)
        r = cost_dN(_fit_range(h, c), N, kind)
        for (_, _, jac), dN in zip(res, _dN_dres(theory, t, res)):
            nz = np.nonzero(jac)[0]
            if nz.size == 0:
                continue
            contrib = r * dN
            for k in nz:
                acc[k].append(contrib * jac[k])
    return np.array([math.fsum(np.concatenate(a)) if a else 0.0 for a in acc])


def grad_abs_scale(theory, histos, counts, p, kind="chi2"):
    """sum over bins of |r_n dN_n/dp_k|: the scale against which a computed
    gradient's rounding error is judged near a minimum."""
    p = np.asarray(p, dtype=np.float64)
    acc = np.zeros(p.size)
    for h, c in zip(histos, counts):
        res = resolve(theory, p, h["map_row"])
        t = time_grid(h)
        N = model(theory, h, p)
        r = cost_dN(_fit_range(h, c), N, kind)
        for (_, _, jac), dN in zip(res, _dN_dres(theory, t, res)):
            for k in np.nonzero(jac)[0]:
                acc[k] += float(np.sum(np.abs(r * dN * jac[k])))
    return acc


def grad_fd(theory, histos, counts, p, kind="chi2", rel=1e-4):
    """Central finite differences with one Richardson step (h and h/2),
    h_k = rel * max(|p_k|, 1): an independent check of grad()."""
    p = np.asarray(p, dtype=np.float64)
    g = np.zeros(p.size)
    for k in range(p.size):
        h = rel * max(abs(p[k]), 1.0)

        def cd(hh):
            pp = p.copy()
            pm = p.copy()
            pp[k] += hh
            pm[k] -= hh
            return (cost(theory, histos, counts, pp, kind) - cost(theory, histos, counts, pm, kind)) / (2 * hh)

        g[k] = (4.0 * cd(h / 2) - cd(h)) / 3.0
    return g
