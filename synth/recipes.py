"""Workload recipes: theory programs, grids, parameter draws, Poisson counts.

Conventions (the paper leaves them open; each is a stated reading):

* time grid: bin n of a histogram sits at t_n = (n - t0_bin) * dt, a point at
  the left bin edge (Eq. 1 text: t = n * dt); t in microseconds;
* rates (lambda, sigma) in 1/us, frequencies nu in MHz, phases phi in radians;
* tau_mu = 2.1969811 us (not printed in the paper);
* a theory program is a sum of terms, each ``coef * amp * prod(factors)``,
  each factor one of the predefined primitives of Listing 2 (se, ge, sg, stg)
  or the precession tf(phi, nu) used in Listing 3.  Every scalar argument is a
  *reference*: ``("p", slot)`` reads ``p[map[row][slot]]``, ``("f", slot)``
  reads the function array ``f[map[row][slot]]`` with ``f = F p + f0``, and
  ``("lit", x)`` is the literal x.  This is the parameter / function / map
  indirection the paper describes for its generated user functions.

The dictionaries below are plain data; both sides of every comparison read
them with their own code.
"""

from __future__ import annotations

import math

import numpy as np

TAU_MU = 2.1969811  # muon lifetime in us
SEED_BASE = 160402334


def ref_p(slot):
    return ("p", int(slot))


def ref_f(slot):
    return ("f", int(slot))


def ref_lit(x):
    return ("lit", float(x))


def rng_for(k):
    """The seeded generator of workload k."""
    return np.random.default_rng(SEED_BASE + k)


def _factor(prim, *args):
    return {"prim": prim, "args": list(args)}


def _single_row(n_par):
    return [list(range(n_par))]


# ---------------------------------------------------------------------------
# Theory programs for a single histogram (parameter vector = map row 0)
# ---------------------------------------------------------------------------

def theory_exp_cos():
    """A(t) = A e^(-lambda t) cos(2 pi nu t + phi); p = [N0, Nbkg, A, lambda, nu, phi]."""
    return {
        "tau_mu": TAU_MU,
        "n0": ref_p(0),
        "nbkg": ref_p(1),
        "terms": [{"coef": 1.0, "amp": ref_p(2),
                   "factors": [_factor("se", ref_p(3)), _factor("tf", ref_p(5), ref_p(4))]}],
        "map": _single_row(6),
        "F": None,
        "f0": None,
        "n_par": 6,
        "names": ["N0", "Nbkg", "A", "lambda", "nu", "phi"],
    }


def theory_gauss_cos():
    """Eq. 4 for one detector: A e^(-(sigma t)^2/2) cos(2 pi nu t + phi); p = [N0, Nbkg, A, sigma, nu, phi]."""
    return {
        "tau_mu": TAU_MU,
        "n0": ref_p(0),
        "nbkg": ref_p(1),
        "terms": [{"coef": 1.0, "amp": ref_p(2),
                   "factors": [_factor("sg", ref_p(3)), _factor("tf", ref_p(5), ref_p(4))]}],
        "map": _single_row(6),
        "F": None,
        "f0": None,
        "n_par": 6,
        "names": ["N0", "Nbkg", "A", "sigma", "nu", "phi"],
    }


def theory_stg():
    """Static Gaussian Kubo-Toyabe: A stg(sigma, t); p = [N0, Nbkg, A, sigma]."""
    return {
        "tau_mu": TAU_MU,
        "n0": ref_p(0),
        "nbkg": ref_p(1),
        "terms": [{"coef": 1.0, "amp": ref_p(2), "factors": [_factor("stg", ref_p(3))]}],
        "map": _single_row(4),
        "F": None,
        "f0": None,
        "n_par": 4,
        "names": ["N0", "Nbkg", "A", "sigma"],
    }


def theory_exp_gkt():
    """A1 e^(-lambda t) + A2 stg(sigma, t); p = [N0, Nbkg, A1, lambda, A2, sigma]."""
    return {
        "tau_mu": TAU_MU,
        "n0": ref_p(0),
        "nbkg": ref_p(1),
        "terms": [{"coef": 1.0, "amp": ref_p(2), "factors": [_factor("se", ref_p(3))]},
                  {"coef": 1.0, "amp": ref_p(4), "factors": [_factor("stg", ref_p(5))]}],
        "map": _single_row(6),
        "F": None,
        "f0": None,
        "n_par": 6,
        "names": ["N0", "Nbkg", "A1", "lambda", "A2", "sigma"],
    }


FAMILIES = ("exp_cos", "gauss_cos", "stg", "exp_gkt")
_FAMILY_THEORY = {"exp_cos": theory_exp_cos, "gauss_cos": theory_gauss_cos,
                  "stg": theory_stg, "exp_gkt": theory_exp_gkt}


# ---------------------------------------------------------------------------
# Multi-detector theory programs (one map row per detector)
# ---------------------------------------------------------------------------

def theory_c2(n_det=16, weight=0.3):
    """Shared A, lambda, nu, sigma; per detector N0_j, Nbkg_j, phi_j.

    A^j(t) = A [(1-w) e^(-lambda t) cos(2 pi nu t + phi_j) + w stg(sigma, t)],
    written as two terms with literal coefficients (1-w) and w.
    Parameter layout: [A, lambda, nu, sigma] + [N0_j, Nbkg_j, phi_j] per detector.
    Map row j slots: 0 N0, 1 Nbkg, 2 A, 3 lambda, 4 nu, 5 phi, 6 sigma.
    """
    rows = []
    for j in range(n_det):
        b = 4 + 3 * j
        rows.append([b, b + 1, 0, 1, 2, b + 2, 3])
    names = ["A", "lambda", "nu", "sigma"]
    for j in range(n_det):
        names += [f"N0_{j}", f"Nbkg_{j}", f"phi_{j}"]
    return {
        "tau_mu": TAU_MU,
        "n0": ref_p(0),
        "nbkg": ref_p(1),
        "terms": [{"coef": 1.0 - weight, "amp": ref_p(2),
                   "factors": [_factor("se", ref_p(3)), _factor("tf", ref_p(5), ref_p(4))]},
                  {"coef": weight, "amp": ref_p(2), "factors": [_factor("stg", ref_p(6))]}],
        "map": rows,
        "F": None,
        "f0": None,
        "n_par": 4 + 3 * n_det,
        "names": names,
    }


def config_multi_run():
    """Two runs fitted together (a multi-run fit): run 0 with 2 histograms of
    4000 bins of 0.004 us from t0_bin = 10.5, run 1 with 3 histograms of 6000
    bins of 0.002 us; A(t) = A_r e^(-lambda t) cos(2 pi nu_r t + phi_h) with
    lambda shared by both runs, A_r and nu_r per run and N0_h, Nbkg_h, phi_h
    per histogram.  Parameter layout: [lambda, A_0, nu_0, A_1, nu_1] +
    [N0_h, Nbkg_h, phi_h] per histogram; map row h slots: 0 N0, 1 Nbkg, 2 A,
    3 lambda, 4 nu, 5 phi (the exp*cos program)."""
    rng = rng_for(9)
    runs = [(2, 4000, 0.004, 10.5), (3, 6000, 0.002, 0.0)]
    rows, histos = [], []
    h = 0
    for r, (nh, nb, dt, t0) in enumerate(runs):
        for _ in range(nh):
            b = 5 + 3 * h
            rows.append([b, b + 1, 1 + 2 * r, 0, 2 + 2 * r, b + 2])
            histos.append(_histo(nb, dt, map_row=h, t0_bin=t0, first=int(t0) + 1))
            h += 1
    n_par = 5 + 3 * h
    th = theory_exp_cos()
    th["map"] = rows
    th["n_par"] = n_par
    th["names"] = ["lambda", "A_0", "nu_0", "A_1", "nu_1"] + [f"{x}_{k}" for k in range(h)
                                                              for x in ("N0", "Nbkg", "phi")]
    p = np.zeros(n_par)
    p[:5] = [0.45, 0.22, 1.1, 0.18, 2.3]
    for k in range(h):
        p[5 + 3 * k] = rng.uniform(800.0, 1500.0)
        p[6 + 3 * k] = rng.uniform(1.0, 10.0)
        p[7 + 3 * k] = (k % 2) * math.pi + rng.uniform(-0.2, 0.2)
    return {"name": "multi_run_2x", "theory": th, "histos": histos, "p_true": p, "rng": rng, "seed_k": 9}


def theory_paper_eq4(n_det=16):
    """Eq. 4 over n_det detectors with the precession frequency taken from the
    function array, as in Listing 3: nu = f[0] = (gamma_mu / 2 pi) * B.

    Parameter layout: [sigma, B] + [N0_j, Nbkg_j, A0_j, phi_j] per detector,
    with B in kG and gamma_mu / 2 pi = 13.553879 MHz/kG.
    Map row j slots: 0 N0, 1 Nbkg, 2 A0, 3 sigma, 4 phi, 5 -> f index 0.
    """
    rows = []
    for j in range(n_det):
        b = 2 + 4 * j
        rows.append([b, b + 1, b + 2, 0, b + 3, 0])
    n_par = 2 + 4 * n_det
    F = [[0.0] * n_par]
    F[0][1] = 13.553879
    names = ["sigma", "B"]
    for j in range(n_det):
        names += [f"N0_{j}", f"Nbkg_{j}", f"A0_{j}", f"phi_{j}"]
    return {
        "tau_mu": TAU_MU,
        "n0": ref_p(0),
        "nbkg": ref_p(1),
        "terms": [{"coef": 1.0, "amp": ref_p(2),
                   "factors": [_factor("sg", ref_p(3)), _factor("tf", ref_p(4), ref_f(5))]}],
        "map": rows,
        "F": F,
        "f0": [0.0],
        "n_par": n_par,
        "names": names,
    }


# ---------------------------------------------------------------------------
# Configurations
# ---------------------------------------------------------------------------

def _histo(n_bins, dt, map_row=0, t0_bin=0.0, first=0, last=None):
    return {"n_bins": int(n_bins), "dt": float(dt), "t0_bin": float(t0_bin),
            "first": int(first), "last": int(n_bins - 1 if last is None else last),
            "map_row": int(map_row)}


def config_c1():
    """One histogram, 8192 bins of 0.001 us, exp*cos truth (N0 1000, A 0.25,
    lambda 0.5, nu 1.355, phi 0, Nbkg 5)."""
    p = np.array([1000.0, 5.0, 0.25, 0.5, 1.355, 0.0])
    return {"name": "c1_single_8192", "theory": theory_exp_cos(),
            "histos": [_histo(8192, 0.001)], "p_true": p, "seed_k": 1}


def config_c2(n_bins=65536, dt=0.0002, n_det=16, seed_k=2, name="c2_16x65536"):
    """16 detectors x 65536 bins of 0.0002 us, theory_c2 with A 0.25,
    lambda 0.5, nu 1.355, sigma 0.3, w 0.3, N0_j ~ U[500,2000],
    Nbkg_j ~ U[1,10], phi_j = 2 pi j / 16."""
    th = theory_c2(n_det)
    rng = rng_for(seed_k)
    p = np.zeros(th["n_par"])
    p[0:4] = [0.25, 0.5, 1.355, 0.3]
    n0 = rng.uniform(500.0, 2000.0, n_det)
    nb = rng.uniform(1.0, 10.0, n_det)
    for j in range(n_det):
        p[4 + 3 * j] = n0[j]
        p[5 + 3 * j] = nb[j]
        p[6 + 3 * j] = 2.0 * math.pi * j / n_det
    histos = [_histo(n_bins, dt, map_row=j) for j in range(n_det)]
    return {"name": name, "theory": th, "histos": histos, "p_true": p,
            "seed_k": seed_k, "rng": rng}


def config_c2_large():
    """The 16-detector theory of config_c2 over 16 x 2^23 bins spanning the
    same 13.1072 us window: 537 MB of FP32 counts, larger than the MALL."""
    n = 1 << 23
    return config_c2(n_bins=n, dt=13.1072 / n, seed_k=22, name="c2_16x8388608")


def config_c3(n_vec=4096, rel=1e-4):
    """n_vec parameter vectors around the C1 truth: p (1 + u), u ~ U[-rel, rel];
    phi (zero at truth) gets an absolute +-rel offset."""
    c1 = config_c1()
    rng = rng_for(3)
    p0 = c1["p_true"]
    u = rng.uniform(-rel, rel, size=(n_vec, p0.size))
    P = p0[None, :] * (1.0 + u)
    P[:, 5] = p0[5] + u[:, 5]
    c1 = dict(c1)
    c1.update({"name": f"c3_{n_vec}vec_on_c1", "P": P})
    return c1


def _loguniform(rng, lo, hi, size=None):
    return np.exp(rng.uniform(math.log(lo), math.log(hi), size))


def _family_truth(rng, fam):
    n0 = _loguniform(rng, 100.0, 1e5)
    nbkg = rng.uniform(1.0, 10.0)
    if fam == "exp_cos":
        return np.array([n0, nbkg, rng.uniform(0.05, 0.3), _loguniform(rng, 0.05, 5.0),
                         _loguniform(rng, 0.1, 50.0), rng.uniform(0.0, 2 * math.pi)])
    if fam == "gauss_cos":
        return np.array([n0, nbkg, rng.uniform(0.05, 0.3), _loguniform(rng, 0.05, 1.0),
                         _loguniform(rng, 0.1, 50.0), rng.uniform(0.0, 2 * math.pi)])
    if fam == "stg":
        return np.array([n0, nbkg, rng.uniform(0.05, 0.3), _loguniform(rng, 0.05, 1.0)])
    if fam == "exp_gkt":
        return np.array([n0, nbkg, rng.uniform(0.05, 0.3), _loguniform(rng, 0.05, 5.0),
                         rng.uniform(0.05, 0.3), _loguniform(rng, 0.05, 1.0)])
    raise ValueError(fam)


_PHASE_SLOT = {"exp_cos": 5, "gauss_cos": 5, "stg": None, "exp_gkt": None}


def config_c4(n_sets=512, window_us=10.0, lo_exp=12, hi_exp=20):
    """n_sets independent single-histogram datasets: n_b = round(2^U[lo,hi]),
    dt = window / n_b, family uniform over the four, parameters drawn from the
    seeder ranges; start = truth (1 + U[-0.05, 0.05]), phase + U[-0.05, 0.05]."""
    rng = rng_for(4)
    sets = []
    for i in range(n_sets):
        n_b = int(round(2.0 ** rng.uniform(lo_exp, hi_exp)))
        fam = FAMILIES[int(rng.integers(0, 4))]
        p = _family_truth(rng, fam)
        start = p * (1.0 + rng.uniform(-0.05, 0.05, p.size))
        ps = _PHASE_SLOT[fam]
        if ps is not None:
            start[ps] = p[ps] + rng.uniform(-0.05, 0.05)
        sets.append({"family": fam, "theory": _FAMILY_THEORY[fam](),
                     "histos": [_histo(n_b, window_us / n_b)], "p_true": p, "start": start})
    return {"name": f"c4_{n_sets}sets", "sets": sets, "rng": rng, "seed_k": 4}


def config_c5_ranges():
    """Parameter ranges of the seeder's exp*cos family and its grid
    (8192 bins of 0.001 us, rebinned by 8 to 1024)."""
    return {"n_bins": 8192, "dt": 0.001, "rebin": 8,
            "N0": (100.0, 1e5), "Nbkg": (1.0, 10.0), "A": (0.05, 0.3),
            "lambda": (0.05, 5.0), "nu": (0.1, 50.0), "phi": (0.0, 2 * math.pi)}


def config_paper_shape(n_bins=85320, window_us=10.0, n_det=16):
    """Eq. 4 over 16 detectors at one of the Table 1 sizes (85,320 ...
    426,601 bins); the window is not stated in the paper (10 us assumed)."""
    th = theory_paper_eq4(n_det)
    rng = rng_for(7)
    p = np.zeros(th["n_par"])
    p[0] = 0.35
    p[1] = 1.0
    for j in range(n_det):
        b = 2 + 4 * j
        p[b] = rng.uniform(500.0, 2000.0)
        p[b + 1] = rng.uniform(1.0, 10.0)
        p[b + 2] = rng.uniform(0.2, 0.3)
        p[b + 3] = 2.0 * math.pi * j / n_det
    histos = [_histo(n_bins, window_us / n_bins, map_row=j) for j in range(n_det)]
    return {"name": f"paper_eq4_16x{n_bins}", "theory": th, "histos": histos,
            "p_true": p, "rng": rng, "seed_k": 7}


# ---------------------------------------------------------------------------
# Counts
# ---------------------------------------------------------------------------

def draw_counts(means, rng):
    """One Poisson draw per bin, as float64 integers."""
    m = np.asarray(means, dtype=np.float64)
    if np.any(~np.isfinite(m)) or np.any(m < 0):
        raise ValueError("expected counts must be finite and non-negative")
    return rng.poisson(m).astype(np.float64)


def materialise(theory, histos, p, mean_fn, rng, noiseless=False):
    """Counts for each histogram: Poisson(mean_fn(theory, histo, p)) over the
    whole histogram, or the means themselves when noiseless."""
    out = []
    for h in histos:
        m = np.asarray(mean_fn(theory, h, p), dtype=np.float64)
        if m.shape != (h["n_bins"],):
            raise ValueError("mean_fn must return one value per bin")
        out.append(m.copy() if noiseless else draw_counts(m, rng))
    return out
