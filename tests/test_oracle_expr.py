"""Pins of the oracle's expression theories (oracle/expr.py), the language of
run-time compiled user functions (Sec. 4.2.1, Listing 3):

* an expression that restates a theory program (Listings 2-3) gives the
  program's model values (pinned in test_oracle_primitives / _cost) to a few
  ulps, and the program's analytic gradient;
* for expressions outside the program form (division, sqrt, log, pow, sin,
  function-array references) the symbolic gradient matches Richardson central
  differences of the oracle's own cost;
* syntax errors are refused.
"""

import numpy as np
import pytest

import synth
from oracle import expr, model

from _workloads import counts_for

TAU = synth.TAU_MU


def _h(n=1500, dt=0.004, row=0):
    return {"n_bins": n, "dt": dt, "t0_bin": 0.0, "first": 3, "last": n - 5, "map_row": row}


PROGRAMS = [
    (synth.theory_exp_cos, "p[2]*se(p[3])*tf(p[5],p[4])", [900.0, 3.0, 0.2, 0.8, 1.7, 0.3]),
    (synth.theory_gauss_cos, "p[2]*sg(p[3])*tf(p[5],p[4])", [900.0, 3.0, 0.2, 0.4, 1.7, 0.3]),
    (synth.theory_stg, "p[2]*stg(p[3])", [900.0, 3.0, 0.2, 0.45]),
    (synth.theory_exp_gkt, "p[2]*se(p[3]) + p[4]*stg(p[5])", [900.0, 3.0, 0.15, 0.8, 0.12, 0.4]),
]


def _as_expr(th, e):
    return expr.theory_desc(e, th["tau_mu"], th["n0"], th["nbkg"], th["map"], th["n_par"], th.get("F"), th.get("f0"))


@pytest.mark.parametrize("make,e,p", PROGRAMS)
def test_expression_restating_a_program_matches_it(make, e, p):
    th = make()
    ex = _as_expr(th, e)
    p = np.array(p)
    h = [_h()]
    np.testing.assert_allclose(expr.model_expr(ex, h[0], p), model.model(th, h[0], p), rtol=4e-15, atol=0)
    c = counts_for(th, h, p, np.random.default_rng(3))
    q = p * 1.01
    for kind in ("chi2", "poisson"):
        g = expr.grad_expr(ex, h, c, q, kind)
        ref = model.grad(th, h, c, q, kind)
        scale = model.grad_abs_scale(th, h, c, q, kind)
        assert np.all(np.abs(g - ref) <= 1e-12 * scale), kind
        np.testing.assert_allclose(expr.grad_abs_scale_expr(ex, h, c, q, kind), scale, rtol=1e-12)


def test_symbolic_gradient_against_finite_differences():
    # A = p2 (1 + t)^(-p3) cos(2 pi p4 t + p5) + sqrt(p6) log(1 + p7 t) / (1 + t) + sin(f0 t) p8 ^ 2
    e = "p[2]*pow(1+t, -p[3])*cos(2*pi*p[4]*t + p[5]) + sqrt(p[6])*log(1 + p[7]*t)/(1+t) - 0.01*sin(f[0]*t)*p[8]^2"
    F = np.zeros((1, 9))
    F[0, 4] = 2.0
    ex = expr.theory_desc(e, TAU, ("p", 0), ("p", 1), [list(range(9))], 9, F.tolist(), [0.1])
    p = np.array([900.0, 3.0, 0.2, 0.7, 1.3, 0.4, 0.01, 0.5, 0.3])
    h = [_h(900, 0.008)]
    rng = np.random.default_rng(5)
    c = [rng.poisson(expr.model_expr_full(ex, h[0], p)).astype(float)]
    q = p * (1.0 + 0.02 * np.cos(np.arange(9)))
    for kind in ("chi2", "poisson"):
        g = expr.grad_expr(ex, h, c, q, kind)
        fd = np.zeros(9)
        for k in range(9):
            hk = 1e-4 * max(abs(q[k]), 1e-2)

            def cd(s):
                a, b = q.copy(), q.copy()
                a[k] += s
                b[k] -= s
                return (expr.cost_expr(ex, h, c, a, kind) - expr.cost_expr(ex, h, c, b, kind)) / (2 * s)

            fd[k] = (4 * cd(hk / 2) - cd(hk)) / 3
        assert np.all(np.abs(g - fd) <= 1e-7 * np.abs(fd) + 1e-9 * np.max(np.abs(fd))), (kind, g, fd)


@pytest.mark.parametrize("bad", ["p[2]*", "p[2]*se(p[3]", "q[1]", "se(p[1], p[2])", "p[1.5]", "2 p[1]", "tf(p[1])",
                                 "p[-1]", ""])
def test_syntax_errors(bad):
    with pytest.raises(ValueError):
        expr.parse(bad)
