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


def test_further_primitives_closed_forms():
    """sekt: 1 at t = 0, the 1/3 tail, its minimum 1/3 - (2/3) e^-2 at a t = 2;
    ab: the Gaussian exp(-(sigma t)^2 / 2) as gamma -> 0 and the motional
    narrowing exp(-sigma^2 t / gamma) as gamma -> infinity; b: J0's first zero
    and b(phi, 0) = J0(phi); ifld / ibsl: alpha = 1 and alpha = 0 reduce to
    the single terms."""
    t = np.array([0.0, 2.0, 1e3])
    ev = lambda e, v=None: expr.evaluate(expr.parse(e), t, v or {})
    np.testing.assert_allclose(ev("sekt(1.0)"), [1.0, 1.0 / 3.0 - (2.0 / 3.0) * np.exp(-2.0), 1.0 / 3.0],
                               rtol=1e-15)
    d = expr._expand(expr.parse("sekt(p[0])"))
    dd = expr._eval_safe(expr.derivative(d, ("p", 0)), np.array([2.0]), {("p", 0): 1.0})
    assert abs(dd[0]) < 1e-15  # stationary at a t = 2
    tt = np.linspace(0, 3, 31)
    # small gamma: the exponent's series sigma^2 (t^2/2 - g t^3/6 + g^2 t^4/24 - g^3 t^5/120 + ...),
    # whose leading term is the Gaussian
    g = 1e-2
    a = expr.evaluate(expr.parse(f"ab(0.7, {g})"), tt, {})
    ser = 0.49 * (tt ** 2 / 2 - g * tt ** 3 / 6 + g ** 2 * tt ** 4 / 24 - g ** 3 * tt ** 5 / 120)
    np.testing.assert_allclose(a, np.exp(-ser), rtol=1e-8)
    # large gamma (gamma t >= 1e3 here, e^(-gamma t) negligible): exp(-sigma^2 t / gamma + sigma^2 / gamma^2)
    a = expr.evaluate(expr.parse("ab(0.7, 1e4)"), tt[1:], {})
    np.testing.assert_allclose(a, np.exp(-0.49 * tt[1:] / 1e4 + 0.49 / 1e8), rtol=1e-12)
    z = 2.404825557695773
    assert abs(expr.evaluate(expr.parse(f"b({z}, 0)"), np.array([1.0]), {})[0]) < 1e-15
    assert abs(expr.evaluate(expr.parse("b(0.5, 0)"), np.array([1.0]), {})[0] - 0.938469807240813) < 1e-14
    f1 = expr.evaluate(expr.parse("ifld(1, 0.3, 1.2, 0.4, 2.0)"), tt, {})
    np.testing.assert_allclose(f1, np.cos(2 * np.pi * 1.2 * tt + 0.3) * np.exp(-0.4 * tt), rtol=1e-14)
    f0 = expr.evaluate(expr.parse("ibsl(0, 0.3, 1.2, 0.4, 2.0)"), tt, {})
    np.testing.assert_allclose(f0, np.exp(-2.0 * tt), rtol=1e-14)


def test_further_primitives_gradient_against_finite_differences():
    e = "p[2]*sekt(p[3]) + p[4]*ab(p[5], p[6]) + 0.1*b(p[7], p[8]) + 0.05*ifld(p[9], p[7], p[8], p[3], p[6])" \
        " - 0.02*ibsl(p[9], p[7], p[8], p[5], p[3])"
    n = 10
    ex = expr.theory_desc(e, TAU, ("p", 0), ("p", 1), [list(range(n))], n)
    p = np.array([900.0, 3.0, 0.15, 0.6, 0.1, 0.5, 1.5, 0.3, 0.8, 0.6])
    h = [_h(800, 0.01)]
    c = [np.random.default_rng(6).poisson(expr.model_expr_full(ex, h[0], p)).astype(float)]
    q = p * (1.0 + 0.02 * np.sin(np.arange(n)))
    g = expr.grad_expr(ex, h, c, q)
    for k in range(n):
        hk = 1e-4 * max(abs(q[k]), 1e-2)

        def cd(s):
            a, b = q.copy(), q.copy()
            a[k] += s
            b[k] -= s
            return (expr.cost_expr(ex, h, c, a) - expr.cost_expr(ex, h, c, b)) / (2 * s)

        fd = (4 * cd(hk / 2) - cd(hk)) / 3
        assert abs(g[k] - fd) <= 1e-7 * abs(fd) + 1e-9 * np.max(np.abs(g)), (k, g[k], fd)
