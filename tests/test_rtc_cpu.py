"""Run-time compiled theories without a GPU: the library parses and checks
user expressions (the paper's user functions, Sec. 4.2.1 / Listing 3),
generates their kernel source and compiles it with hipRTC for gfx950."""

import synth
from oracle import expr
from paper_1604_02334_amd import _abi as A
from paper_1604_02334_amd import api


def _th(e, n_par=6, F=None, f0=None, rows=None):
    return expr.theory_desc(e, synth.TAU_MU, ("p", 0), ("p", 1), rows or [list(range(n_par))], n_par, F, f0)


GOOD = [
    "p[2]*se(p[3])*tf(p[5],p[4])",
    "p[2]*ge(p[3], p[4])*cos(2*pi*p[5]*t)",
    "p[2]*pow(1+t, -p[3])/(1 + p[4]*t^2) + sqrt(p[5])*log(1+t)*sin(t)",
    "-p[2]*(stg(p[3]) - sg(p[4])) + exp(-p[5]*t)",
    "0.5e-1 * f[0] * tf(p[5], f[0])",
]


def test_expressions_parse_and_compile_for_gfx950():
    F = [[0, 0, 0, 0, 2.0, 0]]
    for e in GOOD:
        th = _th(e, F=F, f0=[0.1])
        st, msg = api.theory_check_expr(th)
        assert st == A.MU_OK, (e, msg)
        src = api.theory_expr_source(th)
        assert "mu_rtc_kernel" in src and "@K@" not in src and "@EXPR@" not in src
        st, log = api.theory_compile_check(th)
        assert st == A.MU_OK, (e, log)
        assert "gfx950" in log


def test_expression_errors_are_refused_with_their_place():
    cases = [("p[2]*", "offset"), ("p[2]*se(p[3]", "expected"), ("foo(p[1])", "unknown name"),
             ("se(p[1], p[2])", "argument"), ("p[9]", "slot 9"), ("f[0]", "map"), ("p[1] p[2]", "offset"),
             ("", "offset")]
    for e, word in cases:
        st, msg = api.theory_check_expr(_th(e))
        assert st == A.MU_E_ARG and word in msg, (e, st, msg)
    many = " + ".join(f"p[{i}]" for i in range(29))
    st, msg = api.theory_check_expr(_th(many, n_par=29))
    assert st == A.MU_E_UNSUPPORTED and "28" in msg
    # bounded parser and emitter: deep nesting, huge operation counts and
    # overlong text are refused, not followed into the stack
    for e, word in (("(" * 5000 + "p[1]" + ")" * 5000, "nesting"), ("-" * 5000 + "p[1]", "nesting"),
                    (" + ".join(["p[1]"] * 5000), "operations"), ("p[1]" + " " * 70000, "longer")):
        st, msg = api.theory_check_expr(_th(e))
        assert st == A.MU_E_ARG and word in msg, (e[:20], st, msg)
    st, _ = api.theory_check_expr(_th("(" * 150 + "p[1]" + ")" * 150))
    assert st == A.MU_OK
