"""User-defined asymmetry expressions (test infrastructure only).

The paper lets a user write the theory as code that is compiled at run time
(Sec. 4.2.1, Listing 3: a generated function returns, e.g.,
p[m[0]] * se(t, p[m[1]]) * tf(t, p[m[2]], f[m[3]])).  This oracle reads the
same expression language as the library and evaluates it with numpy; its
derivatives come from symbolic differentiation of the parsed tree (not from
the library's dual numbers).

Grammar (whitespace ignored):
    expr    := term (("+" | "-") term)*
    term    := unary (("*" | "/") unary)*
    unary   := ("-" | "+") unary | power
    power   := primary ("^" unary)?
    primary := number | "t" | "pi" | "p" "[" int "]" | "f" "[" int "]"
             | name "(" expr ("," expr)* ")" | "(" expr ")"
names: exp, log, sqrt, sin, cos, pow(a, b), j0 (Bessel function of the first
kind, order 0), the primitives se(lambda), ge(lambda, beta), sg(sigma),
stg(sigma), tf(phi, nu) of Listing 2 / 3, and further relaxation and
precession functions of muSR practice (the paper refers to a full list of
predefined functions without printing it; these are the standard closed
forms): sekt(a) = 1/3 + 2/3 (1 - a t) e^(-a t) (static Lorentzian
Kubo-Toyabe), ab(sigma, gamma) = exp(-(sigma/gamma)^2 (e^(-gamma t) - 1 +
gamma t)) (Abragam), b(phi, nu) = J0(2 pi nu t + phi) (Bessel precession),
ifld(alpha, phi, nu, lT, lL) = alpha cos(2 pi nu t + phi) e^(-lT t) +
(1 - alpha) e^(-lL t) (internal field) and ibsl(...) the same with J0 in
place of cos.  t is implicit in every primitive.  p[i] is the parameter at slot i of the histogram's map
row, f[i] the function value at slot i (f = F p + f0).
"""

from __future__ import annotations

import math
import re

import numpy as np
from scipy import special

from . import model

FUNCS = {"exp": 1, "log": 1, "sqrt": 1, "sin": 1, "cos": 1, "pow": 2, "j0": 1,
         "se": 1, "ge": 2, "sg": 1, "stg": 1, "tf": 2,
         "sekt": 1, "ab": 2, "b": 2, "ifld": 5, "ibsl": 5}
_TOK = re.compile(r"\s*(?:(\d+\.\d*(?:[eE][+-]?\d+)?|\.\d+(?:[eE][+-]?\d+)?|\d+(?:[eE][+-]?\d+)?)|([A-Za-z_]\w*)|(.))")


def _tokens(s):
    out = []
    pos = 0
    s = s.rstrip()
    while pos < len(s):
        m = _TOK.match(s, pos)
        if not m:
            raise ValueError(f"bad character at {pos}")
        num, name, op = m.groups()
        if num is not None:
            out.append(("num", float(num)))
        elif name is not None:
            out.append(("name", name))
        else:
            out.append(("op", op))
        pos = m.end()
    out.append(("end", None))
    return out


class _Parser:
    def __init__(self, s):
        self.t = _tokens(s)
        self.i = 0

    def peek(self):
        return self.t[self.i]

    def take(self, kind=None, val=None):
        tok = self.t[self.i]
        if (kind and tok[0] != kind) or (val is not None and tok[1] != val):
            raise ValueError(f"expected {val or kind}, found {tok[1]!r}")
        self.i += 1
        return tok

    def expr(self):
        node = self.term()
        while self.peek() in (("op", "+"), ("op", "-")):
            op = self.take()[1]
            node = (op, node, self.term())
        return node

    def term(self):
        node = self.unary()
        while self.peek() in (("op", "*"), ("op", "/")):
            op = self.take()[1]
            node = (op, node, self.unary())
        return node

    def unary(self):
        if self.peek() == ("op", "-"):
            self.take()
            return ("neg", self.unary())
        if self.peek() == ("op", "+"):
            self.take()
            return self.unary()
        return self.power()

    def power(self):
        base = self.primary()
        if self.peek() == ("op", "^"):
            self.take()
            return ("pow", base, self.unary())
        return base

    def primary(self):
        kind, v = self.peek()
        if kind == "num":
            self.take()
            return ("num", v)
        if kind == "op" and v == "(":
            self.take()
            node = self.expr()
            self.take("op", ")")
            return node
        if kind == "name":
            self.take()
            if v == "t":
                return ("t",)
            if v == "pi":
                return ("num", math.pi)
            if v in ("p", "f") and self.peek() == ("op", "["):
                self.take()
                k, idx = self.take("num")
                if idx != int(idx) or idx < 0:
                    raise ValueError("slot index must be a non-negative integer")
                self.take("op", "]")
                return ("ref", v, int(idx))
            if v in FUNCS:
                self.take("op", "(")
                args = [self.expr()]
                while self.peek() == ("op", ","):
                    self.take()
                    args.append(self.expr())
                self.take("op", ")")
                if len(args) != FUNCS[v]:
                    raise ValueError(f"{v} takes {FUNCS[v]} argument(s)")
                return ("call", v, args)
            raise ValueError(f"unknown name {v!r}")
        raise ValueError(f"unexpected {v!r}")


def parse(s):
    """The expression tree of s (ValueError on a syntax error)."""
    p = _Parser(s)
    node = p.expr()
    if p.peek()[0] != "end":
        raise ValueError(f"unexpected {p.peek()[1]!r} after the expression")
    return node


def refs(node, out=None):
    """The (kind, slot) references of the tree, in first-appearance order."""
    out = [] if out is None else out
    if node[0] == "ref":
        if (node[1], node[2]) not in out:
            out.append((node[1], node[2]))
    elif node[0] in ("+", "-", "*", "/", "pow"):
        refs(node[1], out)
        refs(node[2], out)
    elif node[0] == "neg":
        refs(node[1], out)
    elif node[0] == "call":
        for a in node[2]:
            refs(a, out)
    return out


def evaluate(node, t, val):
    """Value of the tree on the time array t; val maps (kind, slot) to a number."""
    k = node[0]
    if k == "num":
        return np.full_like(t, node[1])
    if k == "t":
        return t
    if k == "ref":
        return np.full_like(t, val[(node[1], node[2])])
    if k == "neg":
        return -evaluate(node[1], t, val)
    if k in ("+", "-", "*", "/"):
        a, b = evaluate(node[1], t, val), evaluate(node[2], t, val)
        return {"+": a + b, "-": a - b, "*": a * b, "/": a / b}[k]
    if k == "pow":
        return np.power(evaluate(node[1], t, val), evaluate(node[2], t, val))
    name, args = node[1], [evaluate(a, t, val) for a in node[2]]
    if name in ("exp", "log", "sqrt", "sin", "cos"):
        return getattr(np, name)(args[0])
    if name in ("j0", "j1"):
        return getattr(special, name)(args[0])
    if name == "pow":
        return np.power(args[0], args[1])
    # the primitives of Listing 2 / 3, with t implicit
    return _prim_array(name, t, args)


def _prim_array(name, t, args):
    if name == "se":
        return np.exp(-args[0] * t)
    if name == "ge":
        return np.exp(-np.power(args[0] * t, args[1]))
    if name == "sg":
        return np.exp(-0.5 * (args[0] * t) ** 2)
    if name == "stg":
        s2 = (args[0] * t) ** 2
        return 1.0 / 3.0 + (2.0 / 3.0) * (1.0 - s2) * np.exp(-0.5 * s2)
    if name == "tf":
        return np.cos(2.0 * np.pi * args[1] * t + args[0])
    if name == "sekt":
        x = args[0] * t
        return 1.0 / 3.0 + (2.0 / 3.0) * (1.0 - x) * np.exp(-x)
    if name == "ab":
        s, g = args
        return np.exp(-(s / g) ** 2 * (np.exp(-g * t) - 1.0 + g * t))
    if name == "b":
        return special.j0(2.0 * np.pi * args[1] * t + args[0])
    if name in ("ifld", "ibsl"):
        al, phi, nu, lt, ll = args
        x = 2.0 * np.pi * nu * t + phi
        osc = np.cos(x) if name == "ifld" else special.j0(x)
        return al * osc * np.exp(-lt * t) + (1.0 - al) * np.exp(-ll * t)
    raise ValueError(name)


def _expand(node):
    """The primitives written out in terms of exp, cos, pow and t, so that the
    derivative rules below cover them."""
    k = node[0]
    if k in ("+", "-", "*", "/", "pow"):
        return (k, _expand(node[1]), _expand(node[2]))
    if k == "neg":
        return ("neg", _expand(node[1]))
    if k != "call":
        return node
    name, args = node[1], [_expand(a) for a in node[2]]
    t = ("t",)
    if name == "se":
        return ("call", "exp", [("neg", ("*", args[0], t))])
    if name == "ge":
        return ("call", "exp", [("neg", ("pow", ("*", args[0], t), args[1]))])
    if name == "sg":
        x = ("*", args[0], t)
        return ("call", "exp", [("*", ("num", -0.5), ("*", x, x))])
    if name == "stg":
        x = ("*", args[0], t)
        s2 = ("*", x, x)
        return ("+", ("/", ("num", 1.0), ("num", 3.0)),
                ("*", ("/", ("num", 2.0), ("num", 3.0)),
                 ("*", ("-", ("num", 1.0), s2), ("call", "exp", [("*", ("num", -0.5), s2)]))))
    if name == "tf":
        return ("call", "cos", [("+", ("*", ("*", ("*", ("num", 2.0), ("num", math.pi)), args[1]), t), args[0])])
    one = ("num", 1.0)
    if name == "sekt":
        x = ("*", args[0], t)
        return ("+", ("/", one, ("num", 3.0)),
                ("*", ("/", ("num", 2.0), ("num", 3.0)), ("*", ("-", one, x), ("call", "exp", [("neg", x)]))))
    if name == "ab":
        s, g = args
        r = ("/", s, g)
        gt = ("*", g, t)
        return ("call", "exp", [("neg", ("*", ("*", r, r), ("+", ("-", ("call", "exp", [("neg", gt)]), one), gt)))])
    phase = lambda phi, nu: ("+", ("*", ("*", ("*", ("num", 2.0), ("num", math.pi)), nu), t), phi)
    if name == "b":
        return ("call", "j0", [phase(args[0], args[1])])
    if name in ("ifld", "ibsl"):
        al, phi, nu, lt, ll = args
        osc = ("call", "cos" if name == "ifld" else "j0", [phase(phi, nu)])
        return ("+", ("*", ("*", al, osc), ("call", "exp", [("neg", ("*", lt, t))])),
                ("*", ("-", one, al), ("call", "exp", [("neg", ("*", ll, t))])))
    return ("call", name, args)


def derivative(node, var):
    """Symbolic d node / d var (var = (kind, slot)) of an expanded tree."""
    k = node[0]
    zero = ("num", 0.0)
    if k in ("num", "t"):
        return zero
    if k == "ref":
        return ("num", 1.0) if (node[1], node[2]) == var else zero
    if k == "neg":
        return ("neg", derivative(node[1], var))
    a = node[1] if k != "call" else None
    if k in ("+", "-"):
        return (k, derivative(node[1], var), derivative(node[2], var))
    if k == "*":
        return ("+", ("*", derivative(node[1], var), node[2]), ("*", node[1], derivative(node[2], var)))
    if k == "/":
        u, v = node[1], node[2]
        return ("/", ("-", ("*", derivative(u, var), v), ("*", u, derivative(v, var))), ("*", v, v))
    if k == "pow":
        u, v = node[1], node[2]
        # d(u^v) = u^v (v' ln u + v u' / u), written for u > 0; v constant: v u^(v-1) u'
        return ("+", ("*", ("*", v, ("pow", u, ("-", v, ("num", 1.0)))), derivative(u, var)),
                ("*", ("*", ("pow", u, v), ("call", "log", [u])), derivative(v, var)))
    name, args = node[1], node[2]
    u = args[0]
    du = derivative(u, var)
    if name == "exp":
        return ("*", node, du)
    if name == "log":
        return ("/", du, u)
    if name == "sqrt":
        return ("/", du, ("*", ("num", 2.0), node))
    if name == "sin":
        return ("*", ("call", "cos", [u]), du)
    if name == "cos":
        return ("neg", ("*", ("call", "sin", [u]), du))
    if name == "j0":
        return ("neg", ("*", ("call", "j1", [u]), du))
    if name == "pow":
        return derivative(("pow", args[0], args[1]), var)
    raise ValueError(name)


def _eval_safe(node, t, val):
    """evaluate() with 0 * (anything non-finite) taken as 0 (a derivative term
    whose factor vanishes, e.g. ln(lambda t) at t = 0 times 0)."""
    k = node[0]
    if k == "*":
        a, b = _eval_safe(node[1], t, val), _eval_safe(node[2], t, val)
        with np.errstate(invalid="ignore"):
            out = a * b
        return np.where((a == 0) | (b == 0), 0.0, out)
    if k in ("+", "-", "/", "pow"):
        a, b = _eval_safe(node[1], t, val), _eval_safe(node[2], t, val)
        with np.errstate(divide="ignore", invalid="ignore"):
            return {"+": a + b, "-": a - b, "/": a / b, "pow": np.power(a, b)}[k]
    if k == "neg":
        return -_eval_safe(node[1], t, val)
    if k == "call":
        args = [_eval_safe(a, t, val) for a in node[2]]
        with np.errstate(divide="ignore", invalid="ignore"):
            if node[1] == "pow":
                return np.power(args[0], args[1])
            if node[1] in ("j0", "j1"):
                return getattr(special, node[1])(args[0])
            return getattr(np, node[1])(args[0])
    return evaluate(node, t, val)


def theory_desc(expr, tau_mu, n0, nbkg, map_rows, n_par, F=None, f0=None):
    """A theory of this language as plain data (the library's and the
    oracle's common input)."""
    return {"expr": expr, "tau_mu": tau_mu, "n0": n0, "nbkg": nbkg, "map": map_rows, "n_par": n_par,
            "F": F, "f0": f0}


def _values(theory, p, row):
    p = np.asarray(p, dtype=np.float64)
    f = model.function_array(theory, p)
    out = {}
    for kind, slot in refs(parse(theory["expr"])):
        i = theory["map"][row][slot]
        out[(kind, slot)] = float(p[i]) if kind == "p" else float(f[i])
    return out


def _scalar(theory, ref, p, f, row):
    v, jac = model._ref_value_and_jac(theory, ref, p, f, row)
    return v, jac


def model_expr(theory, h, p):
    """N(t_n) = N0 e^(-t/tau) (1 + A(t)) + Nbkg over the fit range of h (Eq. 1)."""
    p = np.asarray(p, dtype=np.float64)
    f = model.function_array(theory, p)
    row = h["map_row"]
    n0, _ = _scalar(theory, theory["n0"], p, f, row)
    nbkg, _ = _scalar(theory, theory["nbkg"], p, f, row)
    t = model.time_grid(h)
    a = evaluate(parse(theory["expr"]), t, _values(theory, p, row))
    return n0 * np.exp(-t / theory["tau_mu"]) * (1.0 + a) + nbkg


def model_expr_full(theory, h, p):
    hh = dict(h)
    hh["first"], hh["last"] = 0, h["n_bins"] - 1
    return model_expr(theory, hh, p)


def cost_expr(theory, histos, counts, p, kind="chi2"):
    """Exactly rounded total cost (Eqs. 2-3)."""
    terms = []
    for h, c in zip(histos, counts):
        N = model_expr(theory, h, p)
        terms.append(model.cost_terms(np.asarray(c, dtype=np.float64)[h["first"]:h["last"] + 1], N, kind))
    return math.fsum(np.concatenate(terms))


def _dN_dp(theory, h, p):
    """dN_n/dp_k over the fit range: [bins][n_par], from the symbolic derivatives."""
    p = np.asarray(p, dtype=np.float64)
    f = model.function_array(theory, p)
    row = h["map_row"]
    n0, jn0 = _scalar(theory, theory["n0"], p, f, row)
    nbkg, jbg = _scalar(theory, theory["nbkg"], p, f, row)
    t = model.time_grid(h)
    tree = parse(theory["expr"])
    val = _values(theory, p, row)
    a = evaluate(tree, t, val)
    E = np.exp(-t / theory["tau_mu"])
    J = np.outer(E * (1.0 + a), jn0) + np.outer(np.ones_like(t), jbg)
    ex = _expand(tree)
    for kind, slot in refs(tree):
        dA = _eval_safe(derivative(ex, (kind, slot)), t, val)
        _, jr = _scalar(theory, (kind, slot), p, f, row)
        J += np.outer(n0 * E * dA, jr)
    return J


def grad_expr(theory, histos, counts, p, kind="chi2"):
    """d cost / d p, each component an exactly rounded sum over bins."""
    p = np.asarray(p, dtype=np.float64)
    parts = [[] for _ in range(p.size)]
    for h, c in zip(histos, counts):
        N = model_expr(theory, h, p)
        r = model.cost_dN(np.asarray(c, dtype=np.float64)[h["first"]:h["last"] + 1], N, kind)
        J = _dN_dp(theory, h, p)
        for k in range(p.size):
            if np.any(J[:, k]):
                parts[k].append(r * J[:, k])
    return np.array([math.fsum(np.concatenate(x)) if x else 0.0 for x in parts])


def grad_abs_scale_expr(theory, histos, counts, p, kind="chi2"):
    """sum_n |r_n dN_n/dp_k| (the scale of a gradient's rounding error)."""
    p = np.asarray(p, dtype=np.float64)
    acc = np.zeros(p.size)
    for h, c in zip(histos, counts):
        N = model_expr(theory, h, p)
        r = model.cost_dN(np.asarray(c, dtype=np.float64)[h["first"]:h["last"] + 1], N, kind)
        acc += np.sum(np.abs(r[:, None] * _dN_dp(theory, h, p)), axis=0)
    return acc
