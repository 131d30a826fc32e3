"""Run-time compiled theories (hipRTC; the paper's user functions, Sec. 4.2.1,
Listing 3) against the oracle's expression evaluator (oracle/expr.py:
numpy values, symbolic derivatives) and against the equivalent theory
programs.  Costs within a relative 1e-10 of the oracle; gradients within
1e-10 of sum_n |r_n dN_n/dp_k|; model values within 1e-13 relative."""

import numpy as np
import pytest

import synth
from oracle import expr, model
from paper_1604_02334_amd import api

from _workloads import counts_for, perturbed

pytestmark = pytest.mark.gpu
REL = 1e-10


@pytest.fixture(scope="module")
def ctx():
    c = api.Context(0)
    yield c
    c.close()


def _say(*a):
    print("[case]", *a, flush=True)


def _as_expr(th, e):
    return expr.theory_desc(e, th["tau_mu"], th["n0"], th["nbkg"], th["map"], th["n_par"], th.get("F"), th.get("f0"))


PROGRAMS = [
    (synth.theory_exp_cos, "p[2]*se(p[3])*tf(p[5],p[4])", [900.0, 3.0, 0.2, 0.8, 1.7, 0.3]),
    (synth.theory_gauss_cos, "p[2]*sg(p[3])*tf(p[5],p[4])", [900.0, 3.0, 0.2, 0.4, 1.7, 0.3]),
    (synth.theory_exp_gkt, "p[2]*se(p[3]) + p[4]*stg(p[5])", [900.0, 3.0, 0.15, 0.8, 0.12, 0.4]),
]


def _h1(n=6000, dt=0.0015):
    return [{"n_bins": n, "dt": dt, "t0_bin": 0.0, "first": 2, "last": n - 7, "map_row": 0}]


@pytest.mark.parametrize("kind", ["chi2", "poisson"])
def test_expression_restating_programs(ctx, kind):
    _say("rtc vs programs", kind)
    rng = np.random.default_rng(71)
    for make, e, p in PROGRAMS:
        th_d = make()
        ex = _as_expr(th_d, e)
        p = np.array(p)
        hs = _h1()
        cnt = counts_for(th_d, hs, p, rng)
        q = perturbed(p, 1e-2, 72)
        tp, te, d = api.Theory(ctx, th_d), api.Theory(ctx, ex), api.Data(ctx, hs, cnt)
        c_e, g_e = api.chi2_grad(ctx, d, te, q, kind)
        ref = model.cost(th_d, hs, cnt, q, kind)
        assert abs(c_e[0] - ref) <= REL * ref
        assert abs(api.chi2_eval(ctx, d, te, q, kind)[0] - ref) <= REL * ref
        refg = model.grad(th_d, hs, cnt, q, kind)
        scale = model.grad_abs_scale(th_d, hs, cnt, q, kind)
        assert np.all(np.abs(g_e[0] - refg) <= REL * scale), (e, g_e[0], refg)
        m = api.model_eval(ctx, d, te, q)
        np.testing.assert_allclose(m, model.model(th_d, hs[0], q), rtol=1e-13, atol=0)
        for x in (tp, te, d):
            x.close()


USER = ("p[2]*pow(1+t, -p[3])*cos(2*pi*p[4]*t + p[5]) + sqrt(p[6])*log(1 + p[7]*t)/(1+t)"
        " - 0.01*sin(f[0]*t)*p[8]^2")


def _user_theory():
    F = np.zeros((1, 9))
    F[0, 4] = 2.0
    ex = expr.theory_desc(USER, synth.TAU_MU, ("p", 0), ("p", 1), [list(range(9))], 9, F.tolist(), [0.1])
    p = np.array([900.0, 3.0, 0.2, 0.7, 1.3, 0.4, 0.01, 0.5, 0.3])
    return ex, p


@pytest.mark.parametrize("kind", ["chi2", "poisson"])
def test_user_expression_against_oracle(ctx, kind):
    _say("rtc user expression", kind)
    ex, p = _user_theory()
    hs = [{"n_bins": 5000, "dt": 0.002, "t0_bin": 0.0, "first": 0, "last": 4999, "map_row": 0},
          {"n_bins": 3001, "dt": 0.003, "t0_bin": 3.5, "first": 10, "last": 2990, "map_row": 0}]
    rng = np.random.default_rng(73)
    cnt = [rng.poisson(expr.model_expr_full(ex, h, p)).astype(float) for h in hs]
    te, d = api.Theory(ctx, ex), api.Data(ctx, hs, cnt)
    for seed in (74, 75):
        q = perturbed(p, 1e-2, seed)
        c, g = api.chi2_grad(ctx, d, te, q, kind)
        ref = expr.cost_expr(ex, hs, cnt, q, kind)
        assert abs(c[0] - ref) <= REL * ref
        refg = expr.grad_expr(ex, hs, cnt, q, kind)
        scale = expr.grad_abs_scale_expr(ex, hs, cnt, q, kind)
        assert np.all(np.abs(g[0] - refg) <= REL * scale), (g[0], refg)
        ce = api.chi2_eval(ctx, d, te, np.stack([q, p]), kind)
        assert abs(ce[0] - ref) <= REL * ref
        assert abs(ce[1] - expr.cost_expr(ex, hs, cnt, p, kind)) <= REL * ce[1]
    m = api.model_eval(ctx, d, te, p)
    ref = np.concatenate([expr.model_expr(ex, h, p) for h in hs])
    np.testing.assert_allclose(m, ref, rtol=1e-13, atol=0)
    te.close()
    d.close()


def test_expression_with_map_rows_and_function_array(ctx):
    """Eq. 4 over 8 detectors as an expression: per-detector amplitude and
    phase through the map, shared sigma, and the frequency nu = gamma B / 2 pi
    from the function array."""
    _say("rtc eq4")
    ps = synth.config_paper_shape(n_bins=4000, n_det=8)
    th = ps["theory"]
    # map row j slots: 0 N0, 1 Nbkg, 2 A0, 3 sigma, 4 phi, 5 -> f index of nu
    ex = _as_expr(th, "p[2]*sg(p[3])*tf(p[4], f[5])")
    hs = ps["histos"]
    cnt = counts_for(th, hs, ps["p_true"], ps["rng"])
    te, tp, d = api.Theory(ctx, ex), api.Theory(ctx, th), api.Data(ctx, hs, cnt)
    q = perturbed(ps["p_true"], 1e-3, 76)
    for kind in ("chi2", "poisson"):
        c, g = api.chi2_grad(ctx, d, te, q, kind)
        ref = expr.cost_expr(ex, hs, cnt, q, kind)
        assert abs(c[0] - ref) <= REL * ref
        assert abs(c[0] - model.cost(th, hs, cnt, q, kind)) <= REL * ref
        refg = model.grad(th, hs, cnt, q, kind)
        scale = model.grad_abs_scale(th, hs, cnt, q, kind)
        assert np.all(np.abs(g[0] - refg) <= REL * scale)
    for x in (te, tp, d):
        x.close()


def test_batched_mix_fit_hesse_and_static_entry(ctx):
    """Run-time compiled jobs (two different expressions) batched with
    program jobs in one mu_chi2_batch call; a batched fit of an expression
    theory reaches the equivalent program's minimum; mu_hesse (Gauss-Newton)
    equals the program's; the allocation-free entry point accepts it."""
    import torch
    _say("rtc batch / fit / hesse / static")
    rng = np.random.default_rng(77)
    ex_u, pu = _user_theory()
    jobs = []
    for make, e, p in PROGRAMS:
        th_d = make()
        p = np.array(p)
        hs = _h1(3000, 0.003)
        cnt = counts_for(th_d, hs, p, rng)
        jobs.append((th_d, _as_expr(th_d, e), hs, cnt, perturbed(p, 1e-2, 78)))
    hs = _h1(2500, 0.004)
    cnt_u = [rng.poisson(expr.model_expr_full(ex_u, hs[0], pu)).astype(float)]
    ths, ds, P, refs = [], [], np.zeros((7, 9)), []
    for k, (th_d, ex, hh, cnt, q) in enumerate(jobs):
        ths += [api.Theory(ctx, ex), api.Theory(ctx, th_d)]
        ds += [api.Data(ctx, hh, cnt)] * 2
        P[2 * k, :q.size] = q
        P[2 * k + 1, :q.size] = q
        refs += [model.cost(th_d, hh, cnt, q)] * 2
    ths.append(api.Theory(ctx, ex_u))
    ds.append(api.Data(ctx, hs, cnt_u))
    qu = perturbed(pu, 1e-2, 79)
    P[6] = qu
    refs.append(expr.cost_expr(ex_u, hs, cnt_u, qu))
    c, g = api.chi2_batch(ctx, ds, ths, P, grad=True)
    for j in range(7):
        assert abs(c[j] - refs[j]) <= REL * refs[j], j
    refg = expr.grad_expr(ex_u, hs, cnt_u, qu)
    scale = expr.grad_abs_scale_expr(ex_u, hs, cnt_u, qu)
    assert np.all(np.abs(g[6] - refg) <= REL * scale)
    # fits: expression theory and its program from the same start
    th_d, ex, hh, cnt, q = jobs[0]
    te, tp, d = ths[0], ths[1], ds[0]
    pf, cov, r = api.fit_batch(ctx, [d, d], [te, tp], np.stack([q, q]))
    assert r[0]["status"] == 0 and r[1]["status"] == 0
    sig = np.sqrt(np.diag(cov[1]))
    assert np.all(np.abs(pf[0] - pf[1]) <= 1e-6 * np.maximum(np.abs(pf[1]), sig))
    He, _ = api.hesse(ctx, d, te, pf[1])
    Hp, _ = api.hesse(ctx, d, tp, pf[1])
    dg = np.sqrt(np.abs(np.diag(Hp)))
    assert np.all(np.abs(He - Hp) <= 1e-10 * np.outer(dg, dg))
    with torch.cuda.stream(ctx.torch_stream):
        Pd = torch.tensor(np.stack([q, pf[1]]), dtype=torch.float64, device="cuda")
        out = torch.empty(2, dtype=torch.float64, device="cuda")
        api.chi2_eval_static(ctx, d, te, Pd, out)
        ref = api.chi2_eval(ctx, d, te, Pd)
        torch.cuda.synchronize()
        assert torch.equal(out, ref)
    for x in ths + ds[::2] + [ds[-1]]:
        x.close()


@pytest.mark.parametrize("kind", ["chi2", "poisson"])
def test_further_primitives_against_oracle(ctx, kind):
    """sekt, ab, b, ifld, ibsl and j0 in a run-time compiled theory."""
    _say("rtc further primitives", kind)
    e = ("p[2]*sekt(p[3]) + p[4]*ab(p[5], p[6]) + 0.1*b(p[7], p[8]) + 0.05*ifld(p[9], p[7], p[8], p[3], p[6])"
         " - 0.02*ibsl(p[9], p[7], p[8], p[5], p[3]) + 0.01*j0(p[8]*t)")
    n = 10
    ex = expr.theory_desc(e, synth.TAU_MU, ("p", 0), ("p", 1), [list(range(n))], n)
    p = np.array([900.0, 3.0, 0.15, 0.6, 0.1, 0.5, 1.5, 0.3, 0.8, 0.6])
    hs = [{"n_bins": 4000, "dt": 0.0025, "t0_bin": 0.0, "first": 0, "last": 3999, "map_row": 0}]
    cnt = [np.random.default_rng(81).poisson(expr.model_expr_full(ex, hs[0], p)).astype(float)]
    te, d = api.Theory(ctx, ex), api.Data(ctx, hs, cnt)
    q = p * (1.0 + 0.02 * np.sin(np.arange(n)))
    c, g = api.chi2_grad(ctx, d, te, q, kind)
    ref = expr.cost_expr(ex, hs, cnt, q, kind)
    assert abs(c[0] - ref) <= REL * ref
    refg = expr.grad_expr(ex, hs, cnt, q, kind)
    scale = expr.grad_abs_scale_expr(ex, hs, cnt, q, kind)
    assert np.all(np.abs(g[0] - refg) <= REL * scale), (g[0], refg)
    np.testing.assert_allclose(api.model_eval(ctx, d, te, q), expr.model_expr(ex, hs[0], q), rtol=1e-13, atol=0)
    te.close()
    d.close()
