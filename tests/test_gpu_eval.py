"""GPU parity of the fused evaluation kernels against the FP64 oracle.

Bar (written here, derived from the target): every cost within a relative
1e-10 of the oracle's exactly rounded sum; gradients within 1e-10 of the
scale sum_n |r_n dN_n/dp_k| of the oracle's gradient and within 1e-6 of
central finite differences; model values within 1e-13 relative."""

import math

import numpy as np
import pytest

import synth
from oracle import model
from paper_1604_02334_amd import api

from _workloads import c1, c2, c3, counts_for, perturbed

pytestmark = pytest.mark.gpu
REL = 1e-10


@pytest.fixture(scope="module")
def ctx():
    c = api.Context(0)
    yield c
    c.close()


def _say(*a):
    print("[case]", *a, flush=True)


def _mk(ctx, theory, histos, counts):
    return api.Theory(ctx, theory), api.Data(ctx, histos, counts)


def _rounding_bound(theory, histos, counts, p, kind="chi2", ulps=256):
    """Largest cost difference expected between two evaluations whose expected
    counts N_n each carry up to `ulps` units of rounding (2^-53) of relative
    error, e.g. the cost pass, which folds N0, the lifetime and the term
    weights into its recurrence states, against the gradient pass, which keeps
    them apart. To first order the cost (Eq. 2 or 3) moves by
    sum_n |d term / d N| |N_n| ulps 2^-53; near the minimum |d term / d N| N is
    about 2 sqrt(N) per bin, so the relative bound is far above 2^-53. Anchors
    every 64 lane steps bound the recurrences' own drift well inside 256 ulps."""
    s = 0.0
    for h, c in zip(histos, counts):
        N = model.model(theory, h, p)
        d = np.asarray(c, dtype=np.float64)[h["first"]:h["last"] + 1]
        s += float(np.sum(np.abs(model.cost_dN(d, N, kind) * N)))
    return ulps * 2.0 ** -53 * s


@pytest.mark.parametrize("kind", ["chi2", "poisson"])
def test_c1_cost_parity(ctx, kind):
    _say("c1 cost", kind)
    cfg, counts = c1()
    th, d = _mk(ctx, cfg["theory"], cfg["histos"], counts)
    P = np.stack([cfg["p_true"], perturbed(cfg["p_true"], 1e-2, 1), perturbed(cfg["p_true"], 0.2, 2)])
    got = api.chi2_eval(ctx, d, th, P, kind)
    for v in range(P.shape[0]):
        ref = model.cost(cfg["theory"], cfg["histos"], counts, P[v], kind)
        assert abs(got[v] - ref) <= REL * abs(ref), (v, got[v], ref)


@pytest.mark.parametrize("kind", ["chi2", "poisson"])
def test_c2_cost_and_per_histo_parity(ctx, kind):
    _say("c2 cost", kind)
    cfg, counts = c2()
    th, d = _mk(ctx, cfg["theory"], cfg["histos"], counts)
    P = np.stack([cfg["p_true"], perturbed(cfg["p_true"], 1e-2, 3)])
    got, ph = api.chi2_eval(ctx, d, th, P, kind, per_histo=True)
    for v in range(P.shape[0]):
        ref_h = model.cost_per_histo(cfg["theory"], cfg["histos"], counts, P[v], kind)
        ref = model.cost(cfg["theory"], cfg["histos"], counts, P[v], kind)
        assert abs(got[v] - ref) <= REL * abs(ref), (v, got[v], ref)
        np.testing.assert_allclose(ph[v], ref_h, rtol=REL, atol=0)


def test_model_values_elementwise(ctx):
    _say("model values c2 / eq4")
    cfg, counts = c2()
    th, d = _mk(ctx, cfg["theory"], cfg["histos"], counts)
    p = perturbed(cfg["p_true"], 1e-2, 4)
    got = api.model_eval(ctx, d, th, p)
    ref = np.concatenate([model.model(cfg["theory"], h, p) for h in cfg["histos"]])
    np.testing.assert_allclose(got, ref, rtol=1e-13, atol=0)
    ps = synth.config_paper_shape(n_bins=4099)
    hs = [dict(h, first=7, last=4000) for h in ps["histos"][:3]]
    cnt = counts_for(ps["theory"], hs, ps["p_true"], ps["rng"])
    th2, d2 = _mk(ctx, ps["theory"], hs, cnt)
    got = api.model_eval(ctx, d2, th2, ps["p_true"])
    ref = np.concatenate([model.model(ps["theory"], h, ps["p_true"]) for h in hs])
    # nu = 13.55 MHz over 10 us: arguments of cos reach ~850 rad
    np.testing.assert_allclose(got, ref, rtol=1e-12, atol=0)


@pytest.mark.parametrize("kind", ["chi2", "poisson"])
def test_c1_gradient_parity(ctx, kind):
    _say("c1 grad", kind)
    cfg, counts = c1()
    th, d = _mk(ctx, cfg["theory"], cfg["histos"], counts)
    for seed, rel in ((5, 1e-2), (6, 1e-4)):
        p = perturbed(cfg["p_true"], rel, seed)
        c, g = api.chi2_grad(ctx, d, th, p, kind)
        ref = model.grad(cfg["theory"], cfg["histos"], counts, p, kind)
        scale = model.grad_abs_scale(cfg["theory"], cfg["histos"], counts, p, kind)
        assert np.all(np.abs(g[0] - ref) <= REL * scale), (g[0], ref)
        refc = model.cost(cfg["theory"], cfg["histos"], counts, p, kind)
        assert abs(c[0] - refc) <= REL * refc


def test_c1_gradient_vs_finite_differences(ctx):
    _say("c1 grad vs fd")
    cfg, counts = c1()
    th, d = _mk(ctx, cfg["theory"], cfg["histos"], counts)
    p = perturbed(cfg["p_true"], 1e-2, 7)
    _, g = api.chi2_grad(ctx, d, th, p)
    fd = model.grad_fd(cfg["theory"], cfg["histos"], counts, p)
    scale = np.maximum(np.abs(fd), np.max(np.abs(fd)) * 1e-3)
    assert np.all(np.abs(g[0] - fd) <= 1e-6 * scale)


@pytest.mark.parametrize("kind", ["chi2", "poisson"])
def test_c2_gradient_parity(ctx, kind):
    _say("c2 grad", kind)
    cfg, counts = c2()
    th, d = _mk(ctx, cfg["theory"], cfg["histos"], counts)
    p = perturbed(cfg["p_true"], 1e-2, 8)
    c, g = api.chi2_grad(ctx, d, th, p, kind)
    ref = model.grad(cfg["theory"], cfg["histos"], counts, p, kind)
    scale = model.grad_abs_scale(cfg["theory"], cfg["histos"], counts, p, kind)
    assert np.all(np.abs(g[0] - ref) <= REL * scale)


def test_c3_vectors_sampled(ctx):
    """4096 vectors in one launch (the benchmark's launch); 48 sampled vectors
    checked one by one against the oracle, every vector against a separate
    single-vector launch."""
    _say("c3 4096 vectors")
    cfg, counts = c3()
    th, d = _mk(ctx, cfg["theory"], cfg["histos"], counts)
    P = cfg["P"]
    got = api.chi2_eval(ctx, d, th, P)
    cg, gg = api.chi2_grad(ctx, d, th, P)
    # the cost pass folds N0, the lifetime and the term weights into its
    # recurrence states, the gradient pass keeps them apart: equal to rounding
    bound = np.array([_rounding_bound(cfg["theory"], cfg["histos"], counts, q) for q in P])
    assert np.all(np.abs(cg - got) <= bound)
    idx = np.random.default_rng(0).choice(P.shape[0], 48, replace=False)
    for v in idx:
        ref = model.cost(cfg["theory"], cfg["histos"], counts, P[v])
        assert abs(got[v] - ref) <= REL * ref
        # a separate launch may pick another tile size (other anchor
        # positions): equal to rounding
        one = api.chi2_eval(ctx, d, th, P[v])
        assert abs(one[0] - got[v]) <= bound[v]
    # at one fixed tile size the batched and separate launches are bitwise equal
    try:
        ctx.tile = 4096
        got4 = api.chi2_eval(ctx, d, th, P)
        for v in idx[:8]:
            assert api.chi2_eval(ctx, d, th, P[v])[0] == got4[v]
    finally:
        ctx.tile = 0
    for v in idx[:8]:
        ref = model.grad(cfg["theory"], cfg["histos"], counts, P[v])
        scale = model.grad_abs_scale(cfg["theory"], cfg["histos"], counts, P[v])
        assert np.all(np.abs(gg[v] - ref) <= REL * scale)


def test_deterministic_and_tile_independent(ctx):
    _say("determinism / tiles")
    cfg, counts = c2()
    th, d = _mk(ctx, cfg["theory"], cfg["histos"], counts)
    p = perturbed(cfg["p_true"], 1e-3, 9)
    first = api.chi2_grad(ctx, d, th, p)
    for _ in range(5):
        again = api.chi2_grad(ctx, d, th, p)
        np.testing.assert_array_equal(again[0], first[0])
        np.testing.assert_array_equal(again[1], first[1])
    old = ctx.tile
    try:
        for tb in (256, 1024, 2048, 8192, 16384, 65536):
            ctx.tile = tb
            c, g = api.chi2_grad(ctx, d, th, p)
            assert abs(c[0] - first[0][0]) <= 1e-13 * first[0][0]
            assert np.all(np.abs(g - first[1]) <= 1e-12 * np.max(np.abs(first[1])))
    finally:
        ctx.tile = old


def test_edge_cases(ctx):
    _say("edge cases")
    th_d = synth.theory_exp_cos()
    p = np.array([800.0, 4.0, 0.2, 0.7, 2.3, 0.4])
    rng = np.random.default_rng(12)
    histos = [
        {"n_bins": 1, "dt": 0.01, "t0_bin": 0.0, "first": 0, "last": 0, "map_row": 0},        # one bin
        {"n_bins": 257, "dt": 0.01, "t0_bin": 0.0, "first": 0, "last": 256, "map_row": 0},    # ragged
        {"n_bins": 5000, "dt": 0.002, "t0_bin": 13.5, "first": 100, "last": 4321, "map_row": 0},  # t0, range
        {"n_bins": 3000, "dt": 0.004, "t0_bin": 0.0, "first": 0, "last": 2999, "map_row": 0},
    ]
    cnt = counts_for(th_d, histos, p, rng)
    cnt[3][:] = np.floor(cnt[3] / 200.0)  # many empty bins
    th, d = _mk(ctx, th_d, histos, cnt)
    q = perturbed(p, 1e-2, 13)
    for kind in ("chi2", "poisson"):
        got, ph = api.chi2_eval(ctx, d, th, q, kind, per_histo=True)
        ref_h = model.cost_per_histo(th_d, histos, cnt, q, kind)
        np.testing.assert_allclose(ph[0], ref_h, rtol=REL, atol=1e-300)
        c, g = api.chi2_grad(ctx, d, th, q, kind)
        ref = model.grad(th_d, histos, cnt, q, kind)
        scale = model.grad_abs_scale(th_d, histos, cnt, q, kind)
        assert np.all(np.abs(g[0] - ref) <= REL * scale)
    # FP64 storage: non-integer (noiseless) counts
    hs = [{"n_bins": 700, "dt": 0.01, "t0_bin": 0.0, "first": 0, "last": 699, "map_row": 0}]
    nz = counts_for(th_d, hs, p, rng, noiseless=True)
    th2, d2 = _mk(ctx, th_d, hs, nz)
    assert d2.is_f64
    c = api.chi2_eval(ctx, d2, th2, p)
    assert 0.0 <= c[0] <= 1e-20 * float(np.sum(nz[0]))
    # non-finite parameters give NaN
    bad = p.copy()
    bad[3] = np.nan
    assert math.isnan(api.chi2_eval(ctx, d2, th2, bad)[0])
    # likelihood with N <= 0 < d is +inf
    neg = p.copy()
    neg[0], neg[1] = -100.0, 0.0
    assert api.chi2_eval(ctx, d2, th2, neg, "poisson")[0] == math.inf


def test_likelihood_extreme_expected_counts(ctx):
    """The likelihood's ratio d / N is d times a refined reciprocal while every
    N of a wave lies in [2^-1000, 2^1000], else the division. Expected counts
    from 4e-302 to 1e-299 and from 4e298 to 1e301 (histograms whose waves
    straddle 2^-1000 and 2^1000) take both paths; costs and gradients against
    the oracle at the parity bar."""
    _say("likelihood extreme N")
    th_d = synth.theory_exp_cos()
    hs = [{"n_bins": 6000, "dt": 0.002, "t0_bin": 0.0, "first": 0, "last": 5999, "map_row": 0}]
    rng = np.random.default_rng(5)
    cnt = [(rng.poisson(3.0, 6000) + 1).astype(np.float64)]
    th, d = _mk(ctx, th_d, hs, cnt)
    for n0 in (1e-299, 1e301):
        p = np.array([n0, 0.0, 0.2, 0.7, 2.3, 0.4])
        ref = model.cost(th_d, hs, cnt, p, "poisson")
        got = api.chi2_eval(ctx, d, th, p, "poisson")[0]
        assert math.isfinite(ref) and abs(got - ref) <= REL * abs(ref), (n0, got, ref)
        c, g = api.chi2_grad(ctx, d, th, p, "poisson")
        assert abs(c[0] - ref) <= REL * abs(ref)
        gref = model.grad(th_d, hs, cnt, p, "poisson")
        scale = model.grad_abs_scale(th_d, hs, cnt, p, "poisson")
        assert np.all(np.abs(g[0] - gref) <= REL * scale)


def test_primitive_coverage(ctx):
    """ge with a literal and a free beta, stg, sg and the function-array route."""
    _say("primitives")
    rng = np.random.default_rng(14)
    hs = [{"n_bins": 3000, "dt": 0.003, "t0_bin": 0.0, "first": 0, "last": 2999, "map_row": 0}]
    g = synth.theory_exp_cos()
    g["terms"][0]["factors"][0] = {"prim": "ge", "args": [("p", 3), ("p", 6)]}
    g["map"] = [list(range(7))]
    g["n_par"] = 7
    cases = [
        (g, np.array([900.0, 3.0, 0.2, 0.8, 1.7, 0.3, 1.4])),
        (synth.theory_gauss_cos(), np.array([900.0, 3.0, 0.2, 0.4, 1.7, 0.3])),
        (synth.theory_stg(), np.array([900.0, 3.0, 0.2, 0.45])),
        (synth.theory_exp_gkt(), np.array([900.0, 3.0, 0.15, 0.8, 0.12, 0.4])),
    ]
    for th_d, p in cases:
        cnt = counts_for(th_d, hs, p, rng)
        th, d = _mk(ctx, th_d, hs, cnt)
        q = perturbed(p, 1e-2, 15)
        for kind in ("chi2", "poisson"):
            c, gr = api.chi2_grad(ctx, d, th, q, kind)
            ref = model.cost(th_d, hs, cnt, q, kind)
            assert abs(c[0] - ref) <= REL * ref
            refg = model.grad(th_d, hs, cnt, q, kind)
            scale = model.grad_abs_scale(th_d, hs, cnt, q, kind)
            assert np.all(np.abs(gr[0] - refg) <= REL * scale), (th_d["names"], gr[0], refg)
    ps = synth.config_paper_shape(n_bins=6000)
    hs = ps["histos"][:4]
    cnt = counts_for(ps["theory"], hs, ps["p_true"], ps["rng"])
    th, d = _mk(ctx, ps["theory"], hs, cnt)
    q = perturbed(ps["p_true"], 1e-3, 16)
    c, gr = api.chi2_grad(ctx, d, th, q)
    assert abs(c[0] - model.cost(ps["theory"], hs, cnt, q)) <= REL * c[0]
    refg = model.grad(ps["theory"], hs, cnt, q)
    scale = model.grad_abs_scale(ps["theory"], hs, cnt, q)
    assert np.all(np.abs(gr[0] - refg) <= REL * scale)


def test_batch_uneven_datasets(ctx):
    """Independent datasets of uneven sizes and different theories in one launch."""
    _say("batch uneven")
    cfg = synth.config_c4(n_sets=24, lo_exp=8, hi_exp=14)
    rng = cfg["rng"]
    sets = cfg["sets"]
    cnts = [counts_for(s["theory"], s["histos"], s["p_true"], rng) for s in sets]
    ths = [api.Theory(ctx, s["theory"]) for s in sets]
    ds = [api.Data(ctx, s["histos"], c) for s, c in zip(sets, cnts)]
    ld = 6
    P = np.zeros((len(sets), ld))
    for j, s in enumerate(sets):
        P[j, :s["start"].size] = s["start"]
    for kind in ("chi2", "poisson"):
        c, g = api.chi2_batch(ctx, ds, ths, P, kind, grad=True)
        c_only = api.chi2_batch(ctx, ds, ths, P, kind)
        for j, s in enumerate(sets):
            n = s["start"].size
            # gradient pass against the (scaled-state) cost pass: to rounding
            bound = _rounding_bound(s["theory"], s["histos"], cnts[j], s["start"], kind)
            assert abs(c[j] - c_only[j]) <= bound, (j, c[j] - c_only[j], bound)
            ref = model.cost(s["theory"], s["histos"], cnts[j], s["start"], kind)
            assert abs(c[j] - ref) <= REL * ref, (j, s["family"])
            refg = model.grad(s["theory"], s["histos"], cnts[j], s["start"], kind)
            scale = model.grad_abs_scale(s["theory"], s["histos"], cnts[j], s["start"], kind)
            assert np.all(np.abs(g[j, :n] - refg) <= REL * scale), (j, s["family"])
            one = api.chi2_eval(ctx, ds[j], ths[j], s["start"], kind)
            assert abs(one[0] - c_only[j]) <= bound


def test_torch_device_path_and_autograd(ctx):
    import torch
    _say("torch + autograd")
    from paper_1604_02334_amd import Chi2
    cfg, counts = c1()
    th, d = _mk(ctx, cfg["theory"], cfg["histos"], counts)
    p = torch.tensor(perturbed(cfg["p_true"], 1e-2, 17), dtype=torch.float64, device="cuda", requires_grad=True)
    c = Chi2.apply(p, ctx, d, th, "chi2")
    (2.0 * c).backward()
    torch.cuda.synchronize()
    ref = model.grad(cfg["theory"], cfg["histos"], counts, p.detach().cpu().numpy())
    scale = model.grad_abs_scale(cfg["theory"], cfg["histos"], counts, p.detach().cpu().numpy())
    assert np.all(np.abs(p.grad.cpu().numpy() - 2.0 * ref) <= 2 * REL * scale)
    # the forward pass is the gradient pass: bitwise equal to its host-memory
    # launch, and equal to rounding to the (scaled-state) cost pass
    host_c, _ = api.chi2_grad(ctx, d, th, p.detach().cpu().numpy())
    assert c.item() == host_c[0]
    host = api.chi2_eval(ctx, d, th, p.detach().cpu().numpy())
    assert abs(c.item() - host[0]) <= _rounding_bound(cfg["theory"], cfg["histos"], counts, p.detach().cpu().numpy())


def test_specialised_kernels_match_generic_and_direct(ctx):
    """Each compiled shape against the generic interpreted kernel, and the
    recurrence path (anchor every 64 steps) against the shortest anchor
    interval (every fourth step) and the longest (256)."""
    _say("shapes vs generic, anchors")
    rng = np.random.default_rng(21)
    hs = [{"n_bins": 20000, "dt": 0.0005, "t0_bin": 0.0, "first": 3, "last": 19990, "map_row": 0}]
    cases = [(synth.theory_exp_cos(), np.array([900.0, 3.0, 0.2, 0.8, 7.7, 0.3])),
             (synth.theory_gauss_cos(), np.array([900.0, 3.0, 0.2, 0.9, 7.7, 0.3])),
             (synth.theory_stg(), np.array([900.0, 3.0, 0.2, 0.95])),
             (synth.theory_exp_gkt(), np.array([900.0, 3.0, 0.15, 0.8, 0.12, 0.4]))]
    c2cfg, c2counts = c2()
    for th_d, p in cases + [(c2cfg["theory"], c2cfg["p_true"])]:
        if th_d is c2cfg["theory"]:
            hh, cnt = c2cfg["histos"], c2counts
        else:
            hh, cnt = hs, counts_for(th_d, hs, p, rng)
        th, d = _mk(ctx, th_d, hh, cnt)
        q = perturbed(p, 1e-2, 22)
        for kind in ("chi2", "poisson"):
            ref_c, ref_g = api.chi2_grad(ctx, d, th, q, kind)
            gscale = np.max(np.abs(ref_g))
            try:
                ctx.set_specialize(False)
                c, g = api.chi2_grad(ctx, d, th, q, kind)
                assert abs(c[0] - ref_c[0]) <= 1e-13 * ref_c[0]
                assert np.all(np.abs(g - ref_g) <= 1e-11 * gscale)
                ctx.set_specialize(True)
                for anchor in (1, 256):
                    ctx.anchor = anchor
                    c, g = api.chi2_grad(ctx, d, th, q, kind)
                    assert abs(c[0] - ref_c[0]) <= 1e-12 * ref_c[0], (th_d["names"], kind, anchor, c[0], ref_c[0])
                    assert np.all(np.abs(g - ref_g) <= 1e-10 * gscale)
            finally:
                ctx.set_specialize(True)
                ctx.anchor = 0


def test_autotune_choice_keeps_parity(ctx):
    """The measured tile / anchor choice is remembered and used by later
    launches of the same size; their costs still match the oracle."""
    _say("autotune")
    cfg, counts = c1()
    th, d = _mk(ctx, cfg["theory"], cfg["histos"], counts)
    P = np.stack([perturbed(cfg["p_true"], 1e-3, 30 + v) for v in range(64)])
    tile, anchor, us = api.autotune(ctx, d, th, P)
    # bins per wave: a power of two or a whole-round split, at least one bin per lane
    assert tile >= 64 and anchor in (32, 64, 128, 256) and us > 0
    got = api.chi2_eval(ctx, d, th, P)
    for v in (0, 17, 63):
        ref = model.cost(cfg["theory"], cfg["histos"], counts, P[v])
        assert abs(got[v] - ref) <= REL * ref


def test_autotune_set_replays_a_choice(ctx):
    """Launches of the size a (tile, anchor) was recorded for keep parity
    with it; out-of-range values are refused."""
    _say("autotune_set")
    cfg, counts = c1()
    th, d = _mk(ctx, cfg["theory"], cfg["histos"], counts)
    P = np.stack([perturbed(cfg["p_true"], 1e-3, 50 + v) for v in range(16)])
    api.autotune_set(ctx, d, th, 16, 700, 8)
    api.autotune_set(ctx, d, th, 16, 1000, 16, grad=True)
    got = api.chi2_eval(ctx, d, th, P)
    cg, g = api.chi2_grad(ctx, d, th, P)
    for v in (0, 7, 15):
        ref = model.cost(cfg["theory"], cfg["histos"], counts, P[v])
        assert abs(got[v] - ref) <= REL * ref
        assert abs(cg[v] - ref) <= REL * ref
        rg = model.grad(cfg["theory"], cfg["histos"], counts, P[v])
        sc = model.grad_abs_scale(cfg["theory"], cfg["histos"], counts, P[v])
        assert np.all(np.abs(g[v] - rg) <= REL * sc)
    for bad in ((16, 63, 64), (16, 1 << 27, 64), (16, 1024, 0), (16, 1024, 257), (0, 1024, 64)):
        with pytest.raises(api.A.MuError):
            api.autotune_set(ctx, d, th, *bad)


def test_kernel_timing_records_each_launch(ctx):
    """Event timing counts every evaluation and merge launch by kind and gives
    positive durations; disabling stops recording; enabling clears."""
    _say("kernel timing")
    cfg, counts = c1()
    th, d = _mk(ctx, cfg["theory"], cfg["histos"], counts)
    P = np.stack([perturbed(cfg["p_true"], 1e-3, 40 + v) for v in range(4)])
    ctx.timing(True)
    api.chi2_eval(ctx, d, th, P)
    api.chi2_eval(ctx, d, th, P[:1])
    api.chi2_grad(ctx, d, th, P[:2])
    ctx.timing(False)
    api.chi2_eval(ctx, d, th, P)
    n, ms = ctx.timing_read("cost")
    assert n == 2 and ms > 0
    n, ms = ctx.timing_read("grad")
    assert n == 1 and ms > 0
    n, ms = ctx.timing_read("merge")
    assert n == 3 and ms > 0
    assert ctx.timing_read("model") == (0, 0.0)
    ctx.timing(True)
    assert ctx.timing_read("cost") == (0, 0.0)
    ctx.timing(False)


def _tiny_set(n_bins):
    th_d = synth.theory_exp_cos()
    p = np.array([800.0, 4.0, 0.2, 0.7, 2.3, 0.4])
    hs = [{"n_bins": n_bins, "dt": 0.01, "t0_bin": 0.0, "first": 0, "last": n_bins - 1, "map_row": 0}]
    return th_d, hs, counts_for(th_d, hs, p, np.random.default_rng(77)), p


@pytest.mark.parametrize("kind", ["chi2", "poisson"])
def test_one_vector_matches_two_vector_launch(ctx, kind):
    """At one fixed split, a one-vector call and a two-vector call evaluate
    the first vector's bins as the same segments (a range may run on into the
    second vector) and merge the same slots in the same order, so its cost,
    per-histogram costs and gradient agree bit for bit. Calls alternate and
    repeat; sets of one workgroup, of a ragged last workgroup and of many
    workgroups; costs against the oracle at the parity bar."""
    cfg, counts = c2()
    th2, d2 = _mk(ctx, cfg["theory"], cfg["histos"], counts)
    sets = [("c2", cfg["theory"], cfg["histos"], counts, cfg["p_true"], th2, d2)]
    for n_bins in (300, 64 * 5 * 7 + 13):
        th_d, hs, cnt, p = _tiny_set(n_bins)
        th, d = _mk(ctx, th_d, hs, cnt)
        sets.append((f"{n_bins} bins", th_d, hs, cnt, p, th, d))
    old = ctx.tile
    try:
        for name, th_d, hs, cnt, p_true, th, d in sets:
            for tile in (64, 4096):
                _say("one vs two vectors", kind, name, "tile", tile)
                ctx.tile = tile
                for rep in range(3):
                    p0 = perturbed(p_true, 1e-3, 300 + rep)
                    p1 = perturbed(p_true, 1e-3, 400 + rep)
                    c_one, h_one = api.chi2_eval(ctx, d, th, p0, kind, per_histo=True)
                    c_two, h_two = api.chi2_eval(ctx, d, th, np.stack([p0, p1]), kind, per_histo=True)
                    np.testing.assert_array_equal(c_one[0], c_two[0])
                    np.testing.assert_array_equal(h_one[0], h_two[0])
                    gc_one, g_one = api.chi2_grad(ctx, d, th, p0, kind)
                    gc_two, g_two = api.chi2_grad(ctx, d, th, np.stack([p0, p1]), kind)
                    np.testing.assert_array_equal(gc_one[0], gc_two[0])
                    np.testing.assert_array_equal(g_one[0], g_two[0])
                    if rep == 0 and tile == 4096:
                        ref = model.cost(th_d, hs, cnt, p0, kind)
                        assert abs(c_one[0] - ref) <= REL * abs(ref)
                        assert abs(gc_one[0] - ref) <= REL * abs(ref)
    finally:
        ctx.tile = old


@pytest.mark.parametrize("kind", ["chi2", "poisson"])
def test_eval_grad_overlapped_matches_separate_calls(ctx, kind):
    """The combined gradient + cost call against the separate calls: the
    stencil costs bit for bit (same launch shapes); the gradient pass, which
    in one launch may take longer ranges per wave, to rounding for chi^2 and
    bit for bit for the likelihood (two launches); host and device memory give
    the same bits; the stencil costs and the gradient match the oracle."""
    import torch
    _say("eval_grad overlapped", kind)
    cfg, counts = c2()
    th, d = _mk(ctx, cfg["theory"], cfg["histos"], counts)
    p0 = perturbed(cfg["p_true"], 1e-3, 51)
    P = np.stack([perturbed(cfg["p_true"], 1e-3, 60 + v) for v in range(9)])
    cg, g, cc = api.chi2_eval_grad(ctx, d, th, p0, P, kind)
    sg, sgg = api.chi2_grad(ctx, d, th, p0, kind)
    sc = api.chi2_eval(ctx, d, th, P, kind)
    np.testing.assert_array_equal(cc, sc)
    if kind == "poisson":
        np.testing.assert_array_equal(cg, sg)
        np.testing.assert_array_equal(g, sgg)
    scale = model.grad_abs_scale(cfg["theory"], cfg["histos"], counts, p0, kind)
    assert abs(cg[0] - sg[0]) <= _rounding_bound(cfg["theory"], cfg["histos"], counts, p0, kind)
    assert np.all(np.abs(g[0] - sgg[0]) <= 1e-12 * scale)
    ref_g = model.grad(cfg["theory"], cfg["histos"], counts, p0, kind)
    assert np.all(np.abs(g[0] - ref_g) <= REL * scale)
    for v in (0, 8):
        ref = model.cost(cfg["theory"], cfg["histos"], counts, P[v], kind)
        assert abs(cc[v] - ref) <= REL * ref
    dev = torch.device("cuda:0")
    with torch.cuda.stream(ctx.torch_stream):
        tcg, tg, tcc = api.chi2_eval_grad(ctx, d, th, torch.tensor(p0[None], device=dev),
                                          torch.tensor(P, device=dev), kind)
        torch.cuda.synchronize()
    np.testing.assert_array_equal(tcg.cpu().numpy(), cg)
    np.testing.assert_array_equal(tg.cpu().numpy(), g)
    np.testing.assert_array_equal(tcc.cpu().numpy(), cc)


@pytest.mark.parametrize("shape", ["exp_cos", "gauss_cos", "stg", "exp_gkt"])
def test_eval_grad_single_launch_every_compiled_shape(ctx, shape):
    """The single evaluation launch of the gradient and cost passes for each
    compiled shape (C2's is covered above): costs and gradient against the
    oracle, the costs at the cost vectors bit for bit against a separate
    call, and the gradient pass against a separate call to rounding. Uneven
    fit range, so ranges end inside the last wave."""
    _say("eval_grad single launch", shape)
    rng = np.random.default_rng(23)
    hs = [{"n_bins": 20000, "dt": 0.0005, "t0_bin": 0.0, "first": 3, "last": 19990, "map_row": 0}]
    th_d, p = {"exp_cos": (synth.theory_exp_cos(), np.array([900.0, 3.0, 0.2, 0.8, 7.7, 0.3])),
               "gauss_cos": (synth.theory_gauss_cos(), np.array([900.0, 3.0, 0.2, 0.9, 7.7, 0.3])),
               "stg": (synth.theory_stg(), np.array([900.0, 3.0, 0.2, 0.95])),
               "exp_gkt": (synth.theory_exp_gkt(), np.array([900.0, 3.0, 0.15, 0.8, 0.12, 0.4]))}[shape]
    counts = counts_for(th_d, hs, p, rng)
    th, d = _mk(ctx, th_d, hs, counts)
    p0 = perturbed(p, 1e-2, 24)
    P = np.stack([perturbed(p, 1e-2, 25 + v) for v in range(5)])
    cg, g, cc = api.chi2_eval_grad(ctx, d, th, p0, P)
    sg, sgg = api.chi2_grad(ctx, d, th, p0)
    np.testing.assert_array_equal(cc, api.chi2_eval(ctx, d, th, P))
    ref_c = model.cost(th_d, hs, counts, p0)
    ref_g = model.grad(th_d, hs, counts, p0)
    scale = model.grad_abs_scale(th_d, hs, counts, p0)
    assert abs(cg[0] - ref_c) <= REL * ref_c
    assert np.all(np.abs(g[0] - ref_g) <= REL * scale)
    assert abs(cg[0] - sg[0]) <= _rounding_bound(th_d, hs, counts, p0)
    assert np.all(np.abs(g[0] - sgg[0]) <= 1e-12 * scale)
    for v in range(5):
        ref = model.cost(th_d, hs, counts, P[v])
        assert abs(cc[v] - ref) <= REL * ref


@pytest.mark.parametrize("shape", ["exp_cos", "gauss_cos"])
def test_rotation_recurrences_across_the_switch(ctx, shape):
    """The cost and model passes follow a rotation's real part by a three-term
    recurrence when it turns by at least 1/16 (sine) per lane step, else by the
    complex rotation. Precession frequencies on both sides of that switch and
    far above it, at the longest anchor interval (256 steps): costs and model
    values against the oracle, and the cost pass against the gradient pass
    (which always rotates) to rounding. Lane step here: 64 x 0.0005 us, so
    sin(theta) = 1/16 at nu = 0.311 MHz."""
    _say("rotation recurrences", shape)
    rng = np.random.default_rng(26)
    hs = [{"n_bins": 40000, "dt": 0.0005, "t0_bin": 0.0, "first": 0, "last": 39999, "map_row": 0}]
    th_d = synth.theory_exp_cos() if shape == "exp_cos" else synth.theory_gauss_cos()
    try:
        ctx.anchor = 256
        for nu in (0.05, 0.29, 0.33, 3.0, 40.0):
            p = np.array([2000.0, 4.0, 0.25, 0.4, nu, 0.7])
            counts = counts_for(th_d, hs, p, rng)
            th, d = _mk(ctx, th_d, hs, counts)
            got = api.chi2_eval(ctx, d, th, p)[0]
            ref = model.cost(th_d, hs, counts, p)
            assert abs(got - ref) <= REL * ref, (nu, got, ref)
            cg, _ = api.chi2_grad(ctx, d, th, p)
            assert abs(cg[0] - got) <= _rounding_bound(th_d, hs, counts, p), nu
            m = api.model_eval(ctx, d, th, p)
            ref_m = model.model(th_d, hs[0], p)
            np.testing.assert_allclose(m, ref_m, rtol=1e-12, atol=0)
    finally:
        ctx.anchor = 0


def _stencil(p, rel=1e-4):
    rows = []
    for k in range(p.size):
        h = rel * max(abs(p[k]), 1.0)
        for sgn in (1.0, -1.0):
            q = p.copy()
            q[k] += sgn * h
            rows.append(q)
    return np.array(rows)


def test_bench_launch_configuration_sampled(ctx):
    """The launch the benchmark times: C2 (16 x 65536 bins), the 104-vector
    central-difference stencil plus the gradient at the centre in the same
    call, with the launch shapes the autotuner picks for both (as the
    benchmark does). Sampled stencil vectors against the oracle one by one,
    every vector against the default launch shape to rounding."""
    _say("bench launch configuration")
    cfg, counts = c2()
    th, d = _mk(ctx, cfg["theory"], cfg["histos"], counts)
    p0 = cfg["p_true"] * (1.0 + 1e-3 * np.cos(np.arange(cfg["p_true"].size)))
    S = _stencil(p0)
    assert S.shape == (104, 52)
    default = api.chi2_eval(ctx, d, th, S)
    api.autotune(ctx, d, th, S)
    api.autotune(ctx, d, th, p0[None, :], grad=True)
    cg, g, cc = api.chi2_eval_grad(ctx, d, th, p0, S)
    assert np.all(np.abs(cc - default) <= 1e-13 * default)
    for v in (0, 37, 88, 103):
        ref = model.cost(cfg["theory"], cfg["histos"], counts, S[v])
        assert abs(cc[v] - ref) <= REL * ref, (v, cc[v], ref)
    ref_g = model.grad(cfg["theory"], cfg["histos"], counts, p0)
    scale = model.grad_abs_scale(cfg["theory"], cfg["histos"], counts, p0)
    assert np.all(np.abs(g[0] - ref_g) <= REL * scale)
    assert abs(cg[0] - model.cost(cfg["theory"], cfg["histos"], counts, p0)) <= REL * cg[0]


def test_split_ranges_cross_histogram_and_vector_boundaries(ctx):
    """Uneven fit ranges and bins-per-wave values that divide nothing: wave
    ranges start inside histograms, cover several histograms and
    cross from one vector to the next; costs, per-histogram costs and
    gradients of every vector against the oracle."""
    _say("split ranges")
    th_d = synth.theory_c2(n_det=3)
    hs = [{"n_bins": 6000, "dt": 0.0005, "t0_bin": 0.0, "first": 17, "last": 5016, "map_row": 0},
          {"n_bins": 900, "dt": 0.001, "t0_bin": 2.0, "first": 0, "last": 776, "map_row": 1},
          {"n_bins": 13000, "dt": 0.0002, "t0_bin": 0.0, "first": 300, "last": 12644, "map_row": 2}]
    p = np.array([0.2, 0.5, 1.355, 0.3, 900.0, 2.0, 0.1, 1500.0, 1.0, 2.0, 700.0, 3.0, -1.0])
    counts = counts_for(th_d, hs, p, np.random.default_rng(71))
    th, d = _mk(ctx, th_d, hs, counts)
    P = np.stack([perturbed(p, 1e-2, 80 + v) for v in range(7)])
    refs = [model.cost(th_d, hs, counts, P[v]) for v in range(7)]
    refs_h = [model.cost_per_histo(th_d, hs, counts, P[v]) for v in range(7)]
    ref_g = [model.grad(th_d, hs, counts, P[v]) for v in range(7)]
    scales = [model.grad_abs_scale(th_d, hs, counts, P[v]) for v in range(7)]
    try:
        for W in (64, 100, 256, 300, 777, 1000, 5000, 18122, 20000, 100000):
            ctx.tile = W
            c, ph = api.chi2_eval(ctx, d, th, P, per_histo=True)
            cg, g = api.chi2_grad(ctx, d, th, P)
            for v in range(7):
                assert abs(c[v] - refs[v]) <= REL * refs[v], (W, v)
                assert np.all(np.abs(ph[v] - refs_h[v]) <= REL * np.abs(refs_h[v])), (W, v)
                assert abs(cg[v] - refs[v]) <= REL * refs[v], (W, v)
                assert np.all(np.abs(g[v] - ref_g[v]) <= REL * scales[v]), (W, v)
    finally:
        ctx.tile = 0


def test_reciprocal_table_boundary_counts(ctx):
    """Integer counts around the size of the reciprocal table (3072) and far
    above it, interleaved so that one wave mixes table reads with the
    hardware-reciprocal path; zeros take v = 1. A dataset whose counts all
    fit the table takes the lookup without range test: the same costs."""
    _say("reciprocal table boundary")
    th_d = synth.theory_exp_cos()
    pattern = np.array([0, 1, 2, 3, 2047, 2048, 3070, 3071, 3072, 3073, 4095, 65535, 1000000, 16777216, 123456789, 0])
    n = 50000
    cts = np.resize(pattern, n).astype(np.float64)
    hs = [{"n_bins": n, "dt": 0.0002, "t0_bin": 0.0, "first": 0, "last": n - 1, "map_row": 0}]
    th, d = _mk(ctx, th_d, hs, [cts])
    assert d.is_f64 is False  # every value is an integer below 2^29: 32-bit storage
    p = np.array([3000.0, 5.0, 0.2, 0.7, 3.3, 0.4])
    P = np.stack([p, perturbed(p, 0.1, 90)])
    got = api.chi2_eval(ctx, d, th, P)
    cg, g = api.chi2_grad(ctx, d, th, P)
    for v in range(2):
        ref = model.cost(th_d, hs, [cts], P[v])
        assert abs(got[v] - ref) <= REL * ref
        assert abs(cg[v] - ref) <= REL * ref
        rg = model.grad(th_d, hs, [cts], P[v])
        sc = model.grad_abs_scale(th_d, hs, [cts], P[v])
        assert np.all(np.abs(g[v] - rg) <= REL * sc)
    # the largest integer kept in 32-bit storage (as 8 d: 2^29 - 1) and the
    # first one that is not
    for top, f64 in ((2.0 ** 29 - 1, False), (2.0 ** 29, True)):
        c = cts.copy()
        c[5] = top
        dd = api.Data(ctx, hs, [c])
        assert dd.is_f64 is f64
        got_top = api.chi2_eval(ctx, dd, th, P[0])[0]
        ref_top = model.cost(th_d, hs, [c], P[0])
        assert abs(got_top - ref_top) <= REL * ref_top
    # largest count 3071: every lookup without the range test; one count of
    # 3072 more sends the same bins through the tested lookup
    small = np.resize(np.array([0, 1, 2, 3, 2047, 2048, 3070, 3071]), n).astype(np.float64)
    big = small.copy()
    big[-1] = 3072.0
    th2, d_small = _mk(ctx, th_d, hs, [small])
    d_big = api.Data(ctx, hs, [big])
    for v in range(2):
        c_small = api.chi2_eval(ctx, d_small, th2, P[v])[0]
        c_big = api.chi2_eval(ctx, d_big, th2, P[v])[0]
        ref_small = model.cost(th_d, hs, [small], P[v])
        ref_big = model.cost(th_d, hs, [big], P[v])
        assert abs(c_small - ref_small) <= REL * ref_small
        assert abs(c_big - ref_big) <= REL * ref_big


def test_eval_grad_argument_errors(ctx):
    _say("eval_grad errors")
    import ctypes as C
    from paper_1604_02334_amd import _abi as A
    cfg, counts = c1()
    th, d = _mk(ctx, cfg["theory"], cfg["histos"], counts)
    L = A.lib()
    p = np.ascontiguousarray(cfg["p_true"][None])
    out = np.zeros(8)
    g = np.zeros((1, 6))
    ok = L.mu_chi2_eval_grad(ctx.h, d.h, th.h, 0, p.ctypes.data, 1, p.ctypes.data, 1, A.MU_MEM_HOST,
                             out.ctypes.data, g.ctypes.data, out[1:].ctypes.data)
    assert ok == A.MU_OK
    assert L.mu_chi2_eval_grad(ctx.h, d.h, th.h, 0, p.ctypes.data, 1, p.ctypes.data, 0, A.MU_MEM_HOST,
                               out.ctypes.data, g.ctypes.data, out[1:].ctypes.data) == A.MU_E_ARG
    assert L.mu_chi2_eval_grad(ctx.h, d.h, th.h, 0, p.ctypes.data, 1, p.ctypes.data, 1, A.MU_MEM_HOST,
                               out.ctypes.data, None, out[1:].ctypes.data) == A.MU_E_ARG
    assert L.mu_chi2_eval_grad(ctx.h, d.h, th.h, 7, p.ctypes.data, 1, p.ctypes.data, 1, A.MU_MEM_HOST,
                               out.ctypes.data, g.ctypes.data, out[1:].ctypes.data) == A.MU_E_ARG
    assert b"cost" in L.mu_ctx_last_error(ctx.h)


def test_split_launch_many_histograms_unstaged(ctx):
    """More histograms than a split launch stages in LDS (256): the
    prologue reads offsets and map rows from memory; costs and gradients of
    several vectors against the oracle."""
    _say("split launch, 300 histograms")
    th_d = synth.theory_exp_cos()
    n_h = 300
    hs = [{"n_bins": 150 + (j % 7) * 13, "dt": 0.002, "t0_bin": 0.0, "first": 0, "last": 149 + (j % 7) * 13,
           "map_row": 0} for j in range(n_h)]
    p = np.array([800.0, 2.0, 0.2, 0.5, 3.0, 0.3])
    counts = counts_for(th_d, hs, p, np.random.default_rng(123))
    th, d = _mk(ctx, th_d, hs, counts)
    P = np.stack([perturbed(p, 1e-2, 130 + v) for v in range(3)])
    try:
        for W in (0, 1000, 7777):
            ctx.tile = W
            c = api.chi2_eval(ctx, d, th, P)
            cg, g = api.chi2_grad(ctx, d, th, P)
            for v in range(3):
                ref = model.cost(th_d, hs, counts, P[v])
                assert abs(c[v] - ref) <= REL * ref, (W, v)
                assert abs(cg[v] - ref) <= REL * ref, (W, v)
                rg = model.grad(th_d, hs, counts, P[v])
                sc = model.grad_abs_scale(th_d, hs, counts, P[v])
                assert np.all(np.abs(g[v] - rg) <= REL * sc), (W, v)
    finally:
        ctx.tile = 0


def _theory_multi_function(n_det=3):
    """exp*cos per detector with every phase a function of two parameters
    (phi_j = phi0 + j dphi + 0.1 j) and the frequency a function of two more
    (nu = 13.553879 B + 0.5 dnu + 0.01): n_det + 1 functions, each row of F
    with two non-zero entries, plus offsets f0."""
    from synth.recipes import TAU_MU
    n_par = 6 + 2 * n_det  # [A, lambda, B, dnu, phi0, dphi] + [N0_j, Nbkg_j]
    F = []
    f0 = []
    for j in range(n_det):
        row = [0.0] * n_par
        row[4], row[5] = 1.0, float(j)
        F.append(row)
        f0.append(0.1 * j)
    row = [0.0] * n_par
    row[2], row[3] = 13.553879, 0.5
    F.append(row)
    f0.append(0.01)
    rows = [[6 + 2 * j, 7 + 2 * j, 0, 1, j, n_det] for j in range(n_det)]
    return {"tau_mu": TAU_MU, "n0": ("p", 0), "nbkg": ("p", 1),
            "terms": [{"coef": 1.0, "amp": ("p", 2),
                       "factors": [{"prim": "se", "args": [("p", 3)]},
                                   {"prim": "tf", "args": [("f", 4), ("f", 5)]}]}],
            "map": rows, "F": F, "f0": f0, "n_par": n_par,
            "names": ["A", "lambda", "B", "dnu", "phi0", "dphi"] + sum(([f"N0_{j}", f"Nbkg_{j}"] for j in range(n_det)), [])}


@pytest.mark.parametrize("kind", ["chi2", "poisson"])
def test_function_array_references(ctx, kind):
    """Scalars taken from the function array f = F p + f0 (Sec. 4.2.1,
    Listing 3): Eq. 4 with the frequency a function of the field, and a theory
    whose phases and frequency are functions of several parameters. Costs,
    per-histogram costs and gradients (chain rule through F) against the
    oracle."""
    _say("function array", kind)
    th1 = synth.theory_paper_eq4(n_det=4)
    p1 = np.zeros(th1["n_par"])
    p1[0], p1[1] = 0.35, 1.0
    for j in range(4):
        p1[2 + 4 * j: 6 + 4 * j] = [900.0 + 100 * j, 3.0, 0.25, 2 * math.pi * j / 4]
    hs1 = [{"n_bins": 3000, "dt": 0.004, "t0_bin": 0.0, "first": 0, "last": 2999, "map_row": j} for j in range(4)]
    th2 = _theory_multi_function(3)
    p2 = np.array([0.2, 0.6, 0.1, 0.4, 0.3, 0.7, 1000.0, 2.0, 800.0, 4.0, 1200.0, 1.0])
    hs2 = [{"n_bins": 2500, "dt": 0.004, "t0_bin": 0.0, "first": 0, "last": 2499, "map_row": j} for j in range(3)]
    for th_d, hs, p, seed in ((th1, hs1, p1, 140), (th2, hs2, p2, 141)):
        counts = counts_for(th_d, hs, p, np.random.default_rng(seed))
        th, d = _mk(ctx, th_d, hs, counts)
        P = np.stack([perturbed(p, 1e-2, seed + v) for v in range(3)])
        c, ph = api.chi2_eval(ctx, d, th, P, kind, per_histo=True)
        cg, g = api.chi2_grad(ctx, d, th, P, kind)
        for v in range(3):
            ref = model.cost(th_d, hs, counts, P[v], kind)
            assert abs(c[v] - ref) <= REL * ref, (th_d["names"][:3], v)
            assert abs(cg[v] - ref) <= REL * ref
            rh = model.cost_per_histo(th_d, hs, counts, P[v], kind)
            assert np.all(np.abs(ph[v] - rh) <= REL * np.abs(rh))
            rg = model.grad(th_d, hs, counts, P[v], kind)
            sc = model.grad_abs_scale(th_d, hs, counts, P[v], kind)
            assert np.all(np.abs(g[v] - rg) <= REL * sc), (th_d["names"][:3], v, np.max(np.abs(g[v] - rg) / sc))
