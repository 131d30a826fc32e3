"""Batched launches (mu_chi2_batch): the fit ranges of uneven jobs are
concatenated and cut into equal ranges, one per wave, in one launch for all
jobs of compiled theory shapes (each segment runs its own job's shape) plus
one for interpreted theories.  Parity against the FP64 oracle: costs within a
relative 1e-10, gradients within 1e-10 of sum_n |r_n dN_n/dp_k| (Eqs. 2-3)."""

import numpy as np
import pytest

import synth
from oracle import model
from paper_1604_02334_amd import api

from _workloads import c4, counts_for

pytestmark = pytest.mark.gpu
REL = 1e-10


@pytest.fixture(scope="module")
def ctx():
    c = api.Context(0)
    yield c
    c.close()


def _say(*a):
    print("[case]", *a, flush=True)


def _ge_theory():
    """A stretched exponential with a free beta: no compiled shape (interpreted)."""
    g = synth.theory_exp_cos()
    g["terms"][0]["factors"][0] = {"prim": "ge", "args": [("p", 3), ("p", 6)]}
    g["map"] = [list(range(7))]
    g["n_par"] = 7
    g["names"] = g["names"] + ["beta"]
    return g


@pytest.fixture(scope="module")
def mixed(ctx):
    """40 uneven single-histogram jobs of the four compiled families, two
    jobs of an interpreted theory, and one multi-histogram job (the paper's
    Eq. 4 over 4 detectors) between them."""
    cfg = synth.config_c4(n_sets=40, lo_exp=8, hi_exp=15)
    rng = cfg["rng"]
    jobs = [(s["theory"], s["histos"], s["start"]) for s in cfg["sets"]]
    g = _ge_theory()
    for k, nb in enumerate((3001, 777)):
        h = [{"n_bins": nb, "dt": 0.004, "t0_bin": 0.0, "first": 5, "last": nb - 2, "map_row": 0}]
        jobs.insert(7 + 11 * k, (g, h, np.array([900.0, 3.0, 0.2, 0.8, 1.7, 0.3, 1.3 + 0.2 * k])))
    ps = synth.config_paper_shape(n_bins=5000)
    jobs.insert(20, (ps["theory"], ps["histos"][:4], ps["p_true"] * (1.0 + 1e-3 * np.cos(np.arange(ps["p_true"].size)))))
    out = []
    ld = max(p.size for _, _, p in jobs)
    P = np.zeros((len(jobs), ld))
    for j, (th_d, hs, p) in enumerate(jobs):
        cnt = counts_for(th_d, hs, p * (1.0 + 0.01 * np.sin(np.arange(p.size) + j)), rng)
        out.append((th_d, hs, cnt, p))
        P[j, :p.size] = p
    ths = [api.Theory(ctx, t) for t, _, _, _ in out]
    ds = [api.Data(ctx, h, c) for _, h, c, _ in out]
    return out, ths, ds, P


@pytest.mark.parametrize("tile", [0, 64, 1000, 2048, 8192, 65536, 1 << 20])
def test_batch_ranges_against_oracle(ctx, mixed, tile):
    """Every bins-per-wave value, from one bin per lane to more than the
    whole batch: cost and gradient of every job against the oracle."""
    _say("batch ranges", tile)
    jobs, ths, ds, P = mixed
    old = ctx.tile
    try:
        ctx.tile = tile
        for kind in ("chi2", "poisson"):
            c = api.chi2_batch(ctx, ds, ths, P, kind)
            cg, g = api.chi2_batch(ctx, ds, ths, P, kind, grad=True)
            for j, (th_d, hs, cnt, p) in enumerate(jobs):
                ref = model.cost(th_d, hs, cnt, p, kind)
                assert abs(c[j] - ref) <= REL * ref, (tile, kind, j, c[j], ref)
                assert abs(cg[j] - ref) <= REL * ref, (tile, kind, j, cg[j], ref)
                refg = model.grad(th_d, hs, cnt, p, kind)
                scale = model.grad_abs_scale(th_d, hs, cnt, p, kind)
                assert np.all(np.abs(g[j, :p.size] - refg) <= REL * scale), (tile, kind, j)
                assert np.all(g[j, p.size:] == 0.0)
    finally:
        ctx.tile = old


def test_batch_job_order_and_repeats(ctx, mixed):
    """A job's cost does not depend on its neighbours beyond rounding: the
    same jobs reversed, and one job repeated, give the same costs to 1e-13;
    repeating a call gives bitwise equal results."""
    _say("batch order")
    jobs, ths, ds, P = mixed
    c = api.chi2_batch(ctx, ds, ths, P)
    np.testing.assert_array_equal(api.chi2_batch(ctx, ds, ths, P), c)
    r = api.chi2_batch(ctx, ds[::-1], ths[::-1], P[::-1].copy())[::-1]
    np.testing.assert_allclose(r, c, rtol=1e-13, atol=0)
    rep = api.chi2_batch(ctx, [ds[3]] * 5, [ths[3]] * 5, np.repeat(P[3:4], 5, axis=0))
    np.testing.assert_allclose(rep, c[3], rtol=1e-13, atol=0)


def test_batch_autotune_keeps_parity_and_cache_round_trip(ctx, mixed, tmp_path):
    """mu_autotune_batch picks a (bins per wave, anchor) pair for this batch
    and later launches use it with unchanged parity; the choice survives a
    save / load round trip of the tuning cache, and a corrupt or foreign
    cache loads nothing."""
    _say("batch autotune")
    jobs, ths, ds, P = mixed
    tile, anchor, us = api.autotune_batch(ctx, ds, ths, P)
    assert tile >= 64 and 32 <= anchor <= 256 and us > 0
    c = api.chi2_batch(ctx, ds, ths, P)
    for j, (th_d, hs, cnt, p) in enumerate(jobs):
        ref = model.cost(th_d, hs, cnt, p)
        assert abs(c[j] - ref) <= REL * ref
    path = str(tmp_path / "tune.txt")
    api.autotune_save(ctx, path)
    text = open(path).read()
    assert text.startswith("mu-autotune 1\narch gfx950")
    assert f" {tile} {anchor}\n" in text
    c2 = api.Context(0)
    try:
        api.autotune_load(c2, path)
        th2 = [api.Theory(c2, t) for t, _, _, _ in jobs]
        d2 = [api.Data(c2, h, cnt) for _, h, cnt, _ in jobs]
        # the loaded choice reproduces the tuned launch bit for bit
        np.testing.assert_array_equal(api.chi2_batch(c2, d2, th2, P), c)
        bad = tmp_path / "bad.txt"
        bad.write_text("mu-autotune 1\narch gfx950\n6 0 0 0 26 16384\n")
        with pytest.raises(api.A.MuError):
            api.autotune_load(c2, str(bad))
        other = tmp_path / "other.txt"
        other.write_text(text.replace("arch gfx950", "arch gfx942", 1))
        with pytest.raises(api.A.MuError) as e:
            api.autotune_load(c2, str(other))
        assert e.value.status == api.A.MU_E_UNSUPPORTED
        for x in th2 + d2:
            x.close()
    finally:
        c2.close()


def test_c4_one_pass_full_size(ctx):
    """The benchmark's C4 pass exactly as timed: 512 datasets of 2^12 .. 2^20
    bins in the four families, one vector each, default launch shape; every
    job's chi^2 and likelihood against the oracle."""
    _say("c4 one pass 512 datasets")
    cfg, cnts = c4()
    sets = cfg["sets"]
    ths = [api.Theory(ctx, s["theory"]) for s in sets]
    ds = [api.Data(ctx, s["histos"], c) for s, c in zip(sets, cnts)]
    P = np.zeros((len(sets), 6))
    for j, s in enumerate(sets):
        P[j, :s["start"].size] = s["start"]
    for kind in ("chi2", "poisson"):
        c = api.chi2_batch(ctx, ds, ths, P, kind)
        for j, s in enumerate(sets):
            ref = model.cost(s["theory"], s["histos"], cnts[j], s["start"], kind)
            assert abs(c[j] - ref) <= REL * ref, (kind, j, s["family"], c[j], ref)
    for x in ths + ds:
        x.close()
