"""Seeded test inputs: synth recipes with expected counts from the oracle's
model (the GPU path never produces a test input or an expected value)."""

import functools

import numpy as np

import synth
from oracle import model


def counts_for(theory, histos, p, rng, noiseless=False):
    return synth.materialise(theory, histos, p, model.model_full, rng, noiseless=noiseless)


@functools.lru_cache(maxsize=None)
def c1():
    cfg = synth.config_c1()
    counts = counts_for(cfg["theory"], cfg["histos"], cfg["p_true"], synth.rng_for(cfg["seed_k"]))
    return cfg, counts


@functools.lru_cache(maxsize=None)
def c2():
    cfg = synth.config_c2()
    counts = counts_for(cfg["theory"], cfg["histos"], cfg["p_true"], cfg["rng"])
    return cfg, counts


@functools.lru_cache(maxsize=None)
def c3(n_vec=4096):
    cfg = synth.config_c3(n_vec)
    _, counts = c1()
    return cfg, counts


@functools.lru_cache(maxsize=None)
def c4(n_sets=512, lo=12, hi=20):
    cfg = synth.config_c4(n_sets=n_sets, lo_exp=lo, hi_exp=hi)
    rng = cfg["rng"]
    counts = [counts_for(s["theory"], s["histos"], s["p_true"], rng) for s in cfg["sets"]]
    return cfg, counts


def perturbed(p, rel=1e-2, seed=0):
    rng = np.random.default_rng(seed)
    q = np.asarray(p, dtype=np.float64) * (1.0 + rel * rng.uniform(-1, 1, np.size(p)))
    return q
