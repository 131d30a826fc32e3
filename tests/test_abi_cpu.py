"""The C ABI library without a GPU: it loads, exports every symbol that
include/mu.h declares, refuses to create a context, and validates theory
programs and histograms on the host."""

import ctypes
import os
import re
import subprocess

import numpy as np
import pytest

import synth
from paper_1604_02334_amd import _abi as A
from paper_1604_02334_amd import api

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    text = open(os.path.join(ROOT, "include", "mu.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(mu_[a-z0-9_]+)\s*\(", text)))


def test_library_exports_every_declared_symbol():
    L = A.lib()
    out = subprocess.run(["nm", "-D", "--defined-only", A.LIB_PATH], capture_output=True, text=True).stdout
    exported = set(re.findall(r"\bT (mu_[a-z0-9_]+)", out))
    declared = _declared()
    assert declared, "no declarations parsed"
    missing = [s for s in declared if s not in exported]
    assert not missing, missing
    for s in declared:
        assert hasattr(L, s)
    assert set(A.exported_symbols()) <= set(declared)
    assert L.mu_abi_version() == 1


def test_no_device_context_is_refused(monkeypatch):
    L = A.lib()
    h = ctypes.c_void_p()
    monkeypatch.setenv("MU_FORCE_NODEVICE", "1")
    assert L.mu_ctx_create(0, None, 0, ctypes.byref(h)) == A.MU_E_NODEVICE
    assert not h.value


def test_null_arguments_are_rejected():
    L = A.lib()
    assert L.mu_ctx_create(0, None, 0, None) == A.MU_E_ARG
    assert L.mu_ctx_destroy(None) == A.MU_E_ARG
    assert L.mu_data_destroy(None) == A.MU_E_ARG
    assert L.mu_theory_destroy(None) == A.MU_E_ARG
    assert L.mu_chi2_eval(None, None, None, 0, None, 1, 0, None, None) == A.MU_E_ARG
    assert L.mu_data_bins(None) == -1


@pytest.mark.parametrize("theory", [synth.theory_exp_cos(), synth.theory_c2(), synth.theory_paper_eq4(),
                                    synth.theory_stg(), synth.theory_exp_gkt(), synth.theory_gauss_cos()])
def test_valid_theories_pass(theory):
    st, msg = api.theory_check(theory)
    assert st == A.MU_OK, msg


def _bad(mutate):
    th = synth.theory_c2()
    mutate(th)
    return api.theory_check(th)


def test_theory_validation_errors():
    st, msg = _bad(lambda t: t.update(n_par=0))
    assert st == A.MU_E_ARG
    st, msg = _bad(lambda t: t.update(tau_mu=-1.0))
    assert st == A.MU_E_ARG and "tau_mu" in msg
    st, msg = _bad(lambda t: t["map"][3].__setitem__(0, 999))
    assert st == A.MU_E_ARG and "map[3][0]" in msg
    st, msg = _bad(lambda t: t["terms"][0]["factors"].__setitem__(0, {"prim": "xx", "args": [("p", 3)]}))
    assert st == A.MU_E_ARG and "primitive" in msg
    st, msg = _bad(lambda t: t["terms"][0].__setitem__("amp", ("p", 9)))
    assert st == A.MU_E_ARG and "slot" in msg
    st, msg = _bad(lambda t: t["terms"][0].__setitem__("amp", ("f", 2)))  # no function array
    assert st == A.MU_E_ARG
    st, msg = _bad(lambda t: t["terms"].extend([t["terms"][1]] * 3))
    assert st == A.MU_E_UNSUPPORTED
    st, msg = _bad(lambda t: t["terms"][0]["factors"].extend([{"prim": "sg", "args": [("p", 6)]}] * 2))
    assert st == A.MU_E_UNSUPPORTED
    g = synth.theory_exp_cos()
    g["terms"][0]["factors"][0] = {"prim": "ge", "args": [("p", 3), ("lit", 0.0)]}
    st, msg = api.theory_check(g)
    assert st == A.MU_E_ARG and "beta" in msg


def test_histogram_validation_errors():
    h = {"n_bins": 10, "dt": 0.01, "t0_bin": 0.0, "first": 0, "last": 9, "map_row": 0}
    good = np.arange(10, dtype=float)
    assert api.histo_check([h], [good])[0] == A.MU_OK
    assert api.histo_check([dict(h, dt=0.0)], [good])[0] == A.MU_E_ARG
    assert api.histo_check([dict(h, last=10)], [good])[0] == A.MU_E_ARG
    assert api.histo_check([dict(h, first=5, last=4)], [good])[0] == A.MU_E_ARG
    bad = good.copy()
    bad[3] = -1.0
    st, msg = api.histo_check([h], [bad])
    assert st == A.MU_E_ARG and "count 3" in msg
    bad[3] = np.nan
    assert api.histo_check([h], [bad])[0] == A.MU_E_ARG
    # a bad value outside the fit range is not read
    assert api.histo_check([dict(h, first=4)], [bad])[0] == A.MU_OK
    assert api.histo_check([], [])[0] == A.MU_E_ARG


def test_handle_array_is_contiguous_and_refuses_closed_handles():
    """The batched calls' handle arrays: the integer handles in order, one
    pointer to them, and an error (not a null handle passed on) for a closed
    dataset or theory."""
    from paper_1604_02334_amd import api

    class Handle:
        def __init__(self, addr):
            self.addr = addr

    objs = [Handle(4096 * (i + 1)) for i in range(5)]
    keep, ptr = api.handle_array(objs)
    assert [ptr[i] for i in range(5)] == [o.addr for o in objs]
    objs[3].addr = 0
    with pytest.raises(ValueError):
        api.handle_array(objs)


def _cache(tmp_path, text, name="tune.txt"):
    p = tmp_path / name
    p.write_text(text)
    return str(p)


def test_tuning_cache_file_validation(tmp_path):
    """The tuning cache text format is checked without a device: a good file
    passes; a missing file, a wrong header, a missing architecture line, a
    malformed line and every out-of-range field are refused (and a context
    would load nothing from such a file)."""
    head = "mu-autotune 1\narch gfx950:sramecc+:xnack-\n# shape mode cost kind log2 tile anchor\n"
    good = head + "6 0 0 0 26 16384 64\n5 1 0 1 20 8192 128\n\n"
    st, msg = api.autotune_check_file(_cache(tmp_path, good))
    assert st == A.MU_OK and "2 entries" in msg and "gfx950" in msg
    st, msg = api.autotune_check_file(str(tmp_path / "absent.txt"))
    assert st == A.MU_E_ARG and "cannot open" in msg
    st, msg = api.autotune_check_file(_cache(tmp_path, "mu-autotune 2\narch gfx950\n"))
    assert st == A.MU_E_ARG and "header" in msg
    st, msg = api.autotune_check_file(_cache(tmp_path, "mu-autotune 1\n6 0 0 0 26 16384 64\n"))
    assert st == A.MU_E_ARG and "arch" in msg
    st, msg = api.autotune_check_file(_cache(tmp_path, ""))
    assert st == A.MU_E_ARG
    bad_lines = ["6 0 0 0 26 16384", "6 0 0 0 26 16384 64 9", "7 0 0 0 26 16384 64", "6 2 0 0 26 16384 64",
                 "6 0 2 0 26 16384 64", "6 0 0 2 26 16384 64", "6 0 0 0 63 16384 64", "6 0 0 0 26 63 64",
                 "6 0 0 0 26 67108865 64", "6 0 0 0 26 16384 0", "6 0 0 0 26 16384 257", "six 0 0 0 26 16384 64"]
    for i, line in enumerate(bad_lines):
        st, msg = api.autotune_check_file(_cache(tmp_path, head + "6 0 0 0 26 16384 64\n" + line + "\n", f"b{i}.txt"))
        assert st == A.MU_E_ARG and "line 5" in msg, (line, msg)
