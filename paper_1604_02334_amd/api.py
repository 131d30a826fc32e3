"""Python binding of the C ABI in include/mu.h.

Marshalling only: numpy arrays become host pointers (MU_MEM_HOST), CUDA
(HIP) torch tensors become device pointers on the context's stream
(MU_MEM_DEVICE).  Every evaluation runs in the library's HIP kernels.
"""

from __future__ import annotations

import array
import ctypes as C
import os

import numpy as np

from . import _abi as A


def _check(status, ctx_handle=None, what=""):
    if status != A.MU_OK:
        msg = ""
        if ctx_handle:
            raw = A.lib().mu_ctx_last_error(ctx_handle)
            msg = raw.decode() if raw else ""
        raise A.MuError(status, f"{what}: {msg or A.lib().mu_status_string(status).decode()}")


def _is_torch(x):
    try:
        import torch
        return isinstance(x, torch.Tensor)
    except ImportError:  # pragma: no cover
        return False


class Context:
    """A device, a default-priority stream and the library's scratch arena."""

    def __init__(self, device=0):
        import torch
        self.device = int(device)
        self.torch_stream = torch.cuda.Stream(device=self.device)
        h = C.c_void_p()
        st = A.lib().mu_ctx_create(self.device, C.c_void_p(self.torch_stream.cuda_stream), 0, C.byref(h))
        if st != A.MU_OK:
            raise A.MuError(st, "mu_ctx_create: " + A.lib().mu_status_string(st).decode())
        self.h = h
        self._children = []

    def close(self):
        for c in reversed(self._children):
            c.close()
        self._children = []
        if self.h:
            _check(A.lib().mu_ctx_destroy(self.h), self.h, "mu_ctx_destroy")
            self.h = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def synchronize(self):
        _check(A.lib().mu_ctx_synchronize(self.h), self.h, "mu_ctx_synchronize")

    @property
    def tile(self):
        return A.lib().mu_ctx_get_tile(self.h)

    @tile.setter
    def tile(self, bins):
        _check(A.lib().mu_ctx_set_tile(self.h, int(bins)), self.h, "mu_ctx_set_tile")

    @property
    def anchor(self):
        return A.lib().mu_ctx_get_anchor(self.h)

    @anchor.setter
    def anchor(self, every):
        _check(A.lib().mu_ctx_set_anchor(self.h, int(every)), self.h, "mu_ctx_set_anchor")

    def set_specialize(self, on):
        _check(A.lib().mu_ctx_set_specialize(self.h, 1 if on else 0), self.h, "mu_ctx_set_specialize")

    def timing(self, on):
        """Start (discarding earlier records) or stop event timing of kernel launches."""
        _check(A.lib().mu_ctx_timing(self.h, 1 if on else 0), self.h, "mu_ctx_timing")

    _TIME_KINDS = {"cost": 0, "grad": 1, "model": 2, "merge": 3, "grad_cost": 4}

    def timing_read(self, kind):
        """(launch count, summed milliseconds) of the recorded launches of `kind`
        ('cost', 'grad', 'model', 'merge' or 'grad_cost')."""
        n = C.c_int32()
        ms = C.c_double()
        _check(A.lib().mu_ctx_timing_read(self.h, self._TIME_KINDS[kind], C.byref(n), C.byref(ms)), self.h,
               "mu_ctx_timing_read")
        return n.value, ms.value

    # Ordering with torch's current stream for device tensors. A caller that
    # already runs on the context's stream (``with torch.cuda.stream(ctx.torch_stream)``)
    # needs no cross-stream event: work on one stream is ordered by itself.
    def _enter_device(self):
        import torch
        cur = torch.cuda.current_stream(self.device)
        if cur.cuda_stream == self.torch_stream.cuda_stream:
            return None
        self.torch_stream.wait_stream(cur)
        return cur

    def _leave_device(self, cur, tensors):
        if cur is None:
            return
        cur.wait_stream(self.torch_stream)
        for t in tensors:
            if t is not None:
                t.record_stream(self.torch_stream)


def _ref(r):
    kind, x = r
    if kind == "p":
        return A.mu_ref(A.MU_REF_PAR, int(x), 0.0)
    if kind == "f":
        return A.mu_ref(A.MU_REF_FUN, int(x), 0.0)
    if kind == "lit":
        return A.mu_ref(A.MU_REF_LIT, 0, float(x))
    raise ValueError(f"unknown reference kind {kind!r}")


def theory_desc(theory):
    """Build a mu_theory_desc (and the arrays it points to) from a theory dict."""
    terms = theory["terms"]
    facs = []
    tarr = (A.mu_term * max(len(terms), 1))()
    for k, t in enumerate(terms):
        tarr[k].coef = float(t["coef"])
        tarr[k].amp = _ref(t["amp"])
        tarr[k].first_factor = len(facs)
        tarr[k].n_factors = len(t["factors"])
        for f in t["factors"]:
            mf = A.mu_factor()
            mf.prim = A.PRIM_CODES.get(f["prim"], 99) if isinstance(f["prim"], str) else int(f["prim"])
            for a, r in enumerate(f["args"]):
                mf.arg[a] = _ref(r)
            facs.append(mf)
    farr = (A.mu_factor * max(len(facs), 1))(*facs)
    m = np.ascontiguousarray(np.asarray(theory["map"], dtype=np.int32))
    if m.ndim != 2:
        raise ValueError("map must be two-dimensional")
    F = theory.get("F")
    keep = [tarr, farr, m]
    d = A.mu_theory_desc()
    d.tau_mu = float(theory["tau_mu"])
    d.n0 = _ref(theory["n0"])
    d.nbkg = _ref(theory["nbkg"])
    d.terms = C.cast(tarr, C.POINTER(A.mu_term))
    d.n_terms = len(terms)
    d.factors = C.cast(farr, C.POINTER(A.mu_factor))
    d.n_factors = len(facs)
    d.map = m.ctypes.data_as(C.POINTER(C.c_int32))
    d.n_rows, d.n_slots = m.shape
    if F is not None:
        Fa = np.ascontiguousarray(np.asarray(F, dtype=np.float64))
        f0 = np.ascontiguousarray(np.asarray(theory["f0"], dtype=np.float64))
        keep += [Fa, f0]
        d.F = Fa.ctypes.data_as(A.dp)
        d.f0 = f0.ctypes.data_as(A.dp)
        d.n_fun = Fa.shape[0]
    else:
        d.F = None
        d.f0 = None
        d.n_fun = 0
    d.n_par = int(theory["n_par"])
    return d, keep


def theory_check(theory):
    """Validate a theory dict without a device: (status, message)."""
    d, keep = theory_desc(theory)
    buf = C.create_string_buffer(512)
    st = A.lib().mu_theory_check(C.byref(d), buf, 512)
    return st, buf.value.decode()


def _histo_array(histos, counts):
    arr = (A.mu_histo * len(histos))()
    keep = []
    for j, (h, c) in enumerate(zip(histos, counts)):
        c = np.ascontiguousarray(np.asarray(c, dtype=np.float64))
        keep.append(c)
        arr[j].counts = c.ctypes.data
        arr[j].n_bins = int(h["n_bins"])
        arr[j].dt = float(h["dt"])
        arr[j].t0_bin = float(h.get("t0_bin", 0.0))
        arr[j].first = int(h.get("first", 0))
        arr[j].last = int(h.get("last", h["n_bins"] - 1))
        arr[j].map_row = int(h.get("map_row", 0))
    return arr, keep


def histo_check(histos, counts):
    arr, keep = _histo_array(histos, counts)
    buf = C.create_string_buffer(512)
    st = A.lib().mu_histo_check(arr, len(histos), buf, 512)
    return st, buf.value.decode()


def expr_theory_desc(theory):
    """mu_expr_theory_desc (and its arrays) from a dict with "expr" (the
    asymmetry expression), "tau_mu", "n0", "nbkg", "map", "n_par" and
    optionally "F", "f0"."""
    m = np.ascontiguousarray(np.asarray(theory["map"], dtype=np.int32))
    if m.ndim != 2:
        raise ValueError("map must be two-dimensional")
    text = theory["expr"].encode()
    keep = [m, text]
    d = A.mu_expr_theory_desc()
    d.tau_mu = float(theory["tau_mu"])
    d.n0 = _ref(theory["n0"])
    d.nbkg = _ref(theory["nbkg"])
    d.asymmetry = text
    d.map = m.ctypes.data_as(C.POINTER(C.c_int32))
    d.n_rows, d.n_slots = m.shape
    F = theory.get("F")
    if F is not None:
        Fa = np.ascontiguousarray(np.asarray(F, dtype=np.float64))
        f0 = np.ascontiguousarray(np.asarray(theory["f0"], dtype=np.float64))
        keep += [Fa, f0]
        d.F = Fa.ctypes.data_as(A.dp)
        d.f0 = f0.ctypes.data_as(A.dp)
        d.n_fun = Fa.shape[0]
    else:
        d.F = None
        d.f0 = None
        d.n_fun = 0
    d.n_par = int(theory["n_par"])
    return d, keep


def theory_check_expr(theory):
    """Parse and validate an expression theory without a device: (status, message)."""
    d, keep = expr_theory_desc(theory)
    buf = C.create_string_buffer(1024)
    st = A.lib().mu_theory_check_expr(C.byref(d), buf, len(buf))
    return st, buf.value.decode()


def theory_compile_check(theory):
    """Compile an expression theory with hipRTC without a device: (status, message or log)."""
    d, keep = expr_theory_desc(theory)
    buf = C.create_string_buffer(16384)
    st = A.lib().mu_theory_compile_check(C.byref(d), buf, len(buf))
    return st, buf.value.decode(errors="replace")


def theory_expr_source(theory):
    """The generated HIP source of an expression theory."""
    d, keep = expr_theory_desc(theory)
    need = C.c_int64()
    _check(A.lib().mu_theory_expr_source(C.byref(d), None, 0, C.byref(need)), None, "mu_theory_expr_source")
    buf = C.create_string_buffer(need.value)
    _check(A.lib().mu_theory_expr_source(C.byref(d), buf, need.value, None), None, "mu_theory_expr_source")
    return buf.value.decode()


class Theory:
    """A theory on the device: a program dict (terms of primitives) or, with an
    "expr" key, a run-time compiled expression theory."""

    def __init__(self, ctx, theory):
        h = C.c_void_p()
        if "expr" in theory:
            d, keep = expr_theory_desc(theory)
            _check(A.lib().mu_theory_create_expr(ctx.h, C.byref(d), C.byref(h)), ctx.h, "mu_theory_create_expr")
        else:
            d, keep = theory_desc(theory)
            _check(A.lib().mu_theory_create(ctx.h, C.byref(d), C.byref(h)), ctx.h, "mu_theory_create")
        self.h = h
        self.addr = h.value  # the handle as an integer (batched calls pass arrays of them)
        self.ctx = ctx
        self.n_par = int(theory["n_par"])
        ctx._children.append(self)

    def close(self):
        if self.h:
            _check(A.lib().mu_theory_destroy(self.h), None, "mu_theory_destroy")
            self.h = None
            self.addr = 0


class Data:
    def __init__(self, ctx, histos, counts):
        arr, keep = _histo_array(histos, counts)
        h = C.c_void_p()
        _check(A.lib().mu_data_create(ctx.h, arr, len(histos), C.byref(h)), ctx.h, "mu_data_create")
        self.h = h
        self.addr = h.value  # the handle as an integer (batched calls pass arrays of them)
        self.ctx = ctx
        self.n_histo = len(histos)
        self.n_bins = int(A.lib().mu_data_bins(h))
        self.is_f64 = bool(A.lib().mu_data_is_f64(h))
        ctx._children.append(self)

    def close(self):
        if self.h:
            _check(A.lib().mu_data_destroy(self.h), None, "mu_data_destroy")
            self.h = None
            self.addr = 0


def handle_array(objs):
    """(keep-alive buffer, pointer) of the objects' native handles, contiguous,
    for the batched calls."""
    a = array.array("Q", [o.addr for o in objs])
    if 0 in a:
        raise ValueError("a dataset or theory handle is closed")
    return a, C.cast(a.buffer_info()[0], C.POINTER(C.c_void_p))


def _cost_code(cost):
    if cost not in A.COST_CODES:
        raise ValueError(f"cost must be one of {sorted(A.COST_CODES)}")
    return A.COST_CODES[cost]


def _as_host_params(params, n_par):
    p = np.ascontiguousarray(np.asarray(params, dtype=np.float64))
    if p.ndim == 1:
        p = p[None, :]
    if p.ndim != 2 or p.shape[1] != n_par:
        raise ValueError(f"params must have shape [n_vec, {n_par}]")
    return p


def chi2_eval(ctx, data, theory, params, cost="chi2", per_histo=False):
    """Cost of each parameter vector (and optionally of each histogram)."""
    L = A.lib()
    if _is_torch(params) and params.is_cuda:
        import torch
        p = params.detach().to(torch.float64).contiguous()
        if p.dim() == 1:
            p = p[None]
        n_vec = p.shape[0]
        out = torch.empty(n_vec, dtype=torch.float64, device=p.device)
        ph = torch.empty((n_vec, data.n_histo), dtype=torch.float64, device=p.device) if per_histo else None
        cur = ctx._enter_device()
        _check(L.mu_chi2_eval(ctx.h, data.h, theory.h, _cost_code(cost), C.c_void_p(p.data_ptr()), n_vec,
                              A.MU_MEM_DEVICE, C.c_void_p(out.data_ptr()),
                              C.c_void_p(ph.data_ptr()) if ph is not None else None), ctx.h, "mu_chi2_eval")
        ctx._leave_device(cur, [p, out, ph])
        return (out, ph) if per_histo else out
    p = _as_host_params(params, theory.n_par)
    n_vec = p.shape[0]
    out = np.empty(n_vec)
    ph = np.empty((n_vec, data.n_histo)) if per_histo else None
    _check(L.mu_chi2_eval(ctx.h, data.h, theory.h, _cost_code(cost), p.ctypes.data, n_vec, A.MU_MEM_HOST,
                          out.ctypes.data, ph.ctypes.data if ph is not None else None), ctx.h, "mu_chi2_eval")
    return (out, ph) if per_histo else out


def chi2_eval_static(ctx, data, theory, params, out, per_histo=None, cost="chi2"):
    """mu_chi2_eval_static: the cost of each vector of a CUDA tensor params
    [n_vec, n_par] into the caller's CUDA tensors out [n_vec] (and per_histo
    [n_vec, n_histo]), with no allocation by the library; enqueued on the
    context's stream."""
    L = A.lib()
    for t in (params, out) + ((per_histo,) if per_histo is not None else ()):
        if not (_is_torch(t) and t.is_cuda and t.is_contiguous()):
            raise ValueError("chi2_eval_static takes contiguous CUDA tensors only")
    n_vec = params.shape[0] if params.dim() == 2 else 1
    cur = ctx._enter_device()
    _check(L.mu_chi2_eval_static(ctx.h, data.h, theory.h, _cost_code(cost), C.c_void_p(params.data_ptr()), n_vec,
                                 C.c_void_p(out.data_ptr()),
                                 C.c_void_p(per_histo.data_ptr()) if per_histo is not None else None),
           ctx.h, "mu_chi2_eval_static")
    ctx._leave_device(cur, [params, out, per_histo])
    return out


def chi2_grad(ctx, data, theory, params, cost="chi2"):
    """Cost and analytic gradient of each parameter vector."""
    L = A.lib()
    if _is_torch(params) and params.is_cuda:
        import torch
        p = params.detach().to(torch.float64).contiguous()
        if p.dim() == 1:
            p = p[None]
        n_vec = p.shape[0]
        out = torch.empty(n_vec, dtype=torch.float64, device=p.device)
        g = torch.empty((n_vec, theory.n_par), dtype=torch.float64, device=p.device)
        cur = ctx._enter_device()
        _check(L.mu_chi2_grad(ctx.h, data.h, theory.h, _cost_code(cost), C.c_void_p(p.data_ptr()), n_vec,
                              A.MU_MEM_DEVICE, C.c_void_p(out.data_ptr()), C.c_void_p(g.data_ptr())),
               ctx.h, "mu_chi2_grad")
        ctx._leave_device(cur, [p, out, g])
        return out, g
    p = _as_host_params(params, theory.n_par)
    n_vec = p.shape[0]
    out = np.empty(n_vec)
    g = np.empty((n_vec, theory.n_par))
    _check(L.mu_chi2_grad(ctx.h, data.h, theory.h, _cost_code(cost), p.ctypes.data, n_vec, A.MU_MEM_HOST,
                          out.ctypes.data, g.ctypes.data), ctx.h, "mu_chi2_grad")
    return out, g


def chi2_eval_grad(ctx, data, theory, params_grad, params_cost, cost="chi2"):
    """Cost and gradient at params_grad and cost at params_cost in one call
    (the two passes overlap on the device). Returns (cost_grad, grad, cost)."""
    L = A.lib()
    if _is_torch(params_grad) and params_grad.is_cuda:
        import torch
        pg = params_grad.detach().to(torch.float64).contiguous()
        pc = params_cost.detach().to(torch.float64).contiguous()
        if pg.dim() == 1:
            pg = pg[None]
        if pc.dim() == 1:
            pc = pc[None]
        dev = pg.device
        cg = torch.empty(pg.shape[0], dtype=torch.float64, device=dev)
        g = torch.empty((pg.shape[0], theory.n_par), dtype=torch.float64, device=dev)
        cc = torch.empty(pc.shape[0], dtype=torch.float64, device=dev)
        cur = ctx._enter_device()
        _check(L.mu_chi2_eval_grad(ctx.h, data.h, theory.h, _cost_code(cost), C.c_void_p(pg.data_ptr()), pg.shape[0],
                                   C.c_void_p(pc.data_ptr()), pc.shape[0], A.MU_MEM_DEVICE,
                                   C.c_void_p(cg.data_ptr()), C.c_void_p(g.data_ptr()), C.c_void_p(cc.data_ptr())),
               ctx.h, "mu_chi2_eval_grad")
        ctx._leave_device(cur, [pg, pc, cg, g, cc])
        return cg, g, cc
    pg = _as_host_params(params_grad, theory.n_par)
    pc = _as_host_params(params_cost, theory.n_par)
    cg = np.empty(pg.shape[0])
    g = np.empty((pg.shape[0], theory.n_par))
    cc = np.empty(pc.shape[0])
    _check(L.mu_chi2_eval_grad(ctx.h, data.h, theory.h, _cost_code(cost), pg.ctypes.data, pg.shape[0], pc.ctypes.data,
                               pc.shape[0], A.MU_MEM_HOST, cg.ctypes.data, g.ctypes.data, cc.ctypes.data),
           ctx.h, "mu_chi2_eval_grad")
    return cg, g, cc


def chi2_batch(ctx, datas, theories, params, cost="chi2", grad=False):
    """One launch over independent (dataset, theory, vector) jobs.
    params: [n_jobs, ld] with ld >= every theory's n_par."""
    L = A.lib()
    n = len(datas)
    if len(theories) != n:
        raise ValueError("need one theory per dataset")
    keep_d, dh = handle_array(datas)
    keep_t, th = handle_array(theories)
    if _is_torch(params) and params.is_cuda:
        import torch
        p = params.detach().to(torch.float64).contiguous()
        ld = p.shape[1]
        out = torch.empty(n, dtype=torch.float64, device=p.device)
        g = torch.zeros((n, ld), dtype=torch.float64, device=p.device) if grad else None
        cur = ctx._enter_device()
        _check(L.mu_chi2_batch(ctx.h, n, dh, th, _cost_code(cost), ld, C.c_void_p(p.data_ptr()), A.MU_MEM_DEVICE,
                               C.c_void_p(out.data_ptr()), C.c_void_p(g.data_ptr()) if grad else None),
               ctx.h, "mu_chi2_batch")
        ctx._leave_device(cur, [p, out, g])
        return (out, g) if grad else out
    p = np.ascontiguousarray(np.asarray(params, dtype=np.float64))
    if p.ndim != 2 or p.shape[0] != n:
        raise ValueError("params must have shape [n_jobs, ld]")
    ld = p.shape[1]
    out = np.empty(n)
    g = np.zeros((n, ld)) if grad else None
    _check(L.mu_chi2_batch(ctx.h, n, dh, th, _cost_code(cost), ld, p.ctypes.data, A.MU_MEM_HOST, out.ctypes.data,
                           g.ctypes.data if grad else None), ctx.h, "mu_chi2_batch")
    return (out, g) if grad else out


def model_eval(ctx, data, theory, params):
    """Expected counts N (Eq. 1) at every fit-range bin, histograms concatenated."""
    L = A.lib()
    if _is_torch(params) and params.is_cuda:
        import torch
        p = params.detach().to(torch.float64).contiguous().reshape(-1)
        out = torch.empty(data.n_bins, dtype=torch.float64, device=p.device)
        cur = ctx._enter_device()
        _check(L.mu_model_eval(ctx.h, data.h, theory.h, C.c_void_p(p.data_ptr()), A.MU_MEM_DEVICE,
                               C.c_void_p(out.data_ptr())), ctx.h, "mu_model_eval")
        ctx._leave_device(cur, [p, out])
        return out
    p = _as_host_params(params, theory.n_par)[0]
    p = np.ascontiguousarray(p)
    out = np.empty(data.n_bins)
    _check(L.mu_model_eval(ctx.h, data.h, theory.h, p.ctypes.data, A.MU_MEM_HOST, out.ctypes.data), ctx.h,
           "mu_model_eval")
    return out


def autotune(ctx, data, theory, params, cost="chi2", grad=False):
    """Measure tile / anchor candidates for this workload and remember the
    fastest in the context.  Returns (tile, anchor, microseconds per launch)."""
    L = A.lib()
    bt, ba, us = C.c_int32(), C.c_int32(), C.c_double()
    if _is_torch(params) and params.is_cuda:
        import torch
        p = params.detach().to(torch.float64).contiguous()
        if p.dim() == 1:
            p = p[None]
        cur = ctx._enter_device()
        _check(L.mu_autotune(ctx.h, data.h, theory.h, _cost_code(cost), C.c_void_p(p.data_ptr()), p.shape[0],
                             A.MU_MEM_DEVICE, 1 if grad else 0, C.byref(bt), C.byref(ba), C.byref(us)),
               ctx.h, "mu_autotune")
        ctx._leave_device(cur, [p])
    else:
        p = _as_host_params(params, theory.n_par)
        _check(L.mu_autotune(ctx.h, data.h, theory.h, _cost_code(cost), p.ctypes.data, p.shape[0], A.MU_MEM_HOST,
                             1 if grad else 0, C.byref(bt), C.byref(ba), C.byref(us)), ctx.h, "mu_autotune")
    return bt.value, ba.value, us.value


def autotune_set(ctx, data, theory, n_vec, tile, anchor, cost="chi2", grad=False):
    """Record a (tile, anchor) choice for launches of n_vec vectors over this
    dataset and theory, as if autotune had measured it."""
    _check(A.lib().mu_autotune_set(ctx.h, data.h, theory.h, _cost_code(cost), int(n_vec), 1 if grad else 0,
                                   int(tile), int(anchor)), ctx.h, "mu_autotune_set")


def autotune_batch(ctx, datas, theories, params, cost="chi2", grad=False):
    """Measure bins-per-wave / anchor candidates for batched launches of these
    jobs and remember the fastest in the context.  params: [n_jobs, ld] host
    array or CUDA tensor.  Returns (bins per wave, anchor, microseconds per call)."""
    L = A.lib()
    n = len(datas)
    keep_d, dh = handle_array(datas)
    keep_t, th = handle_array(theories)
    bt, ba, us = C.c_int32(), C.c_int32(), C.c_double()
    if _is_torch(params) and params.is_cuda:
        import torch
        p = params.detach().to(torch.float64).contiguous()
        cur = ctx._enter_device()
        _check(L.mu_autotune_batch(ctx.h, n, dh, th, _cost_code(cost), p.shape[1], C.c_void_p(p.data_ptr()),
                                   A.MU_MEM_DEVICE, 1 if grad else 0, C.byref(bt), C.byref(ba), C.byref(us)),
               ctx.h, "mu_autotune_batch")
        ctx._leave_device(cur, [p])
    else:
        p = np.ascontiguousarray(np.asarray(params, dtype=np.float64))
        if p.ndim != 2 or p.shape[0] != n:
            raise ValueError("params must have shape [n_jobs, ld]")
        _check(L.mu_autotune_batch(ctx.h, n, dh, th, _cost_code(cost), p.shape[1], p.ctypes.data, A.MU_MEM_HOST,
                                   1 if grad else 0, C.byref(bt), C.byref(ba), C.byref(us)), ctx.h,
               "mu_autotune_batch")
    return bt.value, ba.value, us.value


def autotune_save(ctx, path):
    """Write the context's remembered tuning choices to a text cache file."""
    _check(A.lib().mu_autotune_save(ctx.h, os.fsencode(path)), ctx.h, "mu_autotune_save")


def autotune_load(ctx, path):
    """Add the choices of a tuning cache file to the context (raises on a
    malformed file or one written for another architecture; nothing is loaded then)."""
    _check(A.lib().mu_autotune_load(ctx.h, os.fsencode(path)), ctx.h, "mu_autotune_load")


def autotune_check_file(path):
    """Validate a tuning cache file without a device: (status, message)."""
    msg = C.create_string_buffer(512)
    st = A.lib().mu_autotune_check_file(os.fsencode(path), msg, len(msg))
    return st, msg.value.decode()


def fit_batch(ctx, datas, theories, start, cost="chi2", fixed=None, analytic_grad=True, batched=True,
              polish=True, max_fcn=0, max_iter=0, tol_edm=0.0, tol_step_rel=0.0, want_cov=True):
    """Minimise n_fits independent fits (host arrays).  start: [n_fits, ld].
    Returns (params [n_fits, ld], cov [n_fits, ld, ld] or None, list of result dicts)."""
    L = A.lib()
    n = len(datas)
    if len(theories) != n:
        raise ValueError("need one theory per dataset")
    s = np.ascontiguousarray(np.asarray(start, dtype=np.float64))
    if s.ndim == 1:
        s = s[None]
    if s.shape[0] != n:
        raise ValueError("start must have shape [n_fits, ld]")
    ld = s.shape[1]
    o = A.mu_fit_opts()
    o.max_fcn, o.max_iter = int(max_fcn), int(max_iter)
    o.tol_edm, o.tol_step_rel = float(tol_edm), float(tol_step_rel)
    o.analytic_grad, o.batched, o.polish = int(bool(analytic_grad)), int(bool(batched)), int(bool(polish))
    fx = None
    if fixed is not None:
        fx = np.ascontiguousarray(np.broadcast_to(np.asarray(fixed, dtype=np.uint8), (n, ld)))
        o.fixed = fx.ctypes.data
    out = np.empty((n, ld))
    cov = np.empty((n, ld, ld)) if want_cov else None
    res = (A.mu_fit_result * n)()
    keep_d, dh = handle_array(datas)
    keep_t, th = handle_array(theories)
    _check(L.mu_fit_batch(ctx.h, n, dh, th, _cost_code(cost), ld, s.ctypes.data, C.byref(o), out.ctypes.data,
                          cov.ctypes.data if want_cov else None, res), ctx.h, "mu_fit_batch")
    rs = [{"cost": r.cost, "edm": r.edm, "n_iter": r.n_iter, "n_fcn": r.n_fcn, "n_grad": r.n_grad,
           "status": r.status} for r in res]
    return out, cov, rs


def _fixed_array(fixed, n):
    if fixed is None:
        return None
    return np.ascontiguousarray(np.broadcast_to(np.asarray(fixed, dtype=np.uint8), (n,)))


def hesse(ctx, data, theory, params, cost="chi2", method="gauss_newton", fixed=None):
    """Hessian and covariance 2 H^-1 at params (host arrays).  method:
    "gauss_newton" (Jacobian rows + FP64 matrix-core Gram kernel) or "diff"
    (central differences of the analytic gradient).  Returns (H, cov or None
    when H is not positive definite)."""
    n = theory.n_par
    p = np.ascontiguousarray(np.asarray(params, dtype=np.float64).reshape(-1))
    if p.size != n:
        raise ValueError("params must have n_par entries")
    fx = _fixed_array(fixed, n)
    H = np.empty((n, n))
    cov = np.empty((n, n))
    pd = C.c_int32()
    m = {"gauss_newton": A.MU_HESSE_GAUSS_NEWTON, "diff": A.MU_HESSE_DIFF}[method]
    _check(A.lib().mu_hesse(ctx.h, data.h, theory.h, _cost_code(cost), m, p.ctypes.data,
                            fx.ctypes.data if fx is not None else None, H.ctypes.data, cov.ctypes.data,
                            C.byref(pd)), ctx.h, "mu_hesse")
    return H, (cov if pd.value else None)


def profile(ctx, data, theory, p_min, k, values, cost="chi2", fixed=None):
    """Profile cost of parameter k at each value (the other free parameters
    minimised in one batched fit).  Returns (costs, params, statuses)."""
    n = theory.n_par
    p = np.ascontiguousarray(np.asarray(p_min, dtype=np.float64).reshape(-1))
    v = np.ascontiguousarray(np.asarray(values, dtype=np.float64).reshape(-1))
    fx = _fixed_array(fixed, n)
    pc = np.empty(v.size)
    pp = np.empty((v.size, n))
    stt = np.empty(v.size, dtype=np.int32)
    _check(A.lib().mu_profile(ctx.h, data.h, theory.h, _cost_code(cost), p.ctypes.data,
                              fx.ctypes.data if fx is not None else None, int(k), v.size, v.ctypes.data,
                              pc.ctypes.data, pp.ctypes.data, stt.ctypes.data), ctx.h, "mu_profile")
    return pc, pp, stt


def minos(ctx, data, theory, p_min, k, cost="chi2", up=1.0, fixed=None):
    """Profile-likelihood errors of parameter k: (err_lo, err_hi, rounds)."""
    n = theory.n_par
    p = np.ascontiguousarray(np.asarray(p_min, dtype=np.float64).reshape(-1))
    fx = _fixed_array(fixed, n)
    lo, hi, r = C.c_double(), C.c_double(), C.c_int32()
    _check(A.lib().mu_minos(ctx.h, data.h, theory.h, _cost_code(cost), p.ctypes.data,
                            fx.ctypes.data if fx is not None else None, int(k), float(up), C.byref(lo), C.byref(hi),
                            C.byref(r)), ctx.h, "mu_minos")
    return lo.value, hi.value, r.value
