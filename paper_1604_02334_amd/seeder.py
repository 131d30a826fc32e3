"""Python binding of the seeder entry points of include/mu.h (marshalling only)."""

from __future__ import annotations

import ctypes as C

import numpy as np

from . import _abi as A
from .api import _check, handle_array

_DECL = {
    "mu_seeder_param_count": (C.c_int64, []),
    "mu_seeder_create": (C.c_int, [C.c_void_p, C.c_void_p, C.POINTER(C.c_void_p)]),
    "mu_seeder_destroy": (C.c_int, [C.c_void_p]),
    "mu_seeder_get_params": (C.c_int, [C.c_void_p, C.c_void_p]),
    "mu_seeder_get_grads": (C.c_int, [C.c_void_p, C.c_void_p]),
    "mu_seeder_steps": (C.c_int64, [C.c_void_p]),
    "mu_gen_histos": (C.c_int, [C.c_void_p, C.c_uint64, C.c_uint64, C.c_int32, C.c_int32, C.c_uint, C.c_void_p,
                                C.c_void_p, C.c_void_p]),
    "mu_seeder_forward": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_int32, C.c_uint, C.c_void_p]),
    "mu_seeder_train_step": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_int32, C.c_float,
                                       C.c_int32, C.c_uint, C.c_void_p]),
    "mu_seeder_train": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]),
    "mu_seed_infer": (C.c_int, [C.c_void_p, C.c_void_p, C.c_int32, C.POINTER(C.c_void_p), C.c_void_p, C.c_void_p]),
    "mu_seeder_save": (C.c_int, [C.c_void_p, C.c_char_p]),
    "mu_seeder_layer": (C.c_int, [C.c_void_p, C.c_void_p, C.c_int32, C.c_int32, C.c_void_p, C.c_void_p, C.c_void_p,
                                  C.c_void_p]),
    "mu_seeder_load": (C.c_int, [C.c_void_p, C.c_char_p, C.POINTER(C.c_void_p)]),
}


DIMS = (1024, 512, 256, 128, 8)  # layer widths of the seeder network


class mu_seed_train_opts(C.Structure):
    _fields_ = [("seed", C.c_uint64), ("first_sample", C.c_uint64), ("batch", C.c_int32), ("steps", C.c_int32),
                ("lr", C.c_float), ("lr_final_frac", C.c_float)]


def _lib():
    L = A.lib()
    if not getattr(L, "_seeder_declared", False):
        for name, (res, args) in _DECL.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        L._seeder_declared = True
    return L


def param_count():
    return int(_lib().mu_seeder_param_count())


def gen_histos(ctx, seed, first, n, fine=False, want_mu=False):
    """(counts [n][nb] float32, theta [n][6], mu [n][nb] or None), nb = 8192 if fine else 1024."""
    nb = 8192 if fine else 1024
    counts = np.empty((n, nb), dtype=np.float32)
    theta = np.empty((n, 6))
    mu = np.empty((n, nb)) if want_mu else None
    _check(_lib().mu_gen_histos(ctx.h, int(seed), int(first), int(n), 1 if fine else 0, A.MU_MEM_HOST,
                                counts.ctypes.data, theta.ctypes.data, mu.ctypes.data if want_mu else None),
           ctx.h, "mu_gen_histos")
    return counts, theta, mu


class Seeder:
    def __init__(self, ctx, init_params=None, handle=None):
        self.ctx = ctx
        L = _lib()
        if handle is None:
            p = np.ascontiguousarray(np.asarray(init_params, dtype=np.float32))
            if p.size != param_count():
                raise ValueError(f"need {param_count()} initial parameters")
            h = C.c_void_p()
            _check(L.mu_seeder_create(ctx.h, p.ctypes.data, C.byref(h)), ctx.h, "mu_seeder_create")
            handle = h
        self.h = handle
        ctx._children.append(self)

    @classmethod
    def load(cls, ctx, path):
        h = C.c_void_p()
        _check(_lib().mu_seeder_load(ctx.h, str(path).encode(), C.byref(h)), ctx.h, "mu_seeder_load")
        return cls(ctx, handle=h)

    def save(self, path):
        _check(_lib().mu_seeder_save(self.h, str(path).encode()), self.ctx.h, "mu_seeder_save")

    def close(self):
        if self.h:
            _check(_lib().mu_seeder_destroy(self.h), None, "mu_seeder_destroy")
            self.h = None

    def params(self):
        out = np.empty(param_count(), dtype=np.float32)
        _check(_lib().mu_seeder_get_params(self.h, out.ctypes.data), self.ctx.h, "mu_seeder_get_params")
        return out

    def grads(self):
        out = np.empty(param_count(), dtype=np.float32)
        _check(_lib().mu_seeder_get_grads(self.h, out.ctypes.data), self.ctx.h, "mu_seeder_get_grads")
        return out

    @property
    def steps(self):
        return int(_lib().mu_seeder_steps(self.h))

    def forward(self, x_bits):
        x = np.ascontiguousarray(np.asarray(x_bits, dtype=np.uint16))
        B = x.shape[0]
        y = np.empty((B, 8), dtype=np.float32)
        _check(_lib().mu_seeder_forward(self.ctx.h, self.h, x.ctypes.data, B, A.MU_MEM_HOST, y.ctypes.data),
               self.ctx.h, "mu_seeder_forward")
        return y

    def train_step(self, x_bits, targets, lr=1e-3, update=True):
        x = np.ascontiguousarray(np.asarray(x_bits, dtype=np.uint16))
        t = np.ascontiguousarray(np.asarray(targets, dtype=np.float32))
        loss = np.zeros(1, dtype=np.float32)
        _check(_lib().mu_seeder_train_step(self.ctx.h, self.h, x.ctypes.data, t.ctypes.data, x.shape[0], float(lr),
                                           1 if update else 0, A.MU_MEM_HOST, loss.ctypes.data),
               self.ctx.h, "mu_seeder_train_step")
        return float(loss[0])

    def layer(self, l, B, backward=False):
        """Buffers of layer l from the last pass: (BF16 input bits [B][K],
        FP32 pre-activation [B][N]) and, with backward, (FP32 dZ, BF16 dZ bits)."""
        K, N = DIMS[l], DIMS[l + 1]
        x = np.empty((B, K), dtype=np.uint16)
        z = np.empty((B, N), dtype=np.float32)
        dz = np.empty((B, N), dtype=np.float32) if backward else None
        g = np.empty((B, N), dtype=np.uint16) if backward else None
        _check(_lib().mu_seeder_layer(self.ctx.h, self.h, int(l), int(B), x.ctypes.data, z.ctypes.data,
                                      dz.ctypes.data if backward else None, g.ctypes.data if backward else None),
               self.ctx.h, "mu_seeder_layer")
        return (x, z, dz, g) if backward else (x, z)

    def train(self, seed, steps, batch=1024, lr=1e-3, lr_final_frac=0.05, first_sample=0):
        o = mu_seed_train_opts(int(seed), int(first_sample), int(batch), int(steps), float(lr), float(lr_final_frac))
        curve = np.empty(steps, dtype=np.float32)
        _check(_lib().mu_seeder_train(self.ctx.h, self.h, C.byref(o), curve.ctypes.data), self.ctx.h,
               "mu_seeder_train")
        return curve

    def infer(self, datas):
        n = len(datas)
        keep_d, dh = handle_array(datas)
        start = np.empty((n, 6))
        ok = np.empty(n, dtype=np.uint8)
        _check(_lib().mu_seed_infer(self.ctx.h, self.h, n, dh, start.ctypes.data, ok.ctypes.data), self.ctx.h,
               "mu_seed_infer")
        return start, ok.astype(bool)
