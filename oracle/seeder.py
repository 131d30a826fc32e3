"""Oracle of the learned seeder: histogram generator, network, loss, Adam,
target encoding and the default start (test infrastructure only).

The network maps a histogram of the exp*cos family, rebinned to 1024 bins and
turned into its asymmetry (counts less background over the lifetime decay,
minus one; network_input), to the hard-to-guess start parameters (A, lambda,
nu, phi); N0 and Nbkg come from the first and last bins.  It is a 1024-512-256-
128-8 multilayer perceptron with ReLU; GEMM operands are BF16 and sums are
kept wider.  Rounding points, in order (the GPU follows the same ones):

  forward, layer l:  Z = bf16(X) bf16(W)^T + b   (sums FP32 on the GPU, FP64 here)
                     H = relu(Z), next X = bf16(H); the last layer's Z is Y
  loss:              L = sum_b sum_o w_o (Y - T)^2 / B,  dY = 2 w_o (Y - T) / B
  backward, layer l: G = bf16(dZ);  dW = G^T bf16(X);  db = sum_b dZ
                     dX = G bf16(W);  dZ_prev = dX * (Z_prev > 0)
  Adam (FP32 master weights): m = b1 m + (1-b1) g, v = b2 v + (1-b2) g^2,
                     w -= lr (m / (1 - b1^t)) / (sqrt(v / (1 - b2^t)) + eps)

The generator draws each sample's parameters from Philox4x32-10 uniforms and
its expected counts over 8192 bins of 0.001 us summed in groups of 8; the
Poisson draws themselves are checked statistically (their exact decisions
depend on the last bits of transcendental functions).
"""

from __future__ import annotations

import math

import numpy as np

from . import model, philox

DIMS = (1024, 512, 256, 128, 8)
N_OUT_USED = 5                     # A, log lambda, log nu, cos phi, sin phi
LOSS_W = np.array([1, 1, 1, 1, 1, 0, 0, 0], dtype=np.float64)
RANGES = {"N0": (100.0, 1e5), "Nbkg": (1.0, 10.0), "A": (0.05, 0.3), "lambda": (0.05, 5.0),
          "nu": (0.1, 50.0), "phi": (0.0, 2 * math.pi)}
N_FINE, DT_FINE, REBIN = 8192, 0.001, 8
N_COARSE = N_FINE // REBIN
THETA_TAG = 0xFFFFFFFF            # Philox counter word 2 of the parameter draws


# ----------------------------------------------------------------- BF16

def bf16(x):
    """Round to the nearest BF16 value (ties to even), returned as float32."""
    a = np.ascontiguousarray(np.asarray(x, dtype=np.float32))
    u = a.view(np.uint32).astype(np.uint64)
    lsb = (u >> np.uint64(16)) & np.uint64(1)
    r = ((u + np.uint64(0x7FFF) + lsb) >> np.uint64(16)) << np.uint64(16)
    out = (r & np.uint64(0xFFFFFFFF)).astype(np.uint32).view(np.float32)
    nan = np.isnan(a)
    if np.any(nan):
        out = out.copy()
        out[nan] = np.float32(np.nan)
    return out


def bf16_bits(x):
    """BF16 bit patterns (uint16) of bf16(x)."""
    return (bf16(x).view(np.uint32) >> np.uint32(16)).astype(np.uint16)


def from_bf16_bits(b):
    return (np.asarray(b, dtype=np.uint32) << np.uint32(16)).view(np.float32)


# ----------------------------------------------------------------- network

def init_params(seed):
    """He-uniform weights (last layer scaled by 0.1) and zero biases, from
    numpy's PCG64 (the initial values are an input, not part of the check)."""
    rng = np.random.default_rng(seed)
    Ws, bs = [], []
    for l in range(len(DIMS) - 1):
        k, n = DIMS[l], DIMS[l + 1]
        bound = math.sqrt(6.0 / k) * (0.1 if l == len(DIMS) - 2 else 1.0)
        Ws.append(rng.uniform(-bound, bound, size=(n, k)).astype(np.float32))
        bs.append(np.zeros(n, dtype=np.float32))
    return Ws, bs


def forward(Ws, bs, X, rounding=True):
    """Returns Y (float64) and the cache for backward."""
    rd = bf16 if rounding else (lambda a: np.asarray(a, dtype=np.float64))
    Xl = np.asarray(rd(X), dtype=np.float64)
    cache = []
    L = len(Ws)
    for l in range(L):
        Wl = np.asarray(rd(Ws[l]), dtype=np.float64)
        Z = Xl @ Wl.T + np.asarray(bs[l], dtype=np.float64)
        cache.append((Xl, Wl, Z))
        if l < L - 1:
            Xl = np.asarray(rd(np.maximum(Z, 0.0)), dtype=np.float64)
    return Z, cache


def loss_and_grad(Y, T):
    """Weighted mean squared error over the batch and dL/dY."""
    B = Y.shape[0]
    D = Y - np.asarray(T, dtype=np.float64)
    loss = float(np.sum(LOSS_W[None, :] * D * D) / B)
    return loss, 2.0 * LOSS_W[None, :] * D / B


def backward(cache, dY, rounding=True):
    """Gradients (dW list, db list) following the rounding points above."""
    rd = bf16 if rounding else (lambda a: np.asarray(a, dtype=np.float64))
    L = len(cache)
    dWs, dbs = [None] * L, [None] * L
    dZ = np.asarray(dY, dtype=np.float64)
    for l in range(L - 1, -1, -1):
        Xl, Wl, Z = cache[l]
        G = np.asarray(rd(dZ), dtype=np.float64)
        dWs[l] = G.T @ Xl
        dbs[l] = dZ.sum(axis=0)
        if l > 0:
            dX = G @ Wl
            dZ = dX * (cache[l - 1][2] > 0.0)
    return dWs, dbs


def adam(params, grads, m, v, t, lr, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam step (in place on float64 copies); t counts from 1."""
    out = []
    for p, g, mm, vv in zip(params, grads, m, v):
        mm[...] = b1 * mm + (1 - b1) * g
        vv[...] = b2 * vv + (1 - b2) * g * g
        mh = mm / (1 - b1 ** t)
        vh = vv / (1 - b2 ** t)
        out.append(p - lr * mh / (np.sqrt(vh) + eps))
    return out


# ----------------------------------------------------------------- targets

def encode(theta):
    """Network targets of parameter rows [N0, Nbkg, A, lambda, nu, phi]."""
    th = np.atleast_2d(np.asarray(theta, dtype=np.float64))
    T = np.zeros((th.shape[0], DIMS[-1]))
    T[:, 0] = th[:, 2] / 0.3
    T[:, 1] = (np.log(th[:, 3]) - math.log(0.05)) / math.log(100.0)
    T[:, 2] = (np.log(th[:, 4]) - math.log(0.1)) / math.log(500.0)
    T[:, 3] = np.cos(th[:, 5])
    T[:, 4] = np.sin(th[:, 5])
    return T


TAU_MU = 2.1969811
WIN = 32  # rebinned bins in each estimation window (256 bins of 0.001 us)


def window_estimates(counts_coarse, tau=TAU_MU):
    """N0 and Nbkg (per 0.001 us bin) from the means of the first and last 256
    fine bins: two equations m = N0 e + Nbkg with e the lifetime decay averaged
    over each window (geometric sums)."""
    c = np.asarray(counts_coarse, dtype=np.float64)
    m1 = c[:WIN].sum() / (WIN * REBIN)
    m2 = c[-WIN:].sum() / (WIN * REBIN)
    r = math.exp(-DT_FINE / tau)
    w = WIN * REBIN
    e1 = (1.0 - r ** w) / (w * (1.0 - r))
    e2 = e1 * r ** (N_FINE - w)
    n0 = (m1 - m2) / (e1 - e2)
    nb = max(m2 - n0 * e2, 0.1)
    n0 = max(n0, 1.0)
    return n0, nb


def network_input(counts_coarse, tau=TAU_MU):
    """The network's view of a rebinned histogram: the asymmetry
    (c_b - 8 Nbkg) / (8 N0 ebar_b) - 1, with ebar_b the lifetime decay averaged
    over rebinned bin b and N0, Nbkg from window_estimates; clipped to [-4, 4]."""
    c = np.asarray(counts_coarse, dtype=np.float64)
    n0, nb = window_estimates(c, tau)
    r = math.exp(-DT_FINE / tau)
    b = np.arange(N_COARSE, dtype=np.float64)
    ebar = np.exp(-(REBIN * DT_FINE / tau) * b) * ((1.0 - r ** REBIN) / (REBIN * (1.0 - r)))
    x = (c - REBIN * nb) / (REBIN * n0 * ebar) - 1.0
    return np.clip(x, -4.0, 4.0)


def default_start(counts_fine, tau=TAU_MU):
    """The non-learned start: N0 and Nbkg from window_estimates, A = 0.175,
    lambda = 0.5 /us, nu = sqrt(5) MHz (geometric midpoints of the ranges),
    phi = 0."""
    coarse = np.asarray(counts_fine, dtype=np.float64).reshape(N_COARSE, REBIN).sum(axis=1)
    n0, nb = window_estimates(coarse, tau)
    return np.array([n0, nb, 0.175, 0.5, math.sqrt(5.0), 0.0])


def decode(Y, counts_fine):
    """Start vector and validity from the network output of one histogram:
    A, lambda, nu, phi from the outputs, N0 and Nbkg from default_start.
    Valid when every decoded value is finite and inside a margin around the
    training ranges (A in [0.01, 1], lambda in [0.005, 50], nu in [0.02, 250])."""
    y = np.asarray(Y, dtype=np.float64)
    s = default_start(counts_fine)
    A = 0.3 * y[0]
    lam = 0.05 * math.exp(y[1] * math.log(100.0)) if np.isfinite(y[1]) else math.nan
    nu = 0.1 * math.exp(y[2] * math.log(500.0)) if np.isfinite(y[2]) else math.nan
    phi = math.atan2(y[4], y[3])
    ok = (np.all(np.isfinite(y[:5])) and 0.01 <= A <= 1.0 and 0.005 <= lam <= 50.0 and 0.02 <= nu <= 250.0)
    if not ok:
        return s, False
    return np.array([s[0], s[1], A, lam, nu, phi]), True


# ----------------------------------------------------------------- generator

def draw_theta(seed, index):
    """Parameters of sample `index` from Philox4x32-10 with key (seed lo, seed
    hi), counters (index lo, index hi, THETA_TAG, 0 and 1)."""
    idx = np.atleast_1d(np.asarray(index, dtype=np.uint64))
    key = np.array([seed & 0xFFFFFFFF, (seed >> 32) & 0xFFFFFFFF], dtype=np.uint32)
    out = []
    for c3 in (0, 1):
        ctr = np.stack([(idx & np.uint64(0xFFFFFFFF)).astype(np.uint32),
                        (idx >> np.uint64(32)).astype(np.uint32),
                        np.full(idx.size, THETA_TAG, np.uint32),
                        np.full(idx.size, c3, np.uint32)], axis=-1)
        out.append(philox.u01(philox.philox4x32_10(ctr, key)))
    u = np.concatenate(out, axis=-1)  # [n, 8]; the first six are used

    def logu(v, lo, hi):
        return np.exp(math.log(lo) + v * (math.log(hi) - math.log(lo)))

    th = np.stack([logu(u[:, 0], *RANGES["N0"]),
                   RANGES["Nbkg"][0] + u[:, 1] * (RANGES["Nbkg"][1] - RANGES["Nbkg"][0]),
                   RANGES["A"][0] + u[:, 2] * (RANGES["A"][1] - RANGES["A"][0]),
                   logu(u[:, 3], *RANGES["lambda"]),
                   logu(u[:, 4], *RANGES["nu"]),
                   u[:, 5] * RANGES["phi"][1]], axis=-1)
    return th


def expected_coarse(theta_row, theory):
    """Expected counts of the 1024 rebinned bins: the model over 8192 bins of
    0.001 us (Eq. 1 with the exp*cos theory), summed in groups of 8."""
    h = {"n_bins": N_FINE, "dt": DT_FINE, "t0_bin": 0.0, "first": 0, "last": N_FINE - 1, "map_row": 0}
    fine = model.model(theory, h, np.asarray(theta_row, dtype=np.float64))
    return fine.reshape(N_COARSE, REBIN).sum(axis=1)


