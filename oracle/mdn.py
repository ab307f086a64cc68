"""FP64 reference of the learned proposal's network (numpy).  TEST
INFRASTRUCTURE ONLY, like the rest of `oracle/`.

A mixture-density network: 576 features -> three GELU layers of 256 -> 56
outputs = 8 components x (logit, mean x, y, t, log sd x, y, t), log sds
clamped per axis; loss = mean negative log-likelihood of the target under
the mixture of untruncated Gaussians.  With ``bf16=True`` the reference
rounds to BF16 exactly where the GPU stores BF16 (features, weight copies,
hidden activations, the loss gradient and the backpropagated GELU
gradients) and otherwise computes in FP64; with ``bf16=False`` it is plain
FP64 throughout (pinned by finite differences).
"""
from __future__ import annotations

import ctypes as C

import numpy as np
from scipy.special import erf

from . import EVENT_DTYPE, Model, _ptr, lib  # noqa: F401

N_IN, N_HID, N_K, N_OUT_PAD = 576, 256, 8, 64
SLO = np.array([np.log(0.025), np.log(0.025), np.log(0.5 / 32)])
SHI = np.array([np.log(1.5), np.log(1.5), 0.0])
LAYERS = [(N_IN, N_HID), (N_HID, N_HID), (N_HID, N_HID), (N_HID, N_OUT_PAD)]


def to_f32(x):
    return np.asarray(x, dtype=np.float32).astype(np.float64)


def to_bf16(x) -> np.ndarray:
    """Round to BF16 (round to nearest, ties to even) through binary32."""
    f = np.ascontiguousarray(np.asarray(x, dtype=np.float32))
    u = f.view(np.uint32).astype(np.uint64)
    r = ((u + 0x7FFF + ((u >> 16) & 1)) >> 16) << 16
    return r.astype(np.uint32).view(np.float32).astype(np.float64)


def param_layout():
    """(name, shape, offset) of the flat FP32 parameter vector."""
    out, o = [], 0
    for l, (fi, fo) in enumerate(LAYERS):
        out.append((f"W{l + 1}", (fo, fi), o))
        o += fi * fo
        out.append((f"b{l + 1}", (fo,), o))
        o += fo
    return out, o


def unflatten(flat: np.ndarray) -> dict:
    lay, n = param_layout()
    assert flat.size == n
    return {name: np.asarray(flat[o:o + int(np.prod(sh))], dtype=np.float64).reshape(sh)
            for name, sh, o in lay}


def flatten(P: dict) -> np.ndarray:
    lay, n = param_layout()
    out = np.zeros(n)
    for name, sh, o in lay:
        out[o:o + int(np.prod(sh))] = P[name].ravel()
    return out


def gelu(z):
    return 0.5 * z * (1.0 + erf(z / np.sqrt(2.0)))


def gelu_grad(z):
    return 0.5 * (1.0 + erf(z / np.sqrt(2.0))) + z * np.exp(-0.5 * z * z) / np.sqrt(2.0 * np.pi)


def forward(P: dict, X: np.ndarray, bf16: bool = True):
    r = to_bf16 if bf16 else (lambda v: np.asarray(v, dtype=np.float64))
    W = [r(P[f"W{l + 1}"]) for l in range(4)]
    a = r(X)
    Zs, As = [], [a]
    for l in range(3):
        z = a @ W[l].T + P[f"b{l + 1}"]
        Zs.append(z)
        a = r(gelu(z))
        As.append(a)
    o = a @ W[3].T + P["b4"]
    return o, Zs, As, W


def mixture_nll(o: np.ndarray, z: np.ndarray):
    """Per-row loss and d loss / d output (not yet divided by the batch)."""
    M = o.shape[0]
    K = N_K
    logit = o[:, 0:7 * K:7]
    mu = np.stack([o[:, 1 + d:7 * K:7] for d in range(3)], axis=-1)      # M x K x 3
    sraw = np.stack([o[:, 4 + d:7 * K:7] for d in range(3)], axis=-1)
    s = np.clip(sraw, SLO, SHI)
    lse = np.log(np.sum(np.exp(logit - logit.max(1, keepdims=True)), 1)) + logit.max(1)
    u = (z[:, None, :] - mu) * np.exp(-s)
    ell = (logit - lse[:, None]) + np.sum(-0.5 * u * u - s - 0.5 * np.log(2 * np.pi), axis=-1)
    best = ell.max(1)
    logp = best + np.log(np.sum(np.exp(ell - best[:, None]), 1))
    gam = np.exp(ell - logp[:, None])
    pik = np.exp(logit - lse[:, None])
    g = np.zeros((M, N_OUT_PAD))
    g[:, 0:7 * K:7] = pik - gam
    free = (sraw > SLO) & (sraw < SHI)
    for d in range(3):
        g[:, 1 + d:7 * K:7] = -gam * u[..., d] * np.exp(-s[..., d])
        g[:, 4 + d:7 * K:7] = np.where(free[..., d], -gam * (u[..., d] ** 2 - 1.0), 0.0)
    return -logp, g


def loss_and_grads(P: dict, X: np.ndarray, Z: np.ndarray, bf16: bool = True,
                   parts: bool = False):
    """Mean loss and gradients of every parameter (dict like P).  parts:
    also the operands of each weight gradient, {layer: (output gradient,
    input activation)}, so that a test can bound a BF16 implementation's
    error element by element."""
    r = to_bf16 if bf16 else (lambda v: np.asarray(v, dtype=np.float64))
    o, Zs, As, W = forward(P, X, bf16)
    M = X.shape[0]
    per_row, g = mixture_nll(o, Z)
    dO = r(g / M)
    G = {"W4": dO.T @ As[3], "b4": dO.sum(0)}
    ops = {4: (dO, As[3])}
    dnext = dO
    for l in (2, 1, 0):
        dA = dnext @ W[l + 1]
        dH = r(dA * gelu_grad(Zs[l]))
        G[f"W{l + 1}"] = dH.T @ As[l]
        G[f"b{l + 1}"] = dH.sum(0)
        ops[l + 1] = (dH, As[l])
        dnext = dH
    if parts:
        return float(per_row.mean()), per_row, G, ops
    return float(per_row.mean()), per_row, G


MU_XY, MU_T_LO, MU_T_HI = 2.0, -1.0, 3.0


def mixture_table(o: np.ndarray, nsx: int, ds: float, n_tau: int, first: int = 0) -> np.ndarray:
    """Mixture table of anchors first .. first + rows - 1 (anchor a: station
    a // n_tau in row-major order, window start 32 (a % n_tau)) from head
    outputs: [rows][8][8] = (mean x, y, t, sd x, y, t, log weight,
    cumulative weight) in absolute units, means clamped to +-2 spacings of
    the station and to [tau - 32, tau + 96], log sds to the training clamps."""
    o = np.asarray(o, dtype=np.float64)
    rows = o.shape[0]
    a = first + np.arange(rows)
    c = a // n_tau
    sx = ((c % nsx) + 0.5) * ds
    sy = ((c // nsx) + 0.5) * ds
    tau = 32.0 * (a % n_tau)
    K = N_K
    logit = o[:, 0:7 * K:7]
    lmax = logit.max(1, keepdims=True)
    lse = lmax[:, 0] + np.log(np.sum(np.exp(logit - lmax), 1))
    T = np.zeros((rows, K, 8))
    T[..., 0] = sx[:, None] + ds * np.clip(o[:, 1:7 * K:7], -MU_XY, MU_XY)
    T[..., 1] = sy[:, None] + ds * np.clip(o[:, 2:7 * K:7], -MU_XY, MU_XY)
    T[..., 2] = tau[:, None] + 32.0 * np.clip(o[:, 3:7 * K:7], MU_T_LO, MU_T_HI)
    scale = (ds, ds, 32.0)
    for d in range(3):
        T[..., 3 + d] = scale[d] * np.exp(np.clip(o[:, 4 + d:7 * K:7], SLO[d], SHI[d]))
    T[..., 6] = logit - lse[:, None]
    cum = np.zeros(rows)
    for k in range(K):                 # sequential running sum, as specified
        cum = cum + np.exp(T[:, k, 6])
        T[:, k, 7] = cum
    return T


# ------------------------------------------------------------- features

def pair(model: Model, seed: int, p: int):
    L = lib()
    L.orc_mdn_pair.argtypes = [C.c_void_p, C.c_uint32, C.c_int64, C.c_void_p, C.c_void_p]
    f = np.zeros(N_IN)
    t = np.zeros(3)
    L.orc_mdn_pair(C.byref(model), seed, p, _ptr(f), _ptr(t))
    return f, t


def pairs(model: Model, seed: int, first: int, count: int):
    F = np.zeros((count, N_IN))
    T = np.zeros((count, 3))
    for q in range(count):
        F[q], T[q] = pair(model, seed, first + q)
    return F, T


def anchor_features(model: Model, s: np.ndarray, n_tau: int, a: int) -> np.ndarray:
    L = lib()
    L.orc_anchor_features.argtypes = [C.c_void_p, C.c_void_p, C.c_int32, C.c_int32, C.c_void_p]
    f = np.zeros(N_IN)
    s = np.ascontiguousarray(s, dtype=np.float64)
    L.orc_anchor_features(C.byref(model), _ptr(s), n_tau, a, _ptr(f))
    return f


def anchor_weight(feat_rounded: np.ndarray) -> float:
    return 1e-3 + float(np.mean(np.maximum(0.0, feat_rounded - 1.0)))
