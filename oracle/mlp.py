"""FP64 reference of the learned eigencomponent-weight network (TEST INFRASTRUCTURE).

Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may use this module. The network replaces a threshold rule of the
Adaptive Thresholding Methods section (Eqs 6 and 9) by a learned map from a
subset's spectrum to soft weights diag(w) for the projection of Eq. 4:

  features  z_i = log10(max(lambda_i, lambda_1 2^-52) / lambda_1) / 8,  i = 1..128
  layer 1   a1 = GELU(W1 z + b1)            W1: 256 x 128
  layer 2   a2 = GELU(W2 a1 + b2)           W2: 256 x 256
  layer 3   w  = sigmoid(W3 a2 + b3)        W3: 128 x 256
  GELU(h) = h * Phi(h) with the normal CDF Phi (erf form).

Loss of one spectrum: sum_i c_i (w_i - t_i)^2 with c_i = lambda_i / sum_j lambda_j t_j^2
(the relative change of the filtered energy sum_i w_i^2 lambda_i, to first order),
averaged over the batch. The forward runs on BF16-rounded weights in FP64
arithmetic, as the GPU kernels do with FP32 accumulation.
"""
from __future__ import annotations

import math

import numpy as np
from scipy.special import erf

NT = 128
H = 256
SHAPES = {"W1": (H, NT), "b1": (H,), "W2": (H, H), "b2": (H,), "W3": (NT, H), "b3": (NT,)}
NPARAM = sum(int(np.prod(s)) for s in SHAPES.values())      # 131712
FEATURE_SCALE = 1.0 / 8.0
FLOOR = 2.0 ** -52


def bf16_round(x: np.ndarray) -> np.ndarray:
    """Round float32 values to the nearest bfloat16 (ties to even), returned as float64."""
    u = np.asarray(x, dtype=np.float32).view(np.uint32).astype(np.uint64)
    r = ((u + 0x7FFF + ((u >> 16) & 1)) >> 16) << 16
    return r.astype(np.uint32).view(np.float32).astype(np.float64)


def features(lam: np.ndarray) -> np.ndarray:
    """Normalised log-spectrum of sorted eigenvalues (rows of lam, descending)."""
    lam = np.atleast_2d(np.asarray(lam, dtype=np.float64))
    l1 = lam[:, :1]
    return np.log10(np.maximum(lam, l1 * FLOOR) / l1) * FEATURE_SCALE


def gelu(h):
    return 0.5 * h * (1.0 + erf(h / math.sqrt(2.0)))


def gelu_grad(h):
    return 0.5 * (1.0 + erf(h / math.sqrt(2.0))) + h * np.exp(-0.5 * h * h) / math.sqrt(2.0 * math.pi)


def init_params(seed: int = 0) -> dict:
    """He-style uniform init in FP32 (the master copy)."""
    rng = np.random.default_rng(seed)
    p = {}
    for name, shp in SHAPES.items():
        if name.startswith("W"):
            bound = math.sqrt(6.0 / shp[1]) * 0.5
            p[name] = rng.uniform(-bound, bound, size=shp).astype(np.float32)
        else:
            p[name] = np.zeros(shp, dtype=np.float32)
    p["b3"][:] = 2.0
    return p


def forward(params: dict, z: np.ndarray, bf16: bool = True):
    """Forward pass on a batch z [B][128]; returns (w, cache)."""
    q = {k: (bf16_round(v) if bf16 and k.startswith("W") else np.asarray(v, dtype=np.float64))
         for k, v in params.items()}
    h1 = z @ q["W1"].T + q["b1"]
    a1 = gelu(h1)
    h2 = a1 @ q["W2"].T + q["b2"]
    a2 = gelu(h2)
    h3 = a2 @ q["W3"].T + q["b3"]
    w = 1.0 / (1.0 + np.exp(-h3))
    return w, dict(z=z, h1=h1, a1=a1, h2=h2, a2=a2, h3=h3, w=w, q=q)


def loss_weights(lam: np.ndarray, target: np.ndarray) -> np.ndarray:
    lam = np.atleast_2d(lam)
    e = np.sum(lam * target * target, axis=1, keepdims=True)
    return lam / np.where(e > 0, e, 1.0)


def loss(w: np.ndarray, target: np.ndarray, c: np.ndarray) -> float:
    return float(np.mean(np.sum(c * (w - target) ** 2, axis=1)))


def backward(cache: dict, target: np.ndarray, c: np.ndarray) -> dict:
    """Gradients of the batch-mean loss w.r.t. the (BF16-rounded) weights and biases."""
    b = target.shape[0]
    w, q = cache["w"], cache["q"]
    dw = 2.0 * c * (w - target) / b
    d3 = dw * w * (1.0 - w)
    g = {"W3": d3.T @ cache["a2"], "b3": d3.sum(0)}
    da2 = d3 @ q["W3"]
    d2 = da2 * gelu_grad(cache["h2"])
    g["W2"] = d2.T @ cache["a1"]
    g["b2"] = d2.sum(0)
    da1 = d2 @ q["W2"]
    d1 = da1 * gelu_grad(cache["h1"])
    g["W1"] = d1.T @ cache["z"]
    g["b1"] = d1.sum(0)
    return g


def adam_step(params: dict, grads: dict, m: dict, v: dict, step: int, lr: float,
              beta1: float = 0.9, beta2: float = 0.999, eps: float = 1e-8) -> None:
    """One Adam update of the FP32 master parameters (in place)."""
    for k in params:
        m[k] = beta1 * m[k] + (1 - beta1) * grads[k]
        v[k] = beta2 * v[k] + (1 - beta2) * grads[k] ** 2
        mh = m[k] / (1 - beta1 ** step)
        vh = v[k] / (1 - beta2 ** step)
        params[k] = (params[k] - lr * mh / (np.sqrt(vh) + eps)).astype(np.float32)


def flatten(params: dict) -> np.ndarray:
    return np.concatenate([np.asarray(params[k], dtype=np.float32).reshape(-1) for k in SHAPES])


def unflatten(vec: np.ndarray) -> dict:
    out, o = {}, 0
    for k, s in SHAPES.items():
        n = int(np.prod(s))
        out[k] = np.asarray(vec[o:o + n], dtype=np.float32).reshape(s)
        o += n
    return out
