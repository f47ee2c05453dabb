"""FP64 CPU oracle of the warm-start network (test infrastructure only).

TEST INFRASTRUCTURE ONLY: imported by the tests, the smoke check and the
benchmark's CPU baseline; the product path never imports it and shares no code
with it.

The network maps the features (J, Delta, K, n / 64) of an ADAPT point at step
n to 64 initial angles (the converged angles of that step, padded): the paper
observes that the initial parameters matter (Sec. V.B, the discussion of random
initialisations) and suggests re-using information across runs (Appendix D,
Hessian recycling); the learned proposal is an addition to the method, on top
of the plain {theta_prev, 0} initialisation of Sec. IV.B.

Architecture 4 -> 128 -> 128 -> 64, SiLU on both hidden layers, linear output.
Precision contract shared with the device path (each step below is what the
device computes, here in float64):
  * inputs and weights are rounded to bfloat16 (round to nearest, ties to
    even); biases stay float32;
  * Z1 = X W1^T + b1, A1 = bf16(silu(Z1)); Z2 = A1 W2^T + b2,
    A2 = bf16(silu(Z2)); Y = A2 W3^T + b3 (not rounded);
  * loss = sum_b sum_{k < n_b} (Y[b,k] - T[b,k])^2 / sum_b n_b (masked MSE);
  * backward: G3 = bf16(2 M (Y - T) / N); dW3 = G3^T A2, db3 = sum_b G3;
    G2 = bf16((G3 W3) * silu'(Z2)); dW2 = G2^T A1, db2 = sum_b G2;
    G1 = bf16((G2 W2) * silu'(Z1)); dW1 = G1^T X, db1 = sum_b G1
    (the gradient with respect to the float32 master weights passes straight
    through the bfloat16 rounding);
  * Adam (Kingma & Ba 2015, Algorithm 1) on the float32 master parameters.

Parameter vector (float32, this order): W1 [128 x 4], b1 [128], W2 [128 x 128],
b2 [128], W3 [64 x 128], b3 [64]; W is [out x in], row-major.
"""
from __future__ import annotations

import numpy as np

N_IN, N_HID, N_OUT = 4, 128, 64
SHAPES = [("W1", (N_HID, N_IN)), ("b1", (N_HID,)), ("W2", (N_HID, N_HID)), ("b2", (N_HID,)),
          ("W3", (N_OUT, N_HID)), ("b3", (N_OUT,))]
N_PARAMS = sum(int(np.prod(s)) for _, s in SHAPES)


def unpack(params):
    """Split the flat parameter vector into named arrays (float64 copies)."""
    out, o = {}, 0
    p = np.asarray(params, dtype=np.float64)
    for name, shp in SHAPES:
        n = int(np.prod(shp))
        out[name] = p[o:o + n].reshape(shp)
        o += n
    return out


def pack(d):
    return np.concatenate([np.asarray(d[name], dtype=np.float64).ravel() for name, _ in SHAPES])


def bf16(x):
    """Round to the nearest bfloat16 value (ties to even), returned as float64.

    bfloat16 keeps the top 16 bits of the IEEE float32 encoding; values are
    first taken to float32 exactly when they are float32 already (weights,
    activations computed in float32 on the device).  From float64 the rounding
    is done on the float64 value directly: the nearest representable bfloat16
    (8 significant bits) with ties to even, by scaling to the unit in the last
    place of the value's binade."""
    x = np.asarray(x, dtype=np.float64)
    out = np.zeros_like(x)
    nz = (x != 0) & np.isfinite(x)
    m, e = np.frexp(x[nz])            # x = m 2^e, 0.5 <= |m| < 1
    e = np.maximum(e, -125)           # subnormal bfloat16 range keeps a fixed quantum
    q = np.ldexp(1.0, e - 8)          # spacing of bfloat16 values in this binade
    out[nz] = np.round(x[nz] / q) * q  # numpy rounds halves to even
    out[~nz] = x[~nz]
    return out


def silu(z):
    return z / (1.0 + np.exp(-z))


def dsilu(z):
    s = 1.0 / (1.0 + np.exp(-z))
    return s * (1.0 + z * (1.0 - s))


def forward(params, X, rounding=True):
    """Outputs Y [B x 64] and the saved values of the backward pass."""
    r = bf16 if rounding else (lambda a: np.asarray(a, dtype=np.float64))
    P = unpack(params)
    Xb = r(X)
    W1, W2, W3 = r(P["W1"]), r(P["W2"]), r(P["W3"])
    Z1 = Xb @ W1.T + P["b1"]
    A1 = r(silu(Z1))
    Z2 = A1 @ W2.T + P["b2"]
    A2 = r(silu(Z2))
    Y = A2 @ W3.T + P["b3"]
    return Y, dict(Xb=Xb, W1=W1, W2=W2, W3=W3, Z1=Z1, A1=A1, Z2=Z2, A2=A2)


def mask(nvalid, B):
    return (np.arange(N_OUT)[None, :] < np.asarray(nvalid)[:, None]).astype(np.float64).reshape(B, N_OUT)


def loss(params, X, T, nvalid, rounding=True):
    Y, _ = forward(params, X, rounding)
    M = mask(nvalid, len(X))
    return float(np.sum(M * (Y - T) ** 2) / np.sum(M))


def loss_and_grad(params, X, T, nvalid, rounding=True):
    """Masked-MSE loss and its gradient (flat, float64) by the backward pass
    of the module docstring."""
    r = bf16 if rounding else (lambda a: np.asarray(a, dtype=np.float64))
    Y, s = forward(params, X, rounding)
    M = mask(nvalid, len(X))
    N = np.sum(M)
    L = float(np.sum(M * (Y - T) ** 2) / N)
    G3 = r(2.0 * M * (Y - T) / N)
    g = {"W3": G3.T @ s["A2"], "b3": G3.sum(axis=0)}
    G2 = r((G3 @ s["W3"]) * dsilu(s["Z2"]))
    g["W2"], g["b2"] = G2.T @ s["A1"], G2.sum(axis=0)
    G1 = r((G2 @ s["W2"]) * dsilu(s["Z1"]))
    g["W1"], g["b1"] = G1.T @ s["Xb"], G1.sum(axis=0)
    return L, pack(g)


def adam_step(params, grad, m, v, t, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update (Kingma & Ba, Algorithm 1) at step t >= 1; returns the
    new (params, m, v)."""
    m = beta1 * m + (1.0 - beta1) * grad
    v = beta2 * v + (1.0 - beta2) * grad * grad
    mh = m / (1.0 - beta1 ** t)
    vh = v / (1.0 - beta2 ** t)
    return params - lr * mh / (np.sqrt(vh) + eps), m, v
