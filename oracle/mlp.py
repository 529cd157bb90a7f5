"""FP64 reference of the learned per-pixel MP surrogate (not part of the paper).

TEST INFRASTRUCTURE ONLY (see the package docstring).

A small per-pixel network stands in for the geometric MP cue of Eq. (5)-(7):
x in R^8 -> 32 -> 32 (ReLU) -> 1 (sigmoid). Weights are used as bfloat16
copies of float32 masters (round to nearest even); biases, activations and
accumulation are wider. The oracle evaluates everything in float64 on exactly
the bfloat16-rounded weight values.

Features (per pixel u), each scaled by a fixed constant:
  x0..2 = C(u) - C_gt(u)                      (colour residual)
  x3    = (D(u) - D_gt(u)) [D_gt > 0] / 0.1 m  (depth residual)
  x4    = M(u)                                (rendered MP channel)
  x5    = T(u)                                (final transmittance)
  x6    = D(u) / 4 m                          (rendered depth)
  x7    = MP_ins(u)                           (instance prior, Eq. (2))

Loss: mean binary cross-entropy against the plain method's M_p. Gradients are
taken with respect to the weights as used (the bfloat16 values) and applied to
the float32 masters (straight-through), followed by an Adam step.

Pinned by tests/test_oracle_mlp.py: zero weights give y = 0.5; a single hidden
path has a closed form; gradients agree with central finite differences; the
bfloat16 rounding agrees with torch's float32 -> bfloat16 conversion.
"""

from __future__ import annotations

import numpy as np

DEPTH_SCALE = 4.0
RESID_SCALE = 0.1
HIDDEN = 32
N_IN = 8
PARAM_NAMES = ("W1", "b1", "W2", "b2", "W3", "b3")


def bf16_round(a):
    """Round float32 values to the nearest bfloat16 (ties to even), returned as
    float32: add 0x7FFF plus the lowest kept bit to the bit pattern, truncate."""
    a = np.ascontiguousarray(a, np.float32)
    u = a.view(np.uint32).astype(np.uint64)
    bias = 0x7FFF + ((u >> 16) & 1)
    r = ((u + bias) & 0xFFFF0000).astype(np.uint32)
    return r.view(np.float32)


def features(color, depth, mpc, T, target_color, target_depth, mp_ins):
    Cd = np.asarray(color, np.float64) - np.asarray(target_color, np.float64)
    Dg = np.asarray(target_depth, np.float64)
    dres = np.where(Dg > 0, np.asarray(depth, np.float64) - Dg, 0.0) / RESID_SCALE
    return np.stack([Cd[0], Cd[1], Cd[2], dres, np.asarray(mpc, np.float64), np.asarray(T, np.float64),
                     np.asarray(depth, np.float64) / DEPTH_SCALE, np.asarray(mp_ins, np.float64)])


def used_weights(params):
    """Weights as the network uses them: bfloat16-rounded W, float32 biases."""
    out = {}
    for k in PARAM_NAMES:
        v = np.asarray(params[k], np.float32)
        out[k] = (bf16_round(v) if k.startswith("W") else v).astype(np.float64)
    return out


def forward(params, x):
    w = used_weights(params)
    x = np.asarray(x, np.float64)
    z1 = w["W1"] @ x + w["b1"][:, None]
    h1 = np.maximum(z1, 0)
    z2 = w["W2"] @ h1 + w["b2"][:, None]
    h2 = np.maximum(z2, 0)
    z3 = w["W3"] @ h2 + w["b3"][:, None]
    y = 1.0 / (1.0 + np.exp(-z3[0]))
    return y, dict(z1=z1, h1=h1, z2=z2, h2=h2, z3=z3, w=w, x=x)


def bce(y, label, eps=1e-7):
    y = np.clip(y, eps, 1 - eps)
    t = np.asarray(label, np.float64)
    return float(np.mean(-(t * np.log(y) + (1 - t) * np.log(1 - y))))


def loss_and_grads(params, x, label):
    """Mean BCE over pixels and its gradient w.r.t. each parameter. The sigmoid
    and BCE combine to dL/dz3 = (y - t) / P."""
    y, c = forward(params, x)
    P = y.shape[0]
    t = np.asarray(label, np.float64)
    L = bce(y, t)
    dz3 = ((y - t) / P)[None, :]
    w = c["w"]
    g = {}
    g["W3"] = dz3 @ c["h2"].T
    g["b3"] = dz3.sum(axis=1)
    dh2 = w["W3"].T @ dz3
    dz2 = dh2 * (c["z2"] > 0)
    g["W2"] = dz2 @ c["h1"].T
    g["b2"] = dz2.sum(axis=1)
    dh1 = w["W2"].T @ dz2
    dz1 = dh1 * (c["z1"] > 0)
    g["W1"] = dz1 @ c["x"].T
    g["b1"] = dz1.sum(axis=1)
    return L, g, y


def adam_step(params, grads, m, v, step, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """Adam (Kingma & Ba) with bias correction; `step` is the 1-based count
    after this update. Returns new (params, m, v) in float64."""
    newp, newm, newv = {}, {}, {}
    b1c = 1.0 - beta1 ** step
    b2c = 1.0 - beta2 ** step
    for k in PARAM_NAMES:
        gk = np.asarray(grads[k], np.float64)
        mk = beta1 * np.asarray(m[k], np.float64) + (1 - beta1) * gk
        vk = beta2 * np.asarray(v[k], np.float64) + (1 - beta2) * gk * gk
        newm[k], newv[k] = mk, vk
        newp[k] = np.asarray(params[k], np.float64) - lr * (mk / b1c) / (np.sqrt(vk / b2c) + eps)
    return newp, newm, newv
