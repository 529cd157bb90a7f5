"""FP64 reference of the optimiser steps of the joint optimisation of
Gaussian parameters and camera poses (Sec. IV-D; the paper refines poses with
Levenberg-Marquardt, the library takes first-order steps on the same
gradients and retracts the pose twist onto SE(3)).

TEST INFRASTRUCTURE ONLY (see the package docstring).

adam_step: Adam (Kingma and Ba 2015) with bias correction.
se3_exp:   the SE(3) exponential of a twist xi = (rho, phi), translation first:
           R = I + sin(t)/t [phi]x + (1 - cos t)/t^2 [phi]x^2,
           V = I + (1 - cos t)/t^2 [phi]x + (t - sin t)/t^3 [phi]x^2, p = V rho,
           t = |phi| (series below t = 1e-4).
pose_update: left retraction T <- Exp(xi) T of a world -> camera pose.

Pinned by tests/test_oracle_optim.py: Adam's first step from zero state and
its constant-gradient steps have closed forms; se3_exp agrees with the matrix
exponential of the 4x4 generator (scipy.linalg.expm) and with Rodrigues'
rotation from scipy.spatial.transform; Exp(xi) Exp(-xi) = I.
"""

from __future__ import annotations

import numpy as np


def adam_step(p, g, m, v, lr, step, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam step in float64; returns (p, m, v)."""
    p, g, m, v = (np.asarray(a, np.float64) for a in (p, g, m, v))
    m = beta1 * m + (1.0 - beta1) * g
    v = beta2 * v + (1.0 - beta2) * g * g
    mh = m / (1.0 - beta1 ** step)
    vh = v / (1.0 - beta2 ** step)
    return p - lr * mh / (np.sqrt(vh) + eps), m, v


def hat(phi):
    x, y, z = phi
    return np.array([[0.0, -z, y], [z, 0.0, -x], [-y, x, 0.0]])


def se3_exp(xi):
    """4x4 homogeneous matrix Exp(xi), xi = (rho, phi)."""
    xi = np.asarray(xi, np.float64)
    rho, phi = xi[:3], xi[3:]
    t2 = float(phi @ phi)
    t = np.sqrt(t2)
    if t < 1e-4:
        A, B, C = 1.0 - t2 / 6.0, 0.5 - t2 / 24.0, 1.0 / 6.0 - t2 / 120.0
    else:
        A, B, C = np.sin(t) / t, (1.0 - np.cos(t)) / t2, (t - np.sin(t)) / (t2 * t)
    K = hat(phi)
    K2 = K @ K
    R = np.eye(3) + A * K + B * K2
    V = np.eye(3) + B * K + C * K2
    out = np.eye(4)
    out[:3, :3] = R
    out[:3, 3] = V @ rho
    return out


def pose_update(T_cw, xi):
    """3x4 world -> camera pose Exp(xi) T_cw."""
    T = np.eye(4)
    T[:3, :] = np.asarray(T_cw, np.float64).reshape(3, 4)
    return (se3_exp(xi) @ T)[:3, :]
