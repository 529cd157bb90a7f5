"""Pins of the optimiser-step oracle (oracle/optim.py)."""

import numpy as np
import scipy.linalg
from scipy.spatial.transform import Rotation

from oracle import optim


def test_adam_first_step_closed_form():
    """From zero moments the bias-corrected first step is -lr g / (|g| + eps)."""
    rng = np.random.default_rng(0)
    g = rng.normal(size=100) * np.logspace(-6, 2, 100)
    p = rng.normal(size=100)
    p1, m, v = optim.adam_step(p, g, np.zeros(100), np.zeros(100), lr=0.01, step=1)
    np.testing.assert_allclose(p1 - p, -0.01 * g / (np.abs(g) + 1e-8), rtol=1e-12, atol=1e-15)
    np.testing.assert_allclose(m, 0.1 * g, rtol=1e-15)
    np.testing.assert_allclose(v, 0.001 * g * g, rtol=1e-12)


def test_adam_constant_gradient():
    """With a constant gradient the corrected moments equal g and g^2 at every
    step, so every step is the same; a zero gradient leaves the parameter."""
    g = np.array([3.0, -0.5, 1e-3])
    p = np.zeros(3)
    m = np.zeros(3)
    v = np.zeros(3)
    for k in range(1, 6):
        p_new, m, v = optim.adam_step(p, g, m, v, lr=0.1, step=k)
        np.testing.assert_allclose(p_new - p, -0.1 * g / (np.abs(g) + 1e-8), rtol=1e-9)
        p = p_new
    p2, _, _ = optim.adam_step(p, np.zeros(3), m, v, lr=0.1, step=6)
    np.testing.assert_allclose(p2, p - 0.1 * (0.9 * m / (1 - 0.9 ** 6)) / (np.sqrt(0.999 * v / (1 - 0.999 ** 6)) + 1e-8))
    assert np.all(np.abs(p2 - p) < np.abs(0.1 * np.ones(3)))


def _generator(xi):
    G = np.zeros((4, 4))
    G[:3, :3] = optim.hat(xi[3:])
    G[:3, 3] = xi[:3]
    return G


def test_se3_exp_matches_matrix_exponential():
    rng = np.random.default_rng(1)
    for scale in (0.0, 1e-7, 1e-5, 1e-3, 0.1, 1.0, 2.5):
        for _ in range(5):
            xi = rng.normal(size=6) * scale
            np.testing.assert_allclose(optim.se3_exp(xi), scipy.linalg.expm(_generator(xi)), atol=1e-12)


def test_se3_exp_special_cases():
    rng = np.random.default_rng(2)
    rho = rng.normal(size=3)
    T = optim.se3_exp(np.concatenate([rho, np.zeros(3)]))
    np.testing.assert_allclose(T[:3, :3], np.eye(3), atol=1e-15)
    np.testing.assert_allclose(T[:3, 3], rho, atol=1e-15)
    phi = rng.normal(size=3)
    R = optim.se3_exp(np.concatenate([np.zeros(3), phi]))[:3, :3]
    np.testing.assert_allclose(R, Rotation.from_rotvec(phi).as_matrix(), atol=1e-12)
    xi = rng.normal(size=6)
    np.testing.assert_allclose(optim.se3_exp(xi) @ optim.se3_exp(-xi), np.eye(4), atol=1e-12)


def test_pose_update_left_perturbation():
    """A small left twist moves a world point's camera coordinates by
    rho + phi x p to first order (the convention of the pose gradient)."""
    rng = np.random.default_rng(3)
    R = Rotation.from_rotvec(rng.normal(size=3)).as_matrix()
    T = np.concatenate([R, rng.normal(size=(3, 1))], axis=1)
    x = rng.normal(size=3)
    p = T[:, :3] @ x + T[:, 3]
    xi = rng.normal(size=6) * 1e-6
    T2 = optim.pose_update(T, xi)
    p2 = T2[:, :3] @ x + T2[:, 3]
    np.testing.assert_allclose(p2 - p, xi[:3] + np.cross(xi[3:], p), atol=1e-11)
