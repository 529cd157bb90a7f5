"""Pins of the FP64 reference of L_MP (Eq. (23)-(24)) and L_edge (Eq. (25)-(26))
(CPU only): closed forms, the Sobel slopes against scipy, the warp's round
trip, and central finite differences of every adjoint."""

import numpy as np
import pytest
from scipy import ndimage
from scipy.linalg import expm

from paper_2602_21644_amd import synth


@pytest.fixture(scope="module")
def obj(orc):
    from oracle import objective
    return objective


def test_mp_regularizer_closed_form(obj):
    """One Gaussian: (1 - M) |mu - mu_prev|^2 and gradient 2 (1 - M)(mu -
    mu_prev); a fully dynamic Gaussian (M = 1) costs nothing; a mean carried
    exactly by the relative motion costs nothing."""
    L, g = obj.mp_regularizer([[1.0], [2.0], [3.0]], [[0.0], [0.0], [0.0]], [0.25])
    assert L == pytest.approx(0.75 * 14.0, rel=1e-15)
    np.testing.assert_allclose(g[:, 0], [1.5, 3.0, 4.5], rtol=1e-15)
    L, g = obj.mp_regularizer([[1.0], [2.0], [3.0]], [[0.0], [0.0], [0.0]], [1.0])
    assert L == 0.0 and np.all(g == 0)
    rng = np.random.default_rng(0)
    T = synth.perturbed_pose(rng, deg=7.0, trans=0.3).astype(np.float64)
    prev = rng.normal(size=(3, 50))
    cur = T[:, :3] @ prev + T[:, 3:4]
    L, g = obj.mp_regularizer(cur, prev, rng.random(50), T=T)
    assert L < 1e-25 and np.abs(g).max() < 1e-12


def test_mp_regularizer_finite_differences(obj):
    rng = np.random.default_rng(1)
    mu, prev, mp = rng.normal(size=(3, 20)), rng.normal(size=(3, 20)), rng.random(20)
    L, g = obj.mp_regularizer(mu, prev, mp, lam=500.0)
    for _ in range(10):
        c, k = rng.integers(3), rng.integers(20)
        h = 1e-6
        a, b = mu.copy(), mu.copy()
        a[c, k] += h
        b[c, k] -= h
        fd = (obj.mp_regularizer(a, prev, mp, lam=500.0)[0] - obj.mp_regularizer(b, prev, mp, lam=500.0)[0]) / (2 * h)
        assert fd == pytest.approx(g[c, k], rel=1e-7, abs=1e-7)


def test_sobel_against_scipy(obj):
    rng = np.random.default_rng(2)
    W, H = 23, 17
    D = rng.uniform(0.5, 4.0, size=H * W).astype(np.float32)
    gx, gy, m2 = obj.sobel_f32(D, W, H)
    A = D.reshape(H, W).astype(np.float64)
    sx = ndimage.sobel(A, axis=1, mode="constant") / 8.0
    sy = ndimage.sobel(A, axis=0, mode="constant") / 8.0
    np.testing.assert_allclose(gx[1:-1, 1:-1], sx[1:-1, 1:-1], rtol=1e-5, atol=1e-6)
    np.testing.assert_allclose(gy[1:-1, 1:-1], sy[1:-1, 1:-1], rtol=1e-5, atol=1e-6)
    # the float32 edge decision agrees with the float64 slope except within rounding
    mag = np.hypot(sx, sy)
    e = obj.edge_mask(D, W, H, 0.3)
    inner = np.zeros((H, W), bool)
    inner[1:-1, 1:-1] = True
    assert np.all(e[inner] | (mag[inner] <= 0.3 * (1 + 1e-5)))
    assert np.all(~e[inner] | (mag[inner] > 0.3 * (1 - 1e-5)))
    assert not e[~inner].any()
    # an unobserved pixel removes its 3x3 neighbourhood from the edges
    D2 = D.copy()
    D2[5 * W + 7] = 0.0
    e2 = obj.edge_mask(D2, W, H, 0.0)
    assert not e2[4:7, 6:9].any() and e2[10, 15]


def test_warp_round_trip(obj):
    """A pixel of frame i lifted with depth d, carried to frame j, and lifted
    there with its camera-j depth comes back to the same pixel."""
    from scipy.spatial.transform import Rotation
    rng = synth.rng_for(3)
    cams = []
    for _ in range(2):  # exactly orthonormal float64 poses, so that R^T is R^-1
        c = synth.camera(64, 48)
        c["T_cw"] = np.concatenate([Rotation.from_rotvec(rng.normal(size=3) * 0.05).as_matrix(),
                                    rng.normal(size=(3, 1)) * 0.1], axis=1)
        cams.append(c)
    ci, cj = cams
    u = np.stack([rng.integers(0, 64, 30), rng.integers(0, 48, 30)]).astype(np.float64)
    d = rng.uniform(0.5, 4.0, 30)
    up, P, Xi = obj.warp(ci, cj, u, d)
    back, P2, X2 = obj.warp(cj, ci, up, P[2])
    np.testing.assert_allclose(back, u, atol=1e-9)
    np.testing.assert_allclose(P2, Xi, atol=1e-12)


def _frames(orc, n=3000, W=64, H=48, seed=4):
    g, cam, tcam = synth.tiny_scene(seed=seed, n=n, width=W, height=H)
    rng = synth.rng_for(seed + 10)
    cj = synth.camera(W, H, synth.perturbed_pose(rng, deg=1.0, trans=0.02))
    obs = orc.render(orc.project(g, cam), g, cam)
    Dobs = np.where(1 - obs["T"] >= 0.5, obs["D"], 0.0).astype(np.float32)
    rj = orc.render(orc.project(g, cj), g, cj)
    return cam, cj, Dobs, rj


def test_edge_warp_zero_motion_closed_form(obj):
    """Frames i and j the same camera, D_j = D_obs + c and w = 1 (M = 0,
    T ~ 0): every edge pixel lands on itself and costs rho(c), in the
    quadratic branch (c < delta) and the linear one (c > delta)."""
    W, H = 40, 30
    yy, xx = np.mgrid[0:H, 0:W]
    D = np.where(xx < 20, 1.0, 2.0) + 0.01 * yy
    D = D.astype(np.float32).ravel()
    cam = synth.camera(W, H)
    for c, expect in ((0.02, 0.5 * 0.02 ** 2), (0.2, 0.05 * (0.2 - 0.025))):
        r = obj.edge_warp(cam, cam, D, D.astype(np.float64) + c, np.zeros(W * H), np.full(W * H, 1e-12), delta=0.05,
                          edge_thresh=0.1)
        ne = r["edges"].size
        assert ne > 0 and r["ok"].all()
        np.testing.assert_allclose(r["up"], np.stack([r["edges"] % W, r["edges"] // W]).astype(float), atol=1e-12)
        assert r["loss"] == pytest.approx(ne * expect, rel=1e-9)
        assert np.abs(r["pose_i"] + np.concatenate([r["pose_j"][:3], r["pose_j"][3:]])).max() < 1e-6 * (
            1 + np.abs(r["pose_j"]).max())


def _retract(cam, xi):
    X = np.zeros((4, 4))
    rho, phi = xi[:3], xi[3:]
    X[:3, :3] = np.array([[0, -phi[2], phi[1]], [phi[2], 0, -phi[0]], [-phi[1], phi[0], 0]])
    X[:3, 3] = rho
    T = np.eye(4)
    T[:3] = np.asarray(cam["T_cw"], float)
    c = dict(cam)
    c["T_cw"] = (expm(X) @ T)[:3]
    return c


def test_edge_warp_finite_differences(orc, obj):
    """Central differences of l4 L_edge (the sampled weights held at their
    values) in frame j's rendered depth and in the left pose twists of both
    frames; a coordinate is used only when two step sizes agree."""
    ci, cj, Dobs, rj = _frames(orc)
    kw = dict(lam=300.0, edge_thresh=0.02, delta=0.05)
    r = obj.edge_warp(ci, cj, Dobs, rj["D"], rj["M"], rj["T"], **kw)
    assert r["ok"].sum() > 20 and r["loss"] > 0
    wf = r["w"]
    # depth image of frame j
    rng = np.random.default_rng(5)
    cand = np.nonzero(np.abs(r["dD"]) > 0)[0]
    for p in rng.choice(cand, size=min(12, cand.size), replace=False):
        vals = []
        for s in (1, -1):
            D = rj["D"].copy()
            D[p] += s * 1e-6
            vals.append(obj.edge_warp(ci, cj, Dobs, D, rj["M"], rj["T"], w_fixed=wf, **kw)["loss"])
        assert (vals[0] - vals[1]) / 2e-6 == pytest.approx(r["dD"][p], rel=1e-6, abs=1e-8)
    # pose twists
    checked = 0
    for which in ("pose_i", "pose_j"):
        for a in range(6):
            ests = []
            for h in (1e-6, 1e-7):
                vals = []
                for s in (1, -1):
                    xi = np.zeros(6)
                    xi[a] = s * h
                    c_i, c_j = (_retract(ci, xi), cj) if which == "pose_i" else (ci, _retract(cj, xi))
                    vals.append(obj.edge_warp(c_i, c_j, Dobs, rj["D"], rj["M"], rj["T"], w_fixed=wf, **kw)["loss"])
                ests.append((vals[0] - vals[1]) / (2 * h))
            if abs(ests[0] - ests[1]) > 1e-4 * abs(ests[0]) + 1e-6:
                continue
            assert ests[1] == pytest.approx(r[which][a], rel=1e-4, abs=1e-5), (which, a, ests, r[which][a])
            checked += 1
    assert checked >= 10
