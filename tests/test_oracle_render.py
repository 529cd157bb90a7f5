"""Pins of the FP64 oracle's projection, render, loss and adjoint (CPU only).

Each test checks the oracle against something other than itself: a closed
form, an ordering identity, an invariant, an independent brute force built on
library routines (scipy rotations, numpy matrix inverse), finite differences
of the oracle's own forward, or exact rigid-motion identities of the gradient.
"""

import numpy as np
import pytest
from scipy.linalg import expm
from scipy.spatial.transform import Rotation

from paper_2602_21644_amd import synth


def one_gaussian(z=2.0, s=0.05, o_logit=1.0, color=(0.2, 0.5, 0.9), mp=0.3, quat=None):
    q = np.array([1.0, 0, 0, 0]) if quat is None else np.asarray(quat, float)
    g = dict(mean=np.array([[0.0], [0.0], [z]], np.float32), log_scale=np.full((3, 1), np.log(s), np.float32),
             quat=q.reshape(4, 1).astype(np.float32), opacity_logit=np.array([o_logit], np.float32),
             color=np.array(color, np.float32).reshape(3, 1), mp=np.array([mp], np.float32))
    return g


def test_single_gaussian_closed_form(orc):
    """Isotropic Gaussian on the optical axis: Sigma2D = ((f s / z)^2 + 0.3) I,
    alpha(i, j) = min(0.99, o exp(-r^2 / (2 sigma^2))) above 1/255, and
    C = alpha c, D = alpha z, M = alpha m, T = 1 - alpha."""
    cam = synth.camera(64, 48)
    quat = Rotation.random(random_state=3).as_quat()[[3, 0, 1, 2]]  # isotropic: rotation irrelevant
    g = one_gaussian(quat=quat)
    s = float(g["log_scale"][0, 0])
    z = float(g["mean"][2, 0])
    o = 1 / (1 + np.exp(-float(g["opacity_logit"][0])))
    sig2 = (cam["fx"] * np.exp(s) / z) ** 2 + 0.3
    pr = orc.project(g, cam)
    assert pr["kept"][0]
    np.testing.assert_allclose(pr["mean2d"][:, 0], [cam["cx"], cam["cy"]], atol=1e-12)
    np.testing.assert_allclose(pr["cov2d"][:, 0], [sig2, 0, sig2], rtol=1e-10, atol=1e-12)
    np.testing.assert_allclose(pr["conic"][:, 0], [1 / sig2, 0, 1 / sig2], rtol=1e-10, atol=1e-12)
    assert pr["radius"][0] == int(np.ceil(np.sqrt(2 * np.log(255 * o) * sig2)))
    im = orc.render(pr, g, cam)
    jj, ii = np.mgrid[0:48, 0:64]
    r2 = (ii - cam["cx"]) ** 2 + (jj - cam["cy"]) ** 2
    a = np.minimum(0.99, o * np.exp(-0.5 * r2 / sig2))
    a = np.where(a >= 1 / 255, a, 0.0).ravel()
    for c in range(3):
        np.testing.assert_allclose(im["C"][c], a * float(g["color"][c, 0]), atol=1e-12)
    np.testing.assert_allclose(im["D"], a * z, atol=1e-12)
    np.testing.assert_allclose(im["M"], a * float(g["mp"][0]), atol=1e-12)
    np.testing.assert_allclose(im["T"], 1 - a, atol=1e-12)


def test_single_gaussian_gradients_closed_form(orc):
    """For one Gaussian and a linear upstream L = sum_u gC . C + gD D, the
    colour adjoint is sum_u alpha gC and the depth adjoint sum_u alpha gD."""
    cam = synth.camera(64, 48)
    g = one_gaussian()
    pr = orc.project(g, cam)
    im = orc.render(pr, g, cam)
    rng = np.random.default_rng(0)
    P = 64 * 48
    gC = rng.normal(size=(3, P))
    gD = rng.normal(size=P)
    g2d = orc.render_backward(pr, g, cam, gC, gD)
    a = 1 - im["T"]
    np.testing.assert_allclose(g2d[6:9, 0], (a[None] * gC).sum(axis=1), rtol=1e-12)
    np.testing.assert_allclose(g2d[9, 0], (a * gD).sum(), rtol=1e-12)


def test_two_gaussians_order(orc):
    """C = a1 c1 + (1 - a1) a2 c2 for the nearer Gaussian 1; swapping the
    depths swaps the roles."""
    cam = synth.camera(64, 48)
    g1 = one_gaussian(z=1.5, color=(1, 0, 0), o_logit=0.5)
    g2 = one_gaussian(z=2.5, color=(0, 1, 0), o_logit=1.5)
    g = synth.concat_gaussians([g1, g2])
    pr = orc.project(g, cam)
    im = orc.render(pr, g, cam)
    pix = 24 * 64 + 32
    a1 = min(0.99, pr["opacity"][0])
    a2 = min(0.99, pr["opacity"][1])
    np.testing.assert_allclose(im["C"][:, pix], [a1, (1 - a1) * a2, 0], atol=1e-12)
    gs = {k: v.copy() for k, v in g.items()}
    gs["mean"][2] = gs["mean"][2][::-1]
    pr = orc.project(gs, cam)
    im = orc.render(pr, gs, cam)
    a1 = min(0.99, pr["opacity"][0])
    a2 = min(0.99, pr["opacity"][1])
    np.testing.assert_allclose(im["C"][:, pix], [(1 - a2) * a1, a2, 0], atol=1e-12)


def _brute_alpha(g, cam, k, i, j):
    """Independent alpha of Gaussian k at pixel (i, j): scipy rotation, numpy
    inverse, explicit pinhole Jacobian."""
    R = np.asarray(cam["T_cw"], float)[:, :3]
    t = np.asarray(cam["T_cw"], float)[:, 3]
    mu = g["mean"][:, k].astype(float)
    p = R @ mu + t
    q = g["quat"][:, k].astype(float)
    Rq = Rotation.from_quat([q[1], q[2], q[3], q[0]]).as_matrix()
    S = np.diag(np.exp(g["log_scale"][:, k].astype(float)))
    Sig = Rq @ S @ S @ Rq.T
    fx, fy = cam["fx"], cam["fy"]
    J = np.array([[fx / p[2], 0, -fx * p[0] / p[2] ** 2], [0, fy / p[2], -fy * p[1] / p[2] ** 2]])
    cov = J @ R @ Sig @ R.T @ J.T + 0.3 * np.eye(2)
    u = np.array([fx * p[0] / p[2] + cam["cx"], fy * p[1] / p[2] + cam["cy"]])
    d = np.array([i, j]) - u
    o = 1 / (1 + np.exp(-float(g["opacity_logit"][k])))
    return min(0.99, o * np.exp(-0.5 * d @ np.linalg.inv(cov) @ d)), p[2]


def test_brute_force_pixels(orc):
    """A few pixels of the perturbed-pose tiny scene recomposited by a plain
    loop over all Gaussians sorted by (depth, id), using _brute_alpha."""
    g, cam, tcam = synth.tiny_scene(seed=5, n=300)
    pr = orc.project(g, tcam)
    pixels = [0, 64 * 20 + 31, 64 * 47 + 63, 64 * 10 + 5, 64 * 33 + 50]
    im = orc.render(pr, g, tcam, pixels=pixels, bg=(0.1, 0.2, 0.3))
    n = g["opacity_logit"].shape[0]
    for q, pix in enumerate(pixels):
        i, j = pix % 64, pix // 64
        al = []
        for k in range(n):
            a, z = _brute_alpha(g, tcam, k, i, j)
            if z > 0.2:
                al.append((z, k, a))
        al.sort()
        T, C, D, M = 1.0, np.zeros(3), 0.0, 0.0
        for z, k, a in al:
            if a < 1 / 255:
                continue
            if T * (1 - a) < 1e-4:
                break
            C += a * T * g["color"][:, k]
            D += a * T * z
            M += a * T * g["mp"][k]
            T *= 1 - a
        np.testing.assert_allclose(im["C"][:, q], C + T * np.array([0.1, 0.2, 0.3]), atol=1e-9)
        np.testing.assert_allclose([im["D"][q], im["M"][q], im["T"][q]], [D, M, T], atol=1e-9)


def test_render_invariants_and_support(orc):
    """T in [1e-4, 1]; A = 1 - T = sum omega <= 1; M <= A; w in [0, 1];
    C in [0, 1]^3; D <= z_max A; and no pixel outside a Gaussian's tile-rect
    pixel range [floor(u) - r, floor(u) + r] reaches alpha >= 1/255."""
    g, cam, tcam = synth.tiny_scene()
    pr = orc.project(g, cam)
    im = orc.render(pr, g, cam)
    T, M, C, D = im["T"], im["M"], im["C"], im["D"]
    A = 1 - T
    assert T.min() >= 1e-4 and T.max() <= 1
    assert np.all(M <= A + 1e-12)
    assert np.all((C >= -1e-12) & (C <= 1 + 1e-12))
    assert np.all(D <= pr["depth"][pr["kept"]].max() * A + 1e-9)
    L = orc.loss(im, np.zeros((3, 64 * 48)), np.zeros(64 * 48))
    assert L["w"].min() >= -1e-12 and L["w"].max() <= 1 + 1e-12
    jj, ii = np.mgrid[0:48, 0:64]
    for k in np.nonzero(pr["kept"])[0]:
        d0 = pr["mean2d"][0, k] - ii
        d1 = pr["mean2d"][1, k] - jj
        k1, k2, k3 = pr["conic"][:, k]
        a = pr["opacity"][k] * np.exp(-0.5 * (k1 * d0 * d0 + k3 * d1 * d1) - k2 * d0 * d1)
        r = pr["radius"][k]
        ix, iy = np.floor(pr["mean2d"][:, k])
        outside = (ii < ix - r) | (ii > ix + r) | (jj < iy - r) | (jj > iy + r)
        assert not np.any((a >= 1 / 255) & outside), k


def test_loss_special_cases(orc):
    """MP = 0 gives the plain L1 loss on covered pixels (w = 1); MP = 1 gives
    zero loss and zero adjoints; MP = m scales the loss by (1 - m)."""
    g, cam, tcam = synth.tiny_scene()
    pr = orc.project(g, cam)
    rng = np.random.default_rng(1)
    tc, td = rng.random((3, 3072)), rng.random(3072) * 3
    td[::7] = 0
    res = []
    for m in (0.0, 1.0, 0.3):
        gm = dict(g)
        gm["mp"] = np.full_like(g["mp"], m)
        im = orc.render(pr, gm, cam)
        res.append(orc.loss(im, tc, td))
        if m == 0.0:
            covered = (1 - im["T"]) > 1e-6
            assert np.allclose(res[-1]["w"][covered], 1.0)
            plain = 0.9 * np.abs(im["C"] - tc).sum(0) + 0.1 * np.where(td > 0, np.abs(im["D"] - td), 0)
            np.testing.assert_allclose(res[-1]["loss"], plain[covered].sum(), rtol=1e-12)
    assert abs(res[1]["loss"]) < 1e-9 and np.abs(res[1]["dC"]).max() < 1e-9
    np.testing.assert_allclose(res[2]["loss"], (1 - float(np.float32(0.3))) * res[0]["loss"], rtol=1e-9)


def _retract(cam, xi):
    """Left perturbation T <- Exp(xi) T with xi = (rho, phi), via scipy expm."""
    X = np.zeros((4, 4))
    rho, phi = xi[:3], xi[3:]
    X[:3, :3] = np.array([[0, -phi[2], phi[1]], [phi[2], 0, -phi[0]], [-phi[1], phi[0], 0]])
    X[:3, 3] = rho
    E = expm(X)
    T = np.eye(4)
    T[:3] = np.asarray(cam["T_cw"], float)
    c = dict(cam)
    c["T_cw"] = (E @ T)[:3]
    return c


def _scene_with_target(orc, seed=1, n=2000):
    g, cam, tcam = synth.tiny_scene(seed=seed, n=n)
    pr_t = orc.project(g, tcam)
    tgt = orc.render(pr_t, g, tcam)
    td = tgt["D"].copy()
    td[(1 - tgt["T"]) < 0.5] = 0.0
    return g, cam, tgt["C"], td


def _as64(g):
    return {k: np.asarray(v, np.float64) for k, v in g.items()}


def test_adjoint_finite_differences(orc):
    """Central differences of the FP64 forward (w held fixed) against the
    adjoint, per parameter group, on coordinates with large gradients. A
    coordinate is used only if two step sizes agree (no threshold crossed)."""
    g, cam, tc, td = _scene_with_target(orc)
    L, im, grads, pr, _ = orc.full_backward(g, cam, tc, td)
    w0 = L["w"]
    g64 = _as64(g)
    rng = np.random.default_rng(2)
    checked = 0
    for name in ("mean", "log_scale", "quat", "opacity_logit", "color"):
        G = grads[name].reshape(-1, g64[name].shape[-1]) if grads[name].ndim > 1 else grads[name][None]
        flat = np.abs(G).ravel()
        cand = np.argsort(flat)[::-1][:40]
        cand = rng.choice(cand, size=6, replace=False)
        for idx in cand:
            row, k = np.unravel_index(idx, G.shape)
            ests = []
            for h in (1e-5, 1e-6):
                vals = []
                for sgn in (1, -1):
                    gp = {kk: v.copy() for kk, v in g64.items()}
                    arr = gp[name] if gp[name].ndim > 1 else gp[name][None]
                    scale = max(1.0, abs(arr[row, k]))
                    arr[row, k] += sgn * h * scale
                    vals.append(orc.forward_loss(gp, cam, tc, td, w_fixed=w0))
                ests.append((vals[0] - vals[1]) / (2 * h * scale))
            if abs(ests[0] - ests[1]) > 1e-6 * max(abs(ests[0]), 1e-9) + 1e-9:
                continue
            an = G[row, k]
            assert abs(an - ests[1]) <= 1e-5 * abs(ests[1]) + 1e-7, (name, row, k, an, ests)
            checked += 1
    assert checked >= 15


def test_pose_gradient_finite_differences(orc):
    """A pose step moves every Gaussian, so step sizes are small enough that no
    alpha or stop threshold is crossed (checked by two step sizes agreeing)."""
    g, cam, tc, td = _scene_with_target(orc, n=500)
    L, im, grads, pr, _ = orc.full_backward(g, cam, tc, td)
    g64 = _as64(g)
    for i in range(6):
        ests = []
        for h in (1e-7, 2e-8):
            xi = np.zeros(6)
            xi[i] = h
            lp = orc.forward_loss(g64, _retract(cam, xi), tc, td, w_fixed=L["w"])
            lm = orc.forward_loss(g64, _retract(cam, -xi), tc, td, w_fixed=L["w"])
            ests.append((lp - lm) / (2 * h))
        assert abs(ests[0] - ests[1]) <= 1e-5 * abs(ests[1]) + 1e-6
        assert abs(grads["pose"][i] - ests[1]) <= 1e-5 * abs(ests[1]) + 1e-6, (i, grads["pose"][i], ests)


def rigid_identity(grads, g, cam):
    """Exact identities between the pose twist adjoint and the per-Gaussian
    adjoints (w detached): moving the camera by Exp(xi) equals moving every
    Gaussian by the inverse motion. rho_bar = R sum_k mu_bar_k and
    phi_bar = sum_k [p_k x (R mu_bar_k) + R (dq'/domega)^T q_bar_k], with
    dq'/domega = 1/2 [-q_v^T ; q_w I - [q_v]x]."""
    R = np.asarray(cam["T_cw"], float)[:, :3]
    t = np.asarray(cam["T_cw"], float)[:, 3]
    mb = np.asarray(grads["mean"], float)
    qb = np.asarray(grads["quat"], float)
    mu = np.asarray(g["mean"], float)
    q = np.asarray(g["quat"], float)
    p = R @ mu + t[:, None]
    Rmb = R @ mb
    rho = Rmb.sum(axis=1)
    phi = np.cross(p.T, Rmb.T).sum(axis=0)
    qw, qv = q[0], q[1:]
    # (dq'/domega)^T q_bar, per Gaussian
    tq = np.zeros((3, q.shape[1]))
    tq += -qv * qb[0]
    tq += qw * qb[1:]
    # ([q_v]x)^T qbv = -[q_v]x qbv = -(q_v x qbv)  -> minus sign folded: -[q_v]x^T = [q_v]x
    tq += np.cross(qv.T, qb[1:].T).T
    phi += (R @ (0.5 * tq)).sum(axis=1)
    return np.concatenate([rho, phi])


def test_pose_gradient_rigid_identity(orc):
    g, cam, tc, td = _scene_with_target(orc, seed=7)
    cam = _retract(cam, np.array([0.01, -0.02, 0.03, 0.02, 0.01, -0.03]))
    L, im, grads, pr, _ = orc.full_backward(g, cam, tc, td)
    ident = rigid_identity(grads, g, cam)
    np.testing.assert_allclose(grads["pose"], ident, rtol=1e-9, atol=1e-9 * np.abs(ident).max())


def test_bin_reference_matches_bruteforce(orc):
    """The stable-sort reference equals a per-tile brute force: for each tile,
    the records whose rectangle contains it, ordered by (depth key, id)."""
    rect, key = synth.bin_inputs(3, 400, 64, 48)
    ids, ranges = orc.bin_reference(rect, key, (4, 3))
    for t in range(12):
        tx, ty = t % 4, t // 4
        mine = [k for k in range(400) if key[k] != 0xFFFFFFFF and rect[k, 0] <= tx <= rect[k, 2]
                and rect[k, 1] <= ty <= rect[k, 3]]
        mine.sort(key=lambda k: (int(key[k]), k))
        b, e = ranges[t]
        assert list(ids[b:e]) == mine


def test_depth_key_is_float32_camera_z(orc):
    """The ordering key is camera z evaluated with float32 roundings in the
    order ((R20 m0 + R21 m1) + R22 m2) + t2; it agrees with the float64 depth
    to float32 precision, and exactly equal keys keep id order."""
    g, cam, tcam, g_t, sl = synth.moving_box_scene(2, 3000, 64, 48)
    pr = orc.project(g, tcam)
    T = np.asarray(tcam["T_cw"], np.float32)
    m = g["mean"]
    f = np.float32
    z32 = (((T[2, 0] * m[0]).astype(f) + (T[2, 1] * m[1]).astype(f)).astype(f) + (T[2, 2] * m[2]).astype(f)).astype(f)
    z32 = (z32 + T[2, 3]).astype(f)
    k = pr["kept"]
    np.testing.assert_array_equal(pr["zkey"][k], z32[k].astype(np.float64))
    np.testing.assert_allclose(pr["zkey"][k], pr["depth"][k], rtol=2e-7)


def test_bin_reference_np_matches_textbook(orc):
    """The array form of the binning reference equals the record-by-record
    stable sort, including ties of equal depth keys and empty records."""
    for seed, m, W, H in ((3, 400, 64, 48), (4, 3000, 200, 150), (5, 1, 64, 48)):
        rect, key = synth.bin_inputs(seed, m, W, H)
        grid = ((W + 15) // 16, (H + 15) // 16)
        a_ids, a_r = orc.bin_reference(rect, key, grid)
        b_ids, b_r = orc.bin_reference_np(rect, key, grid)
        np.testing.assert_array_equal(a_ids, b_ids)
        np.testing.assert_array_equal(a_r, b_r)


def test_compact_reference(orc):
    """Removal by a drop mask against a plain loop: kept elements in order,
    each scene's new offset = the kept elements in front of it."""
    rng = np.random.default_rng(4)
    n = 257
    drop = rng.random(n) < 0.4
    a = rng.random((3, n))
    b = np.arange(n, dtype=np.float32)
    seg = [0, 100, 100, 257]
    (ca, cb), off = orc.compact([a, b], drop, seg)
    kept = [i for i in range(n) if not drop[i]]
    np.testing.assert_array_equal(cb, np.array(kept, np.float32))
    np.testing.assert_array_equal(ca, a[:, kept])
    assert off.tolist() == [0, sum(1 for i in kept if i < 100), sum(1 for i in kept if i < 100), len(kept)]
