"""FP64 reference of the two further terms of the mapping objective (Sec. IV-D):
the MP-based motion consistency L_MP (Eq. (23)-(24)) and the MP-guided
edge-warp term L_edge (Eq. (25)-(26)); with the photometric and depth terms
they make L_G = l1 L_pho + l2 L_depth + l3 L_MP + l4 L_edge (Eq. (27)),
l3 = 500 and l4 = 300 (Sec. V-A).

TEST INFRASTRUCTURE ONLY (see the package docstring).

L_MP: sum_k (1 - M_k) |mu_k - mu_hat_k|^2 with mu_hat_k = T mu_k^{t-1}, the
previous mean carried by the relative transform T (the identity when the means
live in one world frame, as here). Its gradient is 2 (1 - M_k)(mu_k -
mu_hat_k); MP is a state and gets none.

L_edge, for a pair of frames (i, j): over the edge pixels u of frame i, the
observed depth D_i(u) lifts u into camera i, the relative motion T_ji = T_j
T_i^-1 carries the point into camera j and the pinhole K_j projects it to u';
the rendered depth D_j and the static weight w^j (Eq. (20)) of frame j are
sampled bilinearly at u' and rho(w^j(u') (D_j(u') - D_i(u))) is summed, rho
the Huber kernel with threshold delta. Readings (the paper leaves them open):
  * the edge pixels are where the Sobel slope of the observed depth,
    |(S_x, S_y)| / 8 with the 3x3 Sobel kernels, exceeds `edge_thresh`
    (metres per pixel), among interior pixels whose 3x3 neighbourhood is
    fully observed; the decision is taken in float32 (the precision the GPU
    takes it in) with the operation order of `sobel_f32`;
  * D_j is the rendered depth of frame j (the term then reaches the Gaussians
    and frame j's pose through the render) and w^j is held constant in the
    adjoint, as the photometric weight is;
  * bilinear sampling uses the four pixel centres around u' (centres at
    integer coordinates) and skips u' whose four neighbours are not all in
    the image, or whose camera-j depth is not beyond z_near;
  * the adjoint reaches frame j's depth image (four bilinear weights) and the
    left pose twists of both frames through u'.

Pinned by tests/test_oracle_objective.py: closed forms (zero motion, constant
depth offsets in both Huber branches, a single Gaussian's L_MP), the Sobel
slopes against scipy.ndimage.sobel, the warp's round trip i -> j -> i, and
central finite differences of both terms in every input they differentiate.
"""

from __future__ import annotations

import numpy as np

LAMBDA_MP = 500.0
LAMBDA_EDGE = 300.0
EDGE_DEFAULTS = dict(edge_thresh=0.05, delta=0.05, eps_A=1e-6)


# ---------------------------------------------------------------- L_MP
def mp_regularizer(mean, mean_prev, mp, T=None, lam=1.0):
    """(lam * L_MP, dL/dmean [3, n]) with mu_hat = R mean_prev + t, T = [R | t]."""
    mu = np.asarray(mean, np.float64)
    mp_ = np.asarray(mean_prev, np.float64)
    if T is not None:
        T = np.asarray(T, np.float64).reshape(3, 4)
        mp_ = T[:, :3] @ mp_ + T[:, 3:4]
    wbar = 1.0 - np.asarray(mp, np.float64)
    d = mu - mp_
    L = lam * float((wbar * (d * d).sum(axis=0)).sum())
    return L, lam * 2.0 * wbar[None, :] * d


# ---------------------------------------------------------------- L_edge
def sobel_f32(D, W, H):
    """Sobel slopes (S_x / 8, S_y / 8) of a depth image in float32, each sum in
    the order ((a + 2 b) + c) - ((d + 2 e) + f), and the squared magnitude
    gx * gx + gy * gy; zero on the border."""
    A = np.asarray(D, np.float32).reshape(H, W)
    f = np.float32
    gx = np.zeros((H, W), f)
    gy = np.zeros((H, W), f)
    two = f(2.0)
    r = (A[:-2, 2:] + two * A[1:-1, 2:]).astype(f) + A[2:, 2:]
    l = (A[:-2, :-2] + two * A[1:-1, :-2]).astype(f) + A[2:, :-2]
    gx[1:-1, 1:-1] = ((r.astype(f) - l.astype(f)) * f(0.125)).astype(f)
    b = (A[2:, :-2] + two * A[2:, 1:-1]).astype(f) + A[2:, 2:]
    t = (A[:-2, :-2] + two * A[:-2, 1:-1]).astype(f) + A[:-2, 2:]
    gy[1:-1, 1:-1] = ((b.astype(f) - t.astype(f)) * f(0.125)).astype(f)
    m2 = ((gx * gx).astype(f) + (gy * gy).astype(f)).astype(f)
    return gx, gy, m2


def edge_mask(D, W, H, thresh):
    """Edge pixels of an observed depth image (see the module docstring)."""
    A = np.asarray(D, np.float32).reshape(H, W)
    valid = A > 0
    full = np.zeros((H, W), bool)
    full[1:-1, 1:-1] = np.all([valid[1 + dy:H - 1 + dy, 1 + dx:W - 1 + dx] for dy in (-1, 0, 1) for dx in (-1, 0, 1)],
                              axis=0)
    _, _, m2 = sobel_f32(D, W, H)
    t = np.float32(thresh)
    return full & (m2 > (t * t).astype(np.float32))


def _pose(cam):
    T = np.asarray(cam["T_cw"], np.float64).reshape(3, 4)
    return T[:, :3], T[:, 3]


def warp(cam_i, cam_j, u, D_i):
    """Pixels u [2, k] of frame i with depth D_i lifted and carried into frame
    j: returns (u' [2, k], the point in camera j [3, k], the point in camera i
    [3, k])."""
    Ri, ti = _pose(cam_i)
    Rj, tj = _pose(cam_j)
    u = np.asarray(u, np.float64)
    Xi = np.stack([D_i * (u[0] - cam_i["cx"]) / cam_i["fx"], D_i * (u[1] - cam_i["cy"]) / cam_i["fy"], D_i])
    pw = Ri.T @ (Xi - ti[:, None])
    P = Rj @ pw + tj[:, None]
    up = np.stack([cam_j["fx"] * P[0] / P[2] + cam_j["cx"], cam_j["fy"] * P[1] / P[2] + cam_j["cy"]])
    return up, P, Xi


def static_weight(M, T, eps_A=1e-6):
    """w = 1 - M / A where A = 1 - T exceeds eps_A, else 0 (Eq. (20))."""
    A = 1.0 - np.asarray(T, np.float64)
    ok = A > eps_A
    return np.where(ok, 1.0 - np.asarray(M, np.float64) / np.where(ok, A, 1.0), 0.0)


def huber(r, delta):
    a = np.abs(r)
    return np.where(a <= delta, 0.5 * r * r, delta * (a - 0.5 * delta))


def edge_warp(cam_i, cam_j, D_obs_i, D_j, M_j, T_j, lam=1.0, edge_thresh=0.05, delta=0.05, eps_A=1e-6,
              w_fixed=None):
    """lam * L_edge^{i->j} and its adjoints: dD_j [P_j] (frame j's rendered
    depth), the left pose twists (rho, phi) of frames i and j, plus the
    per-edge-pixel details (used for parity): edge list, u', sampled w and
    validity. With w_fixed (per edge pixel of frame i) the sampled weight is
    replaced by it (finite differences hold it constant)."""
    Wi, Hi = cam_i["width"], cam_i["height"]
    Wj, Hj = cam_j["width"], cam_j["height"]
    E = np.nonzero(edge_mask(D_obs_i, Wi, Hi, edge_thresh).ravel())[0]
    u = np.stack([(E % Wi).astype(np.float64), (E // Wi).astype(np.float64)])
    Di = np.asarray(D_obs_i, np.float32).astype(np.float64)[E]
    up, P, Xi = warp(cam_i, cam_j, u, Di)
    x0 = np.floor(up[0])
    y0 = np.floor(up[1])
    ok = (P[2] > cam_j["z_near"]) & (x0 >= 0) & (x0 + 1 <= Wj - 1) & (y0 >= 0) & (y0 + 1 <= Hj - 1)
    x0i = np.where(ok, x0, 0).astype(np.int64)
    y0i = np.where(ok, y0, 0).astype(np.int64)
    fx = np.where(ok, up[0] - x0, 0.0)
    fy = np.where(ok, up[1] - y0, 0.0)
    idx = [y0i * Wj + x0i, y0i * Wj + x0i + 1, (y0i + 1) * Wj + x0i, (y0i + 1) * Wj + x0i + 1]
    bw = [(1 - fx) * (1 - fy), fx * (1 - fy), (1 - fx) * fy, fx * fy]
    Dj = np.asarray(D_j, np.float64)
    wj = static_weight(M_j, T_j, eps_A)
    Ds = sum(b * Dj[i] for b, i in zip(bw, idx))
    ws = sum(b * wj[i] for b, i in zip(bw, idx)) if w_fixed is None else np.asarray(w_fixed, np.float64)
    r = np.where(ok, ws * (Ds - Di), 0.0)
    L = lam * float(huber(r, delta)[ok].sum())
    g = np.where(ok, lam * np.clip(r, -delta, delta) * ws, 0.0)  # dL/dD_j(u')
    dD = np.zeros(Wj * Hj)
    for b, i in zip(bw, idx):
        np.add.at(dD, i[ok], (g * b)[ok])
    # through u' (the sampled weight is held constant)
    dDx = (1 - fy) * (Dj[idx[1]] - Dj[idx[0]]) + fy * (Dj[idx[3]] - Dj[idx[2]])
    dDy = (1 - fx) * (Dj[idx[2]] - Dj[idx[0]]) + fx * (Dj[idx[3]] - Dj[idx[1]])
    gu = np.stack([g * dDx, g * dDy])  # dL/du'
    z = P[2]
    gP = np.stack([gu[0] * cam_j["fx"] / z, gu[1] * cam_j["fy"] / z,
                   -(gu[0] * cam_j["fx"] * P[0] + gu[1] * cam_j["fy"] * P[1]) / (z * z)])
    gP = np.where(ok[None], gP, 0.0)
    Ri, _ = _pose(cam_i)
    Rj, _ = _pose(cam_j)
    Rji = Rj @ Ri.T
    pose_j = np.concatenate([gP.sum(axis=1), np.cross(P.T, gP.T).sum(axis=0)])
    q = Rji.T @ gP
    pose_i = np.concatenate([-q.sum(axis=1), -np.cross(Xi.T, q.T).sum(axis=0)])
    return dict(loss=L, dD=dD, pose_i=pose_i, pose_j=pose_j, edges=E, up=up, ok=ok, w=ws, r=r)
