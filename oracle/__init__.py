"""FP64 CPU oracle for the MP-weighted Gaussian-splatting path.

TEST INFRASTRUCTURE ONLY: the test suite, the smoke check and the benchmark's
CPU-baseline leg are the only users. The GPU library never imports, links or
calls anything here, and nothing here imports the GPU package: the two share
only the seeded input generator (which holds none of the method's arithmetic).

Parts and where they come from:
  * projection / render / render adjoint / projection adjoint: C++ in
    gs_oracle.cpp (EWA splatting with front-to-back alpha compositing; the
    paper relies on this renderer for Eq. (20)-(22) without spelling it out).
  * loss: the MP static weight of Eq. (20) and the weighted L1 colour and
    depth losses of Eq. (21)-(22), combined with lambda1 = 0.9, lambda2 = 0.1
    as in Eq. (27) and the implementation details of Sec. V-A.
  * binning reference: the stable ascending sort of (tile << 32 | depth bits)
    keys, i.e. per-tile lists in (depth, id) order.
  * MP update: Eq. (1)-(13) and (17) of Sec. IV-A/B (mp.py).
  * MLP surrogate (not in the paper): mlp.py.

Parity status of each function is listed in mp.py / mlp.py headers and in the
test files; every function here is pinned by the CPU tests in tests/.
"""

from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "gs_oracle.cpp")
_LIB_PATH = os.path.join(_HERE, "_gs_oracle.so")
_lib = None


def build(force: bool = True) -> str:
    """Compile the C++ oracle with g++ (-O3, OpenMP, FP64; no fast-math)."""
    if force or not os.path.exists(_LIB_PATH):
        tmp = _LIB_PATH + ".tmp"
        cmd = ["g++", "-O3", "-ffp-contract=off", "-fopenmp", "-fPIC", "-shared", "-std=c++17", "-o", tmp, _SRC]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build()
        L = ctypes.CDLL(_LIB_PATH)
        P = ctypes.c_void_p
        I64 = ctypes.c_int64
        L.or_project.argtypes = [I64] + [P] * 5 + [P] * 9
        L.or_render.argtypes = [I64] + [P] * 8 + [ctypes.c_int, ctypes.c_int, P, I64, P] + [P] * 6 + [ctypes.c_int]
        L.or_render_backward.argtypes = [I64] + [P] * 8 + [ctypes.c_int, ctypes.c_int, P, I64, P] + [P] * 5
        L.or_project_backward.argtypes = [I64] + [P] * 5 + [P] * 7
        L.or_num_threads.restype = ctypes.c_int
        L.or_set_threads.argtypes = [ctypes.c_int]
        _lib = L
    return _lib


def num_threads() -> int:
    return int(lib().or_num_threads())


def set_threads(n: int) -> None:
    lib().or_set_threads(int(n))


def _d(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _p(a):
    return a.ctypes.data_as(ctypes.c_void_p)


def cam_vector(cam: dict) -> np.ndarray:
    T = np.asarray(cam["T_cw"], dtype=np.float64).reshape(12)
    return np.concatenate([[cam["width"], cam["height"], cam["fx"], cam["fy"], cam["cx"], cam["cy"],
                            cam["z_near"]], T]).astype(np.float64)


# ------------------------------------------------------------------ projection
def project(g: dict, cam: dict) -> dict:
    """EWA projection of every Gaussian (FP64). Returns planar arrays and the
    `kept` mask (culled: non-finite input, z <= z_near, det <= 0, opacity < 1/255).
    `zkey` is the float32 camera z that orders Gaussians and decides the
    near-plane cull (computed with float32 roundings, as the GPU path does)."""
    n = g["opacity_logit"].shape[0]
    mean, ls, q, opl = _d(g["mean"]), _d(g["log_scale"]), _d(g["quat"]), _d(g["opacity_logit"])
    out = dict(mean2d=np.zeros((2, n)), conic=np.zeros((3, n)), cov2d=np.zeros((3, n)), depth=np.zeros(n),
               opacity=np.zeros(n), extent=np.zeros(n), radius=np.zeros(n, np.int32), kept=np.zeros(n, np.uint8),
               zkey=np.zeros(n))
    cv = cam_vector(cam)
    lib().or_project(n, _p(mean), _p(ls), _p(q), _p(opl), _p(cv), _p(out["mean2d"]), _p(out["conic"]),
                     _p(out["cov2d"]), _p(out["depth"]), _p(out["opacity"]), _p(out["extent"]),
                     _p(out["radius"]), _p(out["kept"]), _p(out["zkey"]))
    out["kept"] = out["kept"].astype(bool)
    return out


def tile_rect(mean2d, radius, kept, width, height, tile=16):
    """Inclusive tile rectangle covering pixel columns floor(u)-r .. floor(u)+r
    (and the same for rows), clipped to the grid; empty for culled Gaussians.
    Every pixel centre the alpha test can accept lies in this range because the
    support extent is at most r. Returns (x0, y0, x1, y1, empty)."""
    gx = (width + tile - 1) // tile
    gy = (height + tile - 1) // tile
    ix = np.floor(mean2d[0]).astype(np.int64)
    iy = np.floor(mean2d[1]).astype(np.int64)
    r = np.asarray(radius, dtype=np.int64)
    x0 = np.maximum(0, np.floor_divide(ix - r, tile))
    x1 = np.minimum(gx - 1, np.floor_divide(ix + r, tile))
    y0 = np.maximum(0, np.floor_divide(iy - r, tile))
    y1 = np.minimum(gy - 1, np.floor_divide(iy + r, tile))
    empty = (x0 > x1) | (y0 > y1) | ~np.asarray(kept, bool)
    return x0, y0, x1, y1, empty


# ------------------------------------------------------------------ render
def render(proj: dict, g: dict, cam: dict, bg=(0.0, 0.0, 0.0), pixels=None, order="f32") -> dict:
    """Tile-free FP64 render: every kept Gaussian per pixel in (float32 depth
    key, id) order with the alpha clamp, the 1/255 cut-off and the T < 1e-4 stop.
    Returns C[3,P], D, M (MP channel), T (final), margin, ncontrib.

    order="f64" orders by the float64 camera z instead, and the margin then
    also holds the smallest relative depth gap between consecutive Gaussians
    that take part in the pixel (used to measure what deciding the order in
    float32 changes)."""
    n = g["opacity_logit"].shape[0]
    W, H = cam["width"], cam["height"]
    if pixels is None:
        npix, pix, P = -1, np.zeros(1, np.int64), W * H
    else:
        pix = np.ascontiguousarray(pixels, dtype=np.int64)
        npix = P = pix.shape[0]
    out = dict(C=np.zeros((3, P)), D=np.zeros(P), M=np.zeros(P), T=np.zeros(P), margin=np.zeros(P),
               ncontrib=np.zeros(P, np.int32))
    kept = np.ascontiguousarray(proj["kept"], np.uint8)
    color, mp, bgv = _d(g["color"]), _d(g["mp"]), _d(bg)
    lib().or_render(n, _p(proj["mean2d"]), _p(proj["conic"]), _p(proj["depth"]), _p(proj["zkey"]),
                    _p(proj["opacity"]),
                    _p(color), _p(mp), _p(kept), W, H, _p(bgv), npix, _p(pix), _p(out["C"]), _p(out["D"]),
                    _p(out["M"]), _p(out["T"]), _p(out["margin"]), _p(out["ncontrib"]), 1 if order == "f64" else 0)
    return out


def render_backward(proj, g, cam, gC, gD, gM=None, gT=None, bg=(0.0, 0.0, 0.0), pixels=None):
    """Reverse mode through `render`. Returns the planar [10, n] 2D adjoint
    (u_x, u_y, k1, k2, k3, opacity, c_r, c_g, c_b, depth)."""
    n = g["opacity_logit"].shape[0]
    W, H = cam["width"], cam["height"]
    if pixels is None:
        npix, pix = -1, np.zeros(1, np.int64)
    else:
        pix = np.ascontiguousarray(pixels, dtype=np.int64)
        npix = pix.shape[0]
    P = W * H if pixels is None else npix
    gC, gD = _d(gC).reshape(3 * P), _d(gD).reshape(P)
    gM = _d(np.zeros(P) if gM is None else gM)
    gT = _d(np.zeros(P) if gT is None else gT)
    g2d = np.zeros((10, n))
    kept = np.ascontiguousarray(proj["kept"], np.uint8)
    color, mp, bgv = _d(g["color"]), _d(g["mp"]), _d(bg)
    lib().or_render_backward(n, _p(proj["mean2d"]), _p(proj["conic"]), _p(proj["depth"]), _p(proj["zkey"]),
                             _p(proj["opacity"]),
                             _p(color), _p(mp), _p(kept), W, H, _p(bgv), npix, _p(pix), _p(gC), _p(gD),
                             _p(gM), _p(gT), _p(g2d))
    return g2d


def project_backward(g: dict, cam: dict, g2d) -> dict:
    """Chain the 2D adjoint through the projection to the Gaussian parameters
    and the pose twist xi = (rho, phi), left perturbation T <- Exp(xi) T."""
    n = g["opacity_logit"].shape[0]
    mean, ls, q, opl = _d(g["mean"]), _d(g["log_scale"]), _d(g["quat"]), _d(g["opacity_logit"])
    out = dict(mean=np.zeros((3, n)), log_scale=np.zeros((3, n)), quat=np.zeros((4, n)),
               opacity_logit=np.zeros(n), color=np.zeros((3, n)), pose=np.zeros(6))
    g2 = _d(g2d)
    lib().or_project_backward(n, _p(mean), _p(ls), _p(q), _p(opl), _p(cam_vector(cam)), _p(g2),
                              _p(out["mean"]), _p(out["log_scale"]), _p(out["quat"]), _p(out["opacity_logit"]),
                              _p(out["color"]), _p(out["pose"]))
    return out


# ------------------------------------------------------------------ loss
def loss(img: dict, target_color, target_depth, lambda_pho=0.9, lambda_depth=0.1, eps_A=1e-6,
         weight_mode=0, grad_through_weight=False, w_fixed=None) -> dict:
    """MP-weighted L1 losses.

    Static weight, Eq. (20): w = sum_k omega_k (1 - M_k) with omega_k the
    compositing weights normalised to sum to one, i.e. w = 1 - M/A with
    A = 1 - T (weight_mode 0); w = 0 where A <= eps_A. weight_mode 1 uses the
    unnormalised sum A - M. L = lambda1 sum_u w |C - C_gt|_1
    + lambda2 sum_u w [D_gt > 0] |D - D_gt|  (Eq. (21), (22), (27); sums, not
    means). Adjoints use sign(0) = 0. `w_fixed` holds w constant (it is
    detached unless grad_through_weight)."""
    C, D, M, T = (np.asarray(img[k], np.float64) for k in ("C", "D", "M", "T"))
    Cg = np.asarray(target_color, np.float64)
    Dg = np.asarray(target_depth, np.float64)
    A = 1.0 - T
    if weight_mode == 0:
        ok = A > eps_A
        Asafe = np.where(ok, A, 1.0)
        w = np.where(ok, 1.0 - M / Asafe, 0.0)
    else:
        ok = np.ones_like(A, bool)
        Asafe = A
        w = A - M
    if w_fixed is not None:
        w = np.asarray(w_fixed, np.float64)
    valid = Dg > 0
    rc = C - Cg
    rd = np.where(valid, D - Dg, 0.0)
    per_px = lambda_pho * np.abs(rc).sum(axis=0) + lambda_depth * np.abs(rd)
    L = float((w * per_px).sum())
    dC = lambda_pho * w[None, :] * np.sign(rc)
    dD = lambda_depth * w * np.sign(rd)
    dM = np.zeros_like(D)
    dT = np.zeros_like(D)
    if grad_through_weight:
        gw = per_px
        if weight_mode == 0:
            dM = np.where(ok, -gw / Asafe, 0.0)
            dT = np.where(ok, -gw * M / (Asafe * Asafe), 0.0)
        else:
            dM = -gw
            dT = -gw
    return dict(loss=L, w=w, dC=dC, dD=dD, dM=dM, dT=dT)


def forward_loss(g: dict, cam: dict, target_color, target_depth, w_fixed=None, bg=(0, 0, 0), **kw) -> float:
    """Projection + render + loss in FP64, for finite differences."""
    pr = project(g, cam)
    im = render(pr, g, cam, bg=bg)
    return loss(im, target_color, target_depth, w_fixed=w_fixed, **kw)["loss"]


def full_backward(g: dict, cam: dict, target_color, target_depth, bg=(0, 0, 0), **kw):
    """Forward, loss and the complete adjoint. Returns (loss dict, image, grads)."""
    pr = project(g, cam)
    im = render(pr, g, cam, bg=bg)
    L = loss(im, target_color, target_depth, **kw)
    g2d = render_backward(pr, g, cam, L["dC"], L["dD"], L["dM"], L["dT"], bg=bg)
    grads = project_backward(g, cam, g2d)
    return L, im, grads, pr, g2d


# ------------------------------------------------------------------ binning reference
def bin_reference(rect, key, tile_grid, tile_base=0):
    """Per-tile lists from the textbook stable sort: for every non-empty
    record k (in index order) and every tile of its inclusive rectangle (row-
    major), emit key64 = (tile << 32) | depth_bits with value k; sort stably by
    key64. rect is [m, 4] int16 (x0, y0, x1, y1), key uint32 (0xFFFFFFFF =
    culled). Returns (ids uint32 [I], ranges int64 [T, 2])."""
    gx, gy = tile_grid
    rect = np.asarray(rect).astype(np.int64)
    key = np.asarray(key, np.uint32)
    keys, vals = [], []
    for k in range(rect.shape[0]):
        if key[k] == 0xFFFFFFFF:
            continue
        x0, y0, x1, y1 = rect[k]
        for ty in range(y0, y1 + 1):
            for tx in range(x0, x1 + 1):
                t = tile_base + ty * gx + tx
                keys.append((t << 32) | int(key[k]))
                vals.append(k)
    keys = np.array(keys, dtype=np.uint64)
    vals = np.array(vals, dtype=np.uint32)
    order = np.argsort(keys, kind="stable")
    keys, vals = keys[order], vals[order]
    T = gx * gy
    tiles = (keys >> np.uint64(32)).astype(np.int64) - tile_base
    ranges = np.zeros((T, 2), np.int64)
    b = np.searchsorted(tiles, np.arange(T), side="left")
    e = np.searchsorted(tiles, np.arange(T), side="right")
    ranges[:, 0], ranges[:, 1] = b, e
    return vals, ranges


def bin_reference_np(rect, key, tile_grid, tile_base=0):
    """The same per-tile lists as `bin_reference`, built with array
    operations so that tens of millions of instances fit in seconds: every
    non-empty record expanded over its rectangle, then numpy's stable sort of
    the (tile << 32 | depth bits) keys."""
    gx, gy = tile_grid
    rect = np.asarray(rect).astype(np.int64)
    key = np.asarray(key, np.uint32)
    ok = key != 0xFFFFFFFF
    rid = np.nonzero(ok)[0]
    x0, y0, x1, y1 = (rect[rid, c] for c in range(4))
    w = x1 - x0 + 1
    cnt = w * (y1 - y0 + 1)
    rec = np.repeat(rid, cnt)
    start = np.cumsum(cnt) - cnt
    j = np.arange(rec.size, dtype=np.int64) - np.repeat(start, cnt)  # index inside the record's rect
    wr = np.repeat(w, cnt)
    tx = np.repeat(x0, cnt) + j % wr
    ty = np.repeat(y0, cnt) + j // wr
    tiles = tile_base + ty * gx + tx
    keys = (tiles.astype(np.uint64) << np.uint64(32)) | key[rec].astype(np.uint64)
    order = np.argsort(keys, kind="stable")
    vals = rec[order].astype(np.uint32)
    st = np.sort(tiles) - tile_base
    T = gx * gy
    ranges = np.stack([np.searchsorted(st, np.arange(T), side="left"),
                       np.searchsorted(st, np.arange(T), side="right")], axis=1).astype(np.int64)
    return vals, ranges


def compact(planes, drop, seg_begin=None):
    """Removal of the Gaussians flagged in `drop` (the prune of the mapping
    window, MP above its threshold): every plane keeps its remaining elements
    in their order. Returns (planes, new segment offsets) where segments are
    the contiguous scenes given by seg_begin (S + 1 offsets)."""
    keep = ~np.asarray(drop, bool)
    out = [np.asarray(p)[..., keep] for p in planes]
    if seg_begin is None:
        seg_begin = [0, keep.size]
    before = np.concatenate([[0], np.cumsum(keep)])
    return out, before[np.asarray(seg_begin, np.int64)]


from . import mp as mp  # noqa: E402
from . import mlp as mlp  # noqa: E402
