"""Seeded synthetic inputs shaped like the paper's 640x480 RGB-D workloads.

The paper evaluates on TUM RGB-D fr3/walking and BONN (Sec. V-A); neither is
available here, so scenes are drawn from fixed distributions instead: static
Gaussians uniform in the camera frustum volume (depth 0.5-4 m), plus
axis-aligned boxes that move between frames (the dynamic objects).

This module holds none of the method's arithmetic (no projection, rendering,
loss or MP update). It only draws parameters, camera poses, masks and
per-pixel fields with numpy's PCG64, so the oracle and the GPU path can be fed
bit-identical inputs. Every array it returns is float32/int32/uint32.
"""

from __future__ import annotations

import numpy as np

Z_NEAR = 0.2


def rng_for(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


def intrinsics(width: int, height: int):
    """Pinhole intrinsics with the same field of view at every resolution:
    fx = fy = W / 1.28, principal point at the image centre (64x48 gives 50, 32, 24)."""
    f = width / 1.28
    return f, f, width / 2.0, height / 2.0


def camera(width: int, height: int, T_cw=None) -> dict:
    fx, fy, cx, cy = intrinsics(width, height)
    if T_cw is None:
        T_cw = np.concatenate([np.eye(3), np.zeros((3, 1))], axis=1)
    return dict(width=int(width), height=int(height), fx=fx, fy=fy, cx=cx, cy=cy,
                z_near=Z_NEAR, T_cw=np.asarray(T_cw, dtype=np.float32).reshape(3, 4))


def _axis_angle_matrix(axis, angle):
    axis = np.asarray(axis, dtype=np.float64)
    axis = axis / np.linalg.norm(axis)
    x, y, z = axis
    K = np.array([[0, -z, y], [z, 0, -x], [-y, x, 0]])
    return np.eye(3) + np.sin(angle) * K + (1 - np.cos(angle)) * (K @ K)


def perturbed_pose(rng, deg=1.0, trans=0.02, base=None):
    """A pose offset from `base` by `deg` degrees about a random axis and `trans`
    metres along a random direction (both applied on the world->camera side)."""
    if base is None:
        base = np.concatenate([np.eye(3), np.zeros((3, 1))], axis=1)
    base = np.asarray(base, dtype=np.float64)
    axis = rng.normal(size=3)
    R = _axis_angle_matrix(axis, np.deg2rad(deg))
    d = rng.normal(size=3)
    d = trans * d / np.linalg.norm(d)
    Rn = R @ base[:, :3]
    tn = R @ base[:, 3] + d
    return np.concatenate([Rn, tn[:, None]], axis=1).astype(np.float32)


def _depth_volume_uniform(rng, n, zmin, zmax):
    # density proportional to z^2 on [zmin, zmax]: uniform in frustum volume
    u = rng.random(n)
    return np.cbrt(zmin ** 3 + u * (zmax ** 3 - zmin ** 3))


def static_gaussians(rng, n, width, height, zmin=0.5, zmax=4.0, mp=None, margin=0.0) -> dict:
    """n Gaussians seen by an identity-pose camera: pixel position uniform in the
    image (widened by `margin` x the image size on every side, for scenes that
    later views see beyond the first one), depth uniform in volume, log-scale
    N(-3, 0.5^2) per axis, random unit quaternion (w,x,y,z), opacity logit
    N(0,1), RGB U[0,1], MP U[0,1]."""
    fx, fy, cx, cy = intrinsics(width, height)
    px = (rng.random(n) * (1 + 2 * margin) - margin) * width
    py = (rng.random(n) * (1 + 2 * margin) - margin) * height
    z = _depth_volume_uniform(rng, n, zmin, zmax)
    mean = np.stack([z * (px - cx) / fx, z * (py - cy) / fy, z])
    log_scale = rng.normal(-3.0, 0.5, size=(3, n))
    q = rng.normal(size=(4, n))
    q /= np.linalg.norm(q, axis=0, keepdims=True)
    opl = rng.normal(0.0, 1.0, size=n)
    color = rng.random((3, n))
    m = rng.random(n) if mp is None else np.full(n, mp)
    return _pack(mean, log_scale, q, opl, color, m)


def _pack(mean, log_scale, quat, opl, color, mp):
    f = np.float32
    return dict(mean=np.ascontiguousarray(mean, f), log_scale=np.ascontiguousarray(log_scale, f),
                quat=np.ascontiguousarray(quat, f), opacity_logit=np.ascontiguousarray(opl, f),
                color=np.ascontiguousarray(color, f), mp=np.ascontiguousarray(mp, f))


def concat_gaussians(parts) -> dict:
    keys = ["mean", "log_scale", "quat", "opacity_logit", "color", "mp"]
    return {k: np.ascontiguousarray(np.concatenate([p[k] for p in parts], axis=-1)) for k in keys}


def n_gaussians(g) -> int:
    return int(g["opacity_logit"].shape[0])


# ---------------------------------------------------------------- moving boxes
def random_boxes(rng, n_boxes, width, height):
    """Axis-aligned boxes, sides U[0.2, 0.5] m, centre depth U[1, 3] m, centre
    pixel uniform in the inner 80% of the image (identity-pose camera)."""
    fx, fy, cx, cy = intrinsics(width, height)
    boxes = []
    for _ in range(n_boxes):
        z = rng.uniform(1.0, 3.0)
        px = rng.uniform(0.1, 0.9) * width
        py = rng.uniform(0.1, 0.9) * height
        centre = np.array([z * (px - cx) / fx, z * (py - cy) / fy, z])
        sides = rng.uniform(0.2, 0.5, size=3)
        base = rng.random(3)
        boxes.append(dict(centre=centre, sides=sides, color=base))
    return boxes


def box_gaussians(rng, box, n) -> dict:
    """n Gaussians with means uniform on the box faces, log-scale N(-4, 0.3^2),
    opacity logit N(4, 0.5^2), colour = box base colour + N(0, 0.02^2), MP = 1."""
    c, s = box["centre"], box["sides"]
    face = rng.integers(0, 6, size=n)
    axis = face // 2
    sign = np.where(face % 2 == 0, -1.0, 1.0)
    local = (rng.random((3, n)) - 0.5) * s[:, None]
    local[axis, np.arange(n)] = sign * s[axis] / 2
    mean = c[:, None] + local
    log_scale = rng.normal(-4.0, 0.3, size=(3, n))
    q = rng.normal(size=(4, n))
    q /= np.linalg.norm(q, axis=0, keepdims=True)
    opl = rng.normal(4.0, 0.5, size=n)
    color = np.clip(box["color"][:, None] + rng.normal(0, 0.02, size=(3, n)), 0, 1)
    return _pack(mean, log_scale, q, opl, color, np.ones(n))


def move_boxes(rng, boxes):
    """Each box moves U[0.05, 0.20] m along a random signed coordinate axis."""
    out = []
    for b in boxes:
        d = np.zeros(3)
        d[rng.integers(0, 3)] = rng.choice([-1.0, 1.0]) * rng.uniform(0.05, 0.20)
        nb = dict(b)
        nb["centre"] = b["centre"] + d
        out.append(nb)
    return out


def translate_gaussians(g, sl, delta) -> dict:
    out = {k: v.copy() for k, v in g.items()}
    out["mean"][:, sl] += np.asarray(delta, dtype=np.float32)[:, None]
    return out


# ---------------------------------------------------------------- configurations
def tiny_scene(seed=1, n=2000, width=64, height=48):
    """64x48 pinhole (fx=fy=50, cx=32, cy=24), 2,000 Gaussians; the target view
    is 1 degree about a random axis and 2 cm away from the rendered view."""
    rng = rng_for(seed)
    g = static_gaussians(rng, n, width, height)
    cam = camera(width, height)
    target_cam = camera(width, height, perturbed_pose(rng))
    return g, cam, target_cam


def moving_box_scene(seed, n, width, height, n_boxes=3, box_frac=0.05, margin=0.0, zmin=0.5, zmax=4.0):
    """Static Gaussians (depth on [zmin, zmax]) plus `n_boxes` boxes that hold
    `box_frac` of the Gaussians. Returns (gaussians, camera, target camera,
    target gaussians, box slices); the target copy has the boxes moved, as in
    a new frame."""
    rng = rng_for(seed)
    nb_total = int(round(n * box_frac)) if n_boxes > 0 else 0
    g_static = static_gaussians(rng, n - nb_total, width, height, margin=margin, zmin=zmin, zmax=zmax)
    parts, slices, start = [g_static], [], n - nb_total
    boxes = random_boxes(rng, n_boxes, width, height)
    per = [nb_total // max(n_boxes, 1)] * n_boxes
    if n_boxes:
        per[-1] += nb_total - sum(per)
    for b, k in zip(boxes, per):
        parts.append(box_gaussians(rng, b, k))
        slices.append(slice(start, start + k))
        start += k
    g = concat_gaussians(parts)
    g["mp"][: n - nb_total] = rng.random(n - nb_total).astype(np.float32)
    moved = move_boxes(rng, boxes)
    g_target = g
    for b0, b1, sl in zip(boxes, moved, slices):
        g_target = translate_gaussians(g_target, sl, b1["centre"] - b0["centre"])
    cam = camera(width, height)
    # camera motion per frame: 1 cm and 0.5 degree in random directions
    target_cam = camera(width, height, perturbed_pose(rng, deg=0.5, trans=0.01))
    return g, cam, target_cam, g_target, slices


def window_cameras(seed, n_views, width, height, spacing=5):
    """Keyframe poses along a random walk of 1 cm / 0.5 degree per frame,
    one keyframe every `spacing` frames."""
    rng = rng_for(seed)
    pose = np.concatenate([np.eye(3), np.zeros((3, 1))], axis=1)
    cams = []
    for v in range(n_views):
        cams.append(camera(width, height, pose))
        for _ in range(spacing):
            pose = perturbed_pose(rng, deg=0.5, trans=0.01, base=pose)
    return cams


def box_sequence(seed, n, width, height, n_frames, n_boxes=3, box_frac=0.05, spacing=1, zmin=0.5, zmax=4.0,
                 materialize=True):
    """A moving-box sequence: the map (the scene at frame 0, boxes at their
    first positions), and per frame the camera pose (a random walk of 1 cm /
    0.5 degree per frame) and the observed scene, whose boxes keep moving
    U[0.05, 0.20] m along a random signed axis per frame. Returns
    dict(map=gaussians, cams=[...], obs=[gaussians per frame], slices=[box
    slices], dynamic=bool[n] ground-truth flags (box Gaussians), deltas=[per
    frame, the translation of each box from the map]). Static depths are
    drawn on [zmin, zmax]. With materialize=False the observed Gaussians are
    not built (obs is None): large sequences apply `deltas` to the map's box
    slices instead."""
    rng = rng_for(seed)
    nb_total = int(round(n * box_frac)) if n_boxes > 0 else 0
    g_static = static_gaussians(rng, n - nb_total, width, height, zmin=zmin, zmax=zmax)
    parts, slices, start = [g_static], [], n - nb_total
    boxes = random_boxes(rng, n_boxes, width, height)
    per = [nb_total // max(n_boxes, 1)] * n_boxes
    if n_boxes:
        per[-1] += nb_total - sum(per)
    for b, k in zip(boxes, per):
        parts.append(box_gaussians(rng, b, k))
        slices.append(slice(start, start + k))
        start += k
    g0 = concat_gaussians(parts)
    g0["mp"][:] = np.float32(0.5)  # no prior knowledge of the state
    dynamic = np.zeros(n, bool)
    for sl in slices:
        dynamic[sl] = True
    cams, obs, deltas = [], [], []
    pose = np.concatenate([np.eye(3), np.zeros((3, 1))], axis=1)
    cur = boxes
    for t in range(n_frames):
        for _ in range(spacing):
            pose = perturbed_pose(rng, deg=0.5, trans=0.01, base=pose)
            cur = move_boxes(rng, cur)
        deltas.append([np.asarray(b1["centre"] - b0["centre"], np.float64) for b0, b1 in zip(boxes, cur)])
        cams.append(camera(width, height, pose))
        if materialize:
            g_t = g0
            for d, sl in zip(deltas[-1], slices):
                g_t = translate_gaussians(g_t, sl, d)
            obs.append(g_t)
    return dict(map=g0, cams=cams, obs=obs if materialize else None, slices=slices, dynamic=dynamic, deltas=deltas)


# ---------------------------------------------------------------- MP-update inputs
def mp_frame_inputs(seed, n, width, height, n_inst=3, invalid_frac=0.05, cull_frac=0.05):
    """Per-pixel and per-Gaussian inputs of one MP update, drawn directly:
    rendered depth/colour, observed depth (with holes = 0), an instance-id map of
    `n_inst` rectangles, per-instance prior/confidence tables, projected means
    (some outside the image), a culled flag and the previous MP state."""
    rng = rng_for(seed)
    P = width * height
    yy, xx = np.mgrid[0:height, 0:width]
    depth = (1.0 + 2.0 * rng.random()) + 0.3 * np.sin(xx / 7.0 + rng.random() * 6) * np.cos(yy / 5.0)
    depth = depth + rng.normal(0, 0.01, size=depth.shape)
    inst = np.zeros((height, width), np.int32)
    obs = depth + rng.normal(0, 0.01, size=depth.shape)
    for k in range(1, n_inst + 1):
        w = rng.integers(max(2, width // 8), max(3, width // 3))
        h = rng.integers(max(2, height // 8), max(3, height // 3))
        x0 = rng.integers(0, width - w)
        y0 = rng.integers(0, height - h)
        inst[y0:y0 + h, x0:x0 + w] = k
        # a moving object: the observation differs from the render inside it
        obs[y0:y0 + h, x0:x0 + w] += rng.uniform(0.05, 0.2) * (1 + 0.5 * rng.random((h, w)))
    holes = rng.random(depth.shape) < invalid_frac
    obs[holes] = 0.0
    color = rng.random((3, height, width))
    tcolor = np.clip(color + rng.normal(0, 0.05, size=color.shape), 0, 1)
    prior = np.concatenate([[0.05], rng.uniform(0.6, 0.95, size=n_inst)])
    conf = np.concatenate([[0.1], rng.uniform(0.5, 0.95, size=n_inst)])
    mean2d = np.stack([rng.uniform(-3, width + 3, size=n), rng.uniform(-3, height + 3, size=n)])
    culled = rng.random(n) < cull_frac
    mp_prev = rng.random(n)
    f = np.float32
    return dict(width=width, height=height,
                depth=np.ascontiguousarray(depth.reshape(P), f),
                color=np.ascontiguousarray(color.reshape(3, P), f),
                target_depth=np.ascontiguousarray(obs.reshape(P), f),
                target_color=np.ascontiguousarray(tcolor.reshape(3, P), f),
                instance_id=np.ascontiguousarray(inst.reshape(P), np.int32),
                inst_prior=prior.astype(f), inst_conf=conf.astype(f),
                mean2d=np.ascontiguousarray(mean2d, f),
                culled=culled, mp=mp_prev.astype(f))


def bin_inputs(seed, m, width, height, tile=16, cull_frac=0.1, max_tiles=6):
    """Synthetic per-Gaussian binning inputs: an inclusive tile rectangle and a
    depth key (IEEE bits of a positive float depth, 0xFFFFFFFF when culled).
    Depths are drawn on a coarse grid so equal keys (ties) occur."""
    rng = rng_for(seed)
    gx = (width + tile - 1) // tile
    gy = (height + tile - 1) // tile
    x0 = rng.integers(-2, gx + 1, size=m)
    y0 = rng.integers(-2, gy + 1, size=m)
    x1 = x0 + rng.integers(0, max_tiles, size=m)
    y1 = y0 + rng.integers(0, max_tiles, size=m)
    x0c, y0c = np.maximum(x0, 0), np.maximum(y0, 0)
    x1c, y1c = np.minimum(x1, gx - 1), np.minimum(y1, gy - 1)
    z = (0.5 + np.floor(rng.random(m) * 512) / 128.0).astype(np.float32)
    key = z.view(np.uint32).copy()
    culled = rng.random(m) < cull_frac
    empty = (x0c > x1c) | (y0c > y1c) | culled
    key[empty] = 0xFFFFFFFF
    rect = np.stack([x0c, y0c, x1c, y1c]).astype(np.int16)
    rect[0, empty] = 1
    rect[2, empty] = 0
    rect[1, empty] = 1
    rect[3, empty] = 0
    return np.ascontiguousarray(rect.T), key


def mlp_inputs(seed, P, hidden=32, n_in=8):
    """Per-pixel MLP features and labels in plausible ranges, plus FP32 master
    weights drawn with a He-style scale."""
    rng = rng_for(seed)
    x = rng.normal(0, 1, size=(n_in, P)).astype(np.float32)
    label = rng.random(P).astype(np.float32)
    W1 = (rng.normal(0, 1, (hidden, n_in)) * np.sqrt(2.0 / n_in)).astype(np.float32)
    b1 = (rng.normal(0, 0.1, hidden)).astype(np.float32)
    W2 = (rng.normal(0, 1, (hidden, hidden)) * np.sqrt(2.0 / hidden)).astype(np.float32)
    b2 = (rng.normal(0, 0.1, hidden)).astype(np.float32)
    W3 = (rng.normal(0, 1, (1, hidden)) * np.sqrt(1.0 / hidden)).astype(np.float32)
    b3 = np.zeros(1, np.float32)
    return x, label, dict(W1=W1, b1=b1, W2=W2, b2=b2, W3=W3, b3=b3)


# ---------------------------------------------------------------- epipolar matches
def _pixels(cam, X):
    """Pinhole pixels of world points X [3][m] (any depth sign)."""
    T = np.asarray(cam["T_cw"], dtype=np.float64)
    Xc = T[:, :3] @ X + T[:, 3:4]
    return np.stack([cam["fx"] * Xc[0] / Xc[2] + cam["cx"], cam["fy"] * Xc[1] / Xc[2] + cam["cy"]])


def epipolar_case(seed, n, width, height, n_cand, per=(0, 24), noise_px=0.3, outlier_frac=0.1, spacing=5,
                  n_boxes=3, box_frac=0.05, suppressed_frac=0.6):
    """Feature matches of candidate Gaussians between two keyframes `spacing`
    frames apart (1 cm / 0.5 degree per frame), in a moving-box scene whose
    boxes move U[0.05, 0.20] m between them. Candidates: a third box
    Gaussians, two thirds static ones; MP is U[0.6, 1] for box candidates and
    for a `suppressed_frac` share of the static candidates (those MP wrongly
    suppresses), U[0, 0.4] otherwise. Each candidate has k ~ U{per[0] ..
    per[1]} matches: points drawn around its mean (normal, its largest scale)
    carried by the Gaussian's own motion and seen by both pinholes; frame-2
    pixels get N(0, noise_px^2) noise and a share `outlier_frac` of them is
    replaced by uniform pixels. Returns dict(cam1, cam2, ids int32 [K], seg
    int64 [K+1], p1, p2 float32 [2][m], mp float32 [n], dynamic bool [n])."""
    rng = rng_for(seed)
    seq = box_sequence(seed, n, width, height, 1, n_boxes=n_boxes, box_frac=box_frac, spacing=spacing)
    cam2 = seq["cams"][0]
    cam1 = camera(width, height)
    g0, g1, dyn = seq["map"], seq["obs"][0], seq["dynamic"]
    nb = int(min(n_cand // 3, dyn.sum()))
    box_ids = rng.choice(np.nonzero(dyn)[0], size=nb, replace=False)
    st_ids = rng.choice(np.nonzero(~dyn)[0], size=n_cand - nb, replace=False)
    ids = rng.permutation(np.concatenate([box_ids, st_ids])).astype(np.int32)
    mp = rng.uniform(0.0, 0.4, n).astype(np.float32)
    hi = dyn.copy()
    hi[st_ids[rng.random(st_ids.size) < suppressed_frac]] = True
    mp[hi] = rng.uniform(0.6, 1.0, int(hi.sum())).astype(np.float32)
    p1, p2, seg = frame_matches(rng, g0, g1, cam1, cam2, ids, per, noise_px, outlier_frac)
    return dict(cam1=cam1, cam2=cam2, ids=ids, seg=seg, p1=p1, p2=p2, mp=mp, dynamic=dyn)


def frame_matches(rng, g_a, g_b, cam_a, cam_b, ids, per=(4, 16), noise_px=0.3, outlier_frac=0.1):
    """Feature matches of Gaussians `ids` between frames a and b: k ~ U{per[0]
    .. per[1]} points each, drawn around the Gaussian's mean in g_a (normal,
    its largest scale) and carried by its motion to g_b, seen by both
    pinholes; frame-b pixels get N(0, noise_px^2) noise and a share
    `outlier_frac` is replaced by uniform pixels. Returns p1, p2 float32
    [2][m] and the segment offsets int64 [K + 1]."""
    counts = rng.integers(per[0], per[1] + 1, size=len(ids))
    seg = np.concatenate([[0], np.cumsum(counts)]).astype(np.int64)
    owner = np.repeat(np.asarray(ids, np.int64), counts)
    m = owner.size
    sig = np.exp(g_a["log_scale"][:, owner].astype(np.float64).max(axis=0))
    Xa = g_a["mean"][:, owner].astype(np.float64) + rng.normal(size=(3, m)) * sig
    Xb = Xa + (g_b["mean"][:, owner].astype(np.float64) - g_a["mean"][:, owner].astype(np.float64))
    p1 = _pixels(cam_a, Xa)
    p2 = _pixels(cam_b, Xb) + rng.normal(0.0, noise_px, size=(2, m))
    out = rng.random(m) < outlier_frac
    p2[0, out] = rng.uniform(0, cam_b["width"], int(out.sum()))
    p2[1, out] = rng.uniform(0, cam_b["height"], int(out.sum()))
    return p1.astype(np.float32), p2.astype(np.float32), seg


def box_masks(cam, g, slices, margin_px=2):
    """Instance-id map of a synthetic detector: box k is the axis-aligned
    rectangle of its Gaussians' pixels (those in front of the camera), grown
    by `margin_px` and clipped to the image; later boxes overwrite earlier
    ones. int32 [H * W]."""
    W, H = cam["width"], cam["height"]
    out = np.zeros((H, W), np.int32)
    T = np.asarray(cam["T_cw"], dtype=np.float64)
    for k, sl in enumerate(slices, start=1):
        X = g["mean"][:, sl].astype(np.float64)
        Xc = T[:, :3] @ X + T[:, 3:4]
        ok = Xc[2] > cam["z_near"]
        if not ok.any():
            continue
        u = cam["fx"] * Xc[0, ok] / Xc[2, ok] + cam["cx"]
        v = cam["fy"] * Xc[1, ok] / Xc[2, ok] + cam["cy"]
        x0, x1 = int(np.floor(u.min())) - margin_px, int(np.ceil(u.max())) + margin_px
        y0, y1 = int(np.floor(v.min())) - margin_px, int(np.ceil(v.max())) + margin_px
        x0, y0, x1, y1 = max(x0, 0), max(y0, 0), min(x1, W - 1), min(y1, H - 1)
        if x0 <= x1 and y0 <= y1:
            out[y0:y1 + 1, x0:x1 + 1] = k
    return out.reshape(-1)


def mp_sequence_inputs(seed, n, width, height, frames, n_inst=3, speed_px=3.0, k_cand=400, burst=(4, 5, 11)):
    """A sequence of MP-update inputs: one background depth/colour, `n_inst`
    rectangular objects that move `speed_px` pixels per frame (the observed
    depth differs from the render inside their current rectangles, which are
    also the frame's fresh instance masks), projected means that drift by a
    small camera motion, and per frame the median epipolar distances and
    states of `k_cand` verification candidates (distances |N(0, 0.3^2)| px,
    |N(0, 6^2)| px at the frames in `burst`, a tenth without matches). The
    first frame carries the starting MP state."""
    rng = rng_for(seed)
    P = width * height
    yy, xx = np.mgrid[0:height, 0:width]
    depth = (1.0 + 2.0 * rng.random()) + 0.3 * np.sin(xx / 7.0 + rng.random() * 6) * np.cos(yy / 5.0)
    color = rng.random((3, height, width))
    boxes = []
    for _ in range(n_inst):
        w = int(rng.integers(max(2, width // 8), max(3, width // 3)))
        h = int(rng.integers(max(2, height // 8), max(3, height // 3)))
        boxes.append(dict(x=float(rng.uniform(0, width - w)), y=float(rng.uniform(0, height - h)), w=w, h=h,
                          vx=float(rng.choice([-1, 1]) * speed_px), vy=float(rng.uniform(-1, 1) * speed_px),
                          dz=float(rng.uniform(0.05, 0.2))))
    prior = np.concatenate([[0.05], rng.uniform(0.6, 0.95, size=n_inst)]).astype(np.float32)
    conf = np.concatenate([[0.1], rng.uniform(0.5, 0.95, size=n_inst)]).astype(np.float32)
    mean0 = np.stack([rng.uniform(-3, width + 3, size=n), rng.uniform(-3, height + 3, size=n)])
    culled = rng.random(n) < 0.05
    mp0 = rng.random(n).astype(np.float32)
    drift = rng.normal(0, 0.5, size=2)
    out = []
    f = np.float32
    for t in range(frames):
        r = depth + rng.normal(0, 0.01, size=depth.shape)
        obs = r + rng.normal(0, 0.01, size=depth.shape)
        inst = np.zeros((height, width), np.int32)
        for k, b in enumerate(boxes, start=1):
            x0 = int(np.clip(round(b["x"] + b["vx"] * t), 0, width - b["w"]))
            y0 = int(np.clip(round(b["y"] + b["vy"] * t), 0, height - b["h"]))
            inst[y0:y0 + b["h"], x0:x0 + b["w"]] = k
            obs[y0:y0 + b["h"], x0:x0 + b["w"]] += b["dz"]
        obs[rng.random(depth.shape) < 0.05] = 0.0
        tcolor = np.clip(color + rng.normal(0, 0.05, size=color.shape), 0, 1)
        sd = 6.0 if t in burst else 0.3
        dbar = np.abs(rng.normal(0, sd, size=k_cand)).astype(f)
        est = rng.choice([2, 2, 2, 2, 2, 2, 0, 1, 3, 2], size=k_cand).astype(np.uint8)
        dbar[est == 3] = np.nan
        out.append(dict(width=width, height=height,
                        depth=np.ascontiguousarray(r.reshape(P), f),
                        color=np.ascontiguousarray(color.reshape(3, P), f),
                        target_depth=np.ascontiguousarray(obs.reshape(P), f),
                        target_color=np.ascontiguousarray(tcolor.reshape(3, P), f),
                        instance_id=np.ascontiguousarray(inst.reshape(P), np.int32),
                        inst_prior=prior, inst_conf=conf,
                        mean2d=np.ascontiguousarray(mean0 + drift[:, None] * t, f),
                        culled=culled, mp=mp0, dbar=dbar, epi_state=est))
    return out
