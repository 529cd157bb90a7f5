"""ctypes binding of libgs.so (include/gs.h), argument marshalling only.

The C structures are mirrored one to one; the functions gs_project,
gs_bin_sort, gs_render_fwd, gs_loss, gs_render_bwd, gs_mp_update (and the
helpers) keep their C names and take those structures. Device memory comes
from torch tensors; every call is enqueued on torch's current HIP stream
unless a stream handle is given. `Pipeline` allocates the buffers of one view
batch and chains the calls of one optimisation iteration.

There is no fallback: if libgs.so is missing or fails to load, lib() raises.
"""

from __future__ import annotations

import ctypes
import os
from ctypes import POINTER, c_float, c_int32, c_int64, c_size_t, c_uint16, c_void_p

import numpy as np
import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libgs.so")
_lib = None

GS_OK, GS_E_ARG, GS_E_CAPACITY, GS_E_HIP, GS_E_UNSUPPORTED = 0, 1, 2, 3, 4
GS_OP_BIN_SORT, GS_OP_RENDER_BWD, GS_OP_LOSS, GS_OP_MP_UPDATE, GS_OP_MLP_TRAIN, GS_OP_COMPACT = 1, 2, 3, 4, 5, 6
GS_OP_MP_REG, GS_OP_EDGE_WARP = 7, 8
GS_COMPACT_MAX_PLANES, GS_COMPACT_MAX_SEGS = 64, 32
GS_MAX_VIEWS = 32
GS_MLP_PARAMS = 1377
GS_MLP_WEIGHTS = 1312


class GSError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{msg} (status {status})")
        self.status = status


class Camera(ctypes.Structure):
    _fields_ = [("width", c_int32), ("height", c_int32), ("fx", c_float), ("fy", c_float), ("cx", c_float),
                ("cy", c_float), ("z_near", c_float), ("pad_", c_float), ("T_cw", c_float * 12)]


class Views(ctypes.Structure):
    _fields_ = [("n_views", c_int32), ("n_scenes", c_int32), ("n_gaussians", c_int64),
                ("cams_host", POINTER(Camera)), ("cams_dev", c_void_p), ("view_scene", POINTER(c_int32)),
                ("scene_begin", POINTER(c_int64))]


class Gaussians(ctypes.Structure):
    _fields_ = [("n", c_int64)] + [(k, c_void_p) for k in ("mean", "log_scale", "quat", "opacity_logit", "color",
                                                          "mp")]


class Proj(ctypes.Structure):
    _fields_ = [("m", c_int64)] + [(k, c_void_p) for k in ("rec", "rect", "depth_key", "mean2d", "conic", "depth",
                                                          "opacity", "radius", "key_hist")] + [("keys_only", c_int32)]


class Bins(ctypes.Structure):
    _fields_ = [("capacity", c_int64)] + [(k, c_void_p) for k in ("gauss_id", "tile_start", "sorted_ids",
                                                                 "n_instances", "overflow", "incomplete")] + [
        ("max_rank", c_int64), ("truncated", c_void_p), ("sticky", c_void_p)]


class Image(ctypes.Structure):
    _fields_ = [(k, c_void_p) for k in ("color", "depth", "mp", "T", "n_last", "tile_work")]


class Target(ctypes.Structure):
    _fields_ = [("color", c_void_p), ("depth", c_void_p)]


class LossParams(ctypes.Structure):
    _fields_ = [("lambda_pho", c_float), ("lambda_depth", c_float), ("eps_A", c_float), ("weight_mode", c_int32),
                ("grad_through_weight", c_int32)]


class PixelGrads(ctypes.Structure):
    _fields_ = [(k, c_void_p) for k in ("dcolor", "ddepth", "dmp", "dT", "view_weight")]


class Grads(ctypes.Structure):
    _fields_ = [(k, c_void_p) for k in ("mean", "log_scale", "quat", "opacity_logit", "color", "pose")] + [
        ("pose_only", c_int32), ("accumulate", c_int32)]


class MPFrame(ctypes.Structure):
    _fields_ = [("instance_id", c_void_p), ("n_inst", c_int32), ("inst_prior", c_void_p), ("inst_conf", c_void_p),
                ("seg_updated", c_int32), ("mlp_mp", c_void_p)]


MP_PARAM_NAMES = ("lambda_e", "sigma_small", "e_floor", "sigma_g", "sigma_c", "lambda_u", "eps", "alpha_min",
                  "alpha_max", "rho", "radius_px", "sigma_w", "beta_color", "prune_above", "logodds_eps",
                  "logodds_max")


class MPParams(ctypes.Structure):
    _fields_ = [(k, c_float) for k in MP_PARAM_NAMES] + [("mode", c_int32), ("u_norm", c_int32)]


class MPOut(ctypes.Structure):
    _fields_ = [(k, c_void_p) for k in ("U_tilde", "alpha", "dynamic", "prune", "M_p", "e", "stats", "judge")]


class AdamGroup(ctypes.Structure):
    _fields_ = [("param", c_void_p), ("grad", c_void_p), ("m", c_void_p), ("v", c_void_p), ("n", c_int64),
                ("lr", c_float)]


class AdamParams(ctypes.Structure):
    _fields_ = [("beta1", c_float), ("beta2", c_float), ("eps", c_float), ("step", c_int32), ("step_dev", c_void_p),
                ("advance", c_int32)]


class EdgePair(ctypes.Structure):
    _fields_ = [("i", c_int32), ("j", c_int32)]


class EdgeParams(ctypes.Structure):
    _fields_ = [("lambda_", c_float), ("delta", c_float), ("edge_thresh", c_float), ("eps_A", c_float)]


class EpiParams(ctypes.Structure):
    _fields_ = [("eps", c_float), ("tau", c_float), ("mp_restore", c_float)]


GS_EPI_KEPT, GS_EPI_RESTORED, GS_EPI_NOT_SUPPRESSED, GS_EPI_NO_MATCHES, GS_EPI_INVALID = 0, 1, 2, 3, 4


class SchedParams(ctypes.Structure):
    _fields_ = [("w_u", c_float), ("w_r", c_float), ("theta", c_float), ("e_ref", c_float), ("n_max", c_int32)]


class SchedState(ctypes.Structure):
    _fields_ = [("dt", c_int32), ("n_refresh", c_int32), ("S", c_float), ("R", c_float), ("e_bar", c_float)]


SCHED_DEFAULTS = dict(w_u=0.5, w_r=0.5, theta=0.5, e_ref=2.0, n_max=10)


class MLP(ctypes.Structure):
    _fields_ = [(k, c_void_p) for k in ("master", "w_bf16", "adam_m", "adam_v")]


MP_DEFAULTS = dict(lambda_e=2.0, sigma_small=1e-3, e_floor=0.0, sigma_g=0.05, sigma_c=0.05, lambda_u=1.0, eps=1e-6,
                   alpha_min=0.1, alpha_max=0.8, rho=0.5, radius_px=2.0, sigma_w=1.0, beta_color=0.0,
                   prune_above=2.0, logodds_eps=0.01, logodds_max=float(np.log(99.0)), mode=0, u_norm=0)


def lib():
    """Load libgs.so (built by __graft_entry__.build / paper_2602_21644_amd.build)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is not built; run __graft_entry__.build()")
        L = ctypes.CDLL(LIB_PATH)
        P = c_void_p
        sig = {
            "gs_status_str": ([c_int32], ctypes.c_char_p),
            "gs_ctx_create": ([ctypes.c_int, POINTER(c_void_p)], c_int32),
            "gs_ctx_destroy": ([P], c_int32),
            "gs_last_error": ([P], ctypes.c_char_p),
            "gs_ctx_set_param": ([P, ctypes.c_char_p, c_int64], c_int32),
            "gs_ctx_get_param": ([P, ctypes.c_char_p, POINTER(c_int64)], c_int32),
            "gs_ctx_kernel_times": ([P, ctypes.c_char_p, c_size_t], c_int32),
            "gs_rec_offset": ([POINTER(Views), c_int32], c_int64),
            "gs_rec_count": ([POINTER(Views)], c_int64),
            "gs_tile_count": ([POINTER(Views)], c_int64),
            "gs_pixel_count": ([POINTER(Views)], c_int64),
            "gs_workspace_size": ([P, POINTER(Views), c_int32, c_int64, POINTER(c_size_t)], c_int32),
            "gs_project": ([P, POINTER(Views), POINTER(Gaussians), POINTER(Proj), P], c_int32),
            "gs_bin_sort": ([P, POINTER(Views), POINTER(Gaussians), POINTER(Proj), POINTER(Bins), P, c_size_t, P],
                            c_int32),
            "gs_render_fwd": ([P, POINTER(Views), POINTER(Gaussians), POINTER(Proj), POINTER(Bins), POINTER(c_float),
                               POINTER(Image), P], c_int32),
            "gs_loss": ([P, POINTER(Views), POINTER(Image), POINTER(Target), POINTER(LossParams), P,
                         POINTER(PixelGrads), P, c_size_t, P], c_int32),
            "gs_render_fwd_loss": ([P, POINTER(Views), POINTER(Gaussians), POINTER(Proj), POINTER(Bins),
                                    POINTER(c_float), POINTER(Image), POINTER(Target), POINTER(LossParams), P,
                                    POINTER(PixelGrads), P, c_size_t, P], c_int32),
            "gs_render_fwd_loss_static": ([P, POINTER(Views), POINTER(Gaussians), POINTER(Proj), POINTER(Bins),
                                           POINTER(c_float), POINTER(Image), POINTER(Target), POINTER(LossParams), P,
                                           POINTER(PixelGrads), P], c_int32),
            "gs_render_bwd": ([P, POINTER(Views), POINTER(Gaussians), POINTER(Proj), POINTER(Bins), POINTER(Image),
                               POINTER(PixelGrads), POINTER(c_float), POINTER(Grads), P, c_size_t, P], c_int32),
            "gs_bins_check": ([P, POINTER(Bins), POINTER(c_int64), POINTER(c_int32), P], c_int32),
            "gs_mp_update": ([P, POINTER(Views), POINTER(Proj), POINTER(Image), POINTER(Target), POINTER(MPFrame),
                              POINTER(MPParams), P, POINTER(MPOut), P, c_size_t, P], c_int32),
            "gs_mp_regularizer": ([P, c_int64, P, P, P, POINTER(c_float), c_float, P, P, P, c_size_t, P], c_int32),
            "gs_edge_warp": ([P, POINTER(Views), POINTER(Image), POINTER(Target), POINTER(EdgePair), c_int32,
                              POINTER(EdgeParams), P, P, P, P, c_size_t, P], c_int32),
            "gs_epipolar_verify": ([P, POINTER(Views), c_int32, c_int32, P, P, c_int64, P, P, c_int64,
                                    POINTER(EpiParams), P, P, P, P, P], c_int32),
            "gs_sched_decide": ([POINTER(SchedParams), POINTER(SchedState), c_float, P, P, c_int64,
                                 POINTER(c_int32)], c_int32),
            "gs_measure_atomics": ([P, P, c_int64, c_int64, c_int32, P], c_int32),
            "gs_compact": ([P, P, c_int64, c_int32, POINTER(c_void_p), POINTER(c_void_p), POINTER(c_int64), c_int32,
                            P, P, P, c_size_t, P], c_int32),
            "gs_mlp_features": ([P, POINTER(Views), POINTER(Image), POINTER(Target), POINTER(MPFrame), P, P],
                                c_int32),
            "gs_mlp_sync": ([P, POINTER(MLP), P], c_int32),
            "gs_mlp_fwd": ([P, POINTER(MLP), P, P, c_int64, P], c_int32),
            "gs_adam_step": ([P, POINTER(AdamGroup), c_int32, POINTER(AdamParams), P], c_int32),
            "gs_pose_update": ([P, c_int32, P, P, P], c_int32),
            "gs_mlp_train_step": ([P, POINTER(MLP), P, P, c_int64, c_float, c_int32, P, P, P, c_size_t, P],
                                  c_int32),
        }
        for name, (args, res) in sig.items():
            f = getattr(L, name)
            f.argtypes = args
            f.restype = res
        _lib = L
    return _lib


EXPORTED = ("gs_status_str", "gs_ctx_create", "gs_ctx_destroy", "gs_last_error", "gs_ctx_set_param",
            "gs_ctx_get_param", "gs_ctx_kernel_times", "gs_rec_offset", "gs_rec_count", "gs_tile_count", "gs_pixel_count",
            "gs_workspace_size", "gs_project", "gs_bin_sort", "gs_render_fwd", "gs_loss", "gs_render_fwd_loss",
            "gs_render_fwd_loss_static",
            "gs_render_bwd", "gs_bins_check", "gs_mp_update", "gs_compact", "gs_mp_regularizer", "gs_edge_warp",
            "gs_epipolar_verify", "gs_sched_decide", "gs_measure_atomics", "gs_mlp_features", "gs_mlp_sync", "gs_mlp_fwd", "gs_mlp_train_step",
            "gs_adam_step", "gs_pose_update")


def ptr(t):
    return None if t is None else c_void_p(t.data_ptr())


def _stream(stream=None):
    if stream is None:
        stream = torch.cuda.current_stream()
    return c_void_p(stream.cuda_stream if hasattr(stream, "cuda_stream") else int(stream))


class Context:
    def __init__(self, device: int = 0):
        self.h = c_void_p()
        st = lib().gs_ctx_create(device, ctypes.byref(self.h))
        if st != GS_OK:
            raise GSError(st, "gs_ctx_create failed")

    def check(self, st, what):
        if st != GS_OK:
            msg = lib().gs_last_error(self.h).decode()
            raise GSError(st, f"{what}: {lib().gs_status_str(st).decode()}: {msg}")

    def set_param(self, name, value):
        self.check(lib().gs_ctx_set_param(self.h, name.encode(), int(value)), "set_param " + name)

    def get_param(self, name):
        v = c_int64()
        self.check(lib().gs_ctx_get_param(self.h, name.encode(), ctypes.byref(v)), "get_param " + name)
        return v.value

    def kernel_times(self):
        """{kernel: (launches, total_ms)} since the last call (timing mode)."""
        buf = ctypes.create_string_buffer(1 << 16)
        self.check(lib().gs_ctx_kernel_times(self.h, buf, len(buf)), "gs_ctx_kernel_times")
        out = {}
        for line in buf.value.decode().splitlines():
            name, n, ms = line.rsplit(" ", 2)
            out[name] = (int(n), float(ms))
        return out

    def __del__(self):
        try:
            if self.h:
                lib().gs_ctx_destroy(self.h)
        except Exception:
            pass


# ---------------------------------------------------------------- the six calls (C names)
def gs_project(ctx, views, g, proj, stream=None):
    ctx.check(lib().gs_project(ctx.h, ctypes.byref(views), ctypes.byref(g), ctypes.byref(proj), _stream(stream)),
              "gs_project")


def gs_bin_sort(ctx, views, g, proj, bins, ws, stream=None):
    ctx.check(lib().gs_bin_sort(ctx.h, ctypes.byref(views), ctypes.byref(g) if g is not None else None,
                                ctypes.byref(proj), ctypes.byref(bins), ptr(ws), ws.numel() * ws.element_size(),
                                _stream(stream)), "gs_bin_sort")


def gs_render_fwd(ctx, views, g, proj, bins, bg, img, stream=None):
    bgv = (c_float * 3)(*[float(x) for x in bg])
    ctx.check(lib().gs_render_fwd(ctx.h, ctypes.byref(views), ctypes.byref(g), ctypes.byref(proj),
                                  ctypes.byref(bins), bgv, ctypes.byref(img), _stream(stream)), "gs_render_fwd")


def gs_loss(ctx, views, img, tgt, params, loss, pg, ws, stream=None):
    ctx.check(lib().gs_loss(ctx.h, ctypes.byref(views), ctypes.byref(img), ctypes.byref(tgt), ctypes.byref(params),
                            ptr(loss), ctypes.byref(pg), ptr(ws), ws.numel() * ws.element_size(), _stream(stream)),
              "gs_loss")


def gs_render_fwd_loss(ctx, views, g, proj, bins, bg, img, tgt, params, loss, pg, ws, stream=None):
    bgv = (c_float * 3)(*[float(x) for x in bg])
    ctx.check(lib().gs_render_fwd_loss(ctx.h, ctypes.byref(views), ctypes.byref(g), ctypes.byref(proj),
                                       ctypes.byref(bins), bgv, ctypes.byref(img), ctypes.byref(tgt),
                                       ctypes.byref(params), ptr(loss), ctypes.byref(pg), ptr(ws),
                                       ws.numel() * ws.element_size(), _stream(stream)), "gs_render_fwd_loss")


def gs_render_fwd_loss_static(ctx, views, g, proj, bins, bg, img, tgt, params, loss, pg, stream=None):
    bgv = (c_float * 3)(*[float(x) for x in bg])
    ctx.check(lib().gs_render_fwd_loss_static(ctx.h, ctypes.byref(views), ctypes.byref(g), ctypes.byref(proj),
                                              ctypes.byref(bins), bgv, ctypes.byref(img), ctypes.byref(tgt),
                                              ctypes.byref(params), ptr(loss), ctypes.byref(pg), _stream(stream)),
              "gs_render_fwd_loss_static")


def gs_render_bwd(ctx, views, g, proj, bins, img, pg, bg, grads, ws, stream=None):
    bgv = (c_float * 3)(*[float(x) for x in bg])
    ctx.check(lib().gs_render_bwd(ctx.h, ctypes.byref(views), ctypes.byref(g), ctypes.byref(proj),
                                  ctypes.byref(bins), ctypes.byref(img), ctypes.byref(pg), bgv, ctypes.byref(grads),
                                  ptr(ws), ws.numel() * ws.element_size(), _stream(stream)), "gs_render_bwd")


def gs_mp_update(ctx, views, proj, img, tgt, frame, params, mp, out, ws, stream=None):
    ctx.check(lib().gs_mp_update(ctx.h, ctypes.byref(views), ctypes.byref(proj), ctypes.byref(img),
                                 ctypes.byref(tgt), ctypes.byref(frame), ctypes.byref(params), ptr(mp),
                                 ctypes.byref(out), ptr(ws), ws.numel() * ws.element_size(), _stream(stream)),
              "gs_mp_update")


def gs_bins_check(ctx, bins, stream=None):
    req = c_int64()
    inc = c_int32()
    st = lib().gs_bins_check(ctx.h, ctypes.byref(bins), ctypes.byref(req), ctypes.byref(inc), _stream(stream))
    if st not in (GS_OK, GS_E_CAPACITY):
        ctx.check(st, "gs_bins_check")
    return st == GS_E_CAPACITY, int(req.value), int(inc.value)


def gs_workspace_size(ctx, views, op, capacity=0):
    b = c_size_t()
    ctx.check(lib().gs_workspace_size(ctx.h, ctypes.byref(views) if views is not None else None, op, int(capacity),
                                      ctypes.byref(b)),
              "gs_workspace_size")
    return int(b.value)


def gs_mp_regularizer(ctx, mean, mean_prev, mp, loss, dmean, ws, T=None, lam=500.0, stream=None):
    """loss[0] = lam L_MP; adds its gradient into dmean [3, n] (Eq. (23)-(24))."""
    n = int(mp.numel())
    Tp = (c_float * 12)(*[float(x) for x in np.asarray(T, np.float64).reshape(12)]) if T is not None else None
    ctx.check(lib().gs_mp_regularizer(ctx.h, n, ptr(mean), ptr(mean_prev), ptr(mp), Tp, float(lam), ptr(loss),
                                      ptr(dmean), ptr(ws), ws.numel() * ws.element_size(), _stream(stream)),
              "gs_mp_regularizer")


def gs_edge_warp(ctx, views, img, tgt, pairs, loss, ddepth, dpose, ws, lam=300.0, delta=0.05, edge_thresh=0.05,
                 eps_A=1e-6, stream=None):
    """loss[k] = lam L_edge for view pairs (i, j) (Eq. (25)-(26)); adds the
    adjoints into ddepth [P] and dpose [V, 6] (nullable)."""
    arr = (EdgePair * max(len(pairs), 1))(*[EdgePair(int(i), int(j)) for i, j in pairs])
    prm = EdgeParams(float(lam), float(delta), float(edge_thresh), float(eps_A))
    ctx.check(lib().gs_edge_warp(ctx.h, ctypes.byref(views), ctypes.byref(img), ctypes.byref(tgt), arr, len(pairs),
                                 ctypes.byref(prm), ptr(loss), ptr(ddepth), ptr(dpose), ptr(ws),
                                 ws.numel() * ws.element_size(), _stream(stream)), "gs_edge_warp")


def gs_epipolar_verify(ctx, views, view1, view2, p1, p2, ids, seg, mp, d, dbar, state, eps=1.0, tau=0.5,
                       mp_restore=0.0, stream=None):
    """Epipolar verification and static recovery (Eq. (18)-(19)) of candidate
    Gaussians ids (int32 [K]) with matches seg[k] .. seg[k + 1] (int64 [K + 1])
    of pixels p1, p2 (float32 [2, m]) between views view1 and view2: writes the
    distances d [m], the medians dbar [K] and the states state (uint8 [K],
    GS_EPI_*), and sets mp (in/out) of restored candidates to mp_restore."""
    m = int(p1.shape[-1]) if p1.numel() else 0
    prm = EpiParams(float(eps), float(tau), float(mp_restore))
    ctx.check(lib().gs_epipolar_verify(ctx.h, ctypes.byref(views), int(view1), int(view2), ptr(p1), ptr(p2), m,
                                       ptr(ids), ptr(seg), int(ids.numel()), ctypes.byref(prm), ptr(d), ptr(dbar),
                                       ptr(state), ptr(mp), _stream(stream)), "gs_epipolar_verify")


def gs_sched_decide(params, state, U_bar, dbar=None, epi_state=None):
    """Eq. (14)-(16) on the host: whether to refresh the instance prior at this
    frame, from the latest frame uncertainty U_bar and the frame's epipolar
    candidates (numpy dbar float32 [K], epi_state uint8 [K]); updates
    `state` (SchedState) in place and returns the decision."""
    import numpy as np
    if dbar is None:
        dbar = np.zeros(0, np.float32)
        epi_state = np.zeros(0, np.uint8)
    dbar = np.ascontiguousarray(dbar, dtype=np.float32)
    epi_state = np.ascontiguousarray(epi_state, dtype=np.uint8)
    if dbar.size != epi_state.size:
        raise ValueError("dbar and epi_state differ in length")
    out = c_int32(0)
    st = lib().gs_sched_decide(ctypes.byref(params), ctypes.byref(state), float(U_bar),
                               dbar.ctypes.data_as(c_void_p), epi_state.ctypes.data_as(c_void_p), int(dbar.size),
                               ctypes.byref(out))
    if st != 0:
        raise GSError(st, "gs_sched_decide: invalid parameters")
    return bool(out.value)


def gs_measure_atomics(ctx, acc, n_records, n_ops, copies=1, stream=None):
    """Atomic-throughput probe on the backward's accumulation pattern (see the
    header); acc: float32 device tensor of at least copies * n_records * 10."""
    if acc.numel() < copies * n_records * 10:
        raise ValueError("acc too small")
    ctx.check(lib().gs_measure_atomics(ctx.h, ptr(acc), int(n_records), int(n_ops), int(copies), _stream(stream)),
              "gs_measure_atomics")


def sched_params(**kw):
    p = dict(SCHED_DEFAULTS)
    p.update(kw)
    return SchedParams(float(p["w_u"]), float(p["w_r"]), float(p["theta"]), float(p["e_ref"]), int(p["n_max"]))


def sched_state(params):
    return SchedState(int(params.n_max), 0, 0.0, 0.0, 0.0)


def gs_compact(ctx, drop, src, dst, n_out, ws, seg_begin=None, seg_out=None, stream=None):
    """Removes the elements with drop != 0 from every plane of `src` (a list of
    1-D float32 device tensors of one length n) into the planes of `dst`,
    keeping their order; n_out (int64 device tensor [1]) gets the count, and
    with seg_begin (S + 1 host offsets) seg_out (int64 device [S + 1]) the new
    scene offsets."""
    n = int(drop.numel())
    k = len(src)
    sa = (c_void_p * max(k, 1))(*[c_void_p(t.data_ptr()) for t in src])
    da = (c_void_p * max(k, 1))(*[c_void_p(t.data_ptr()) for t in dst])
    for t in list(src) + list(dst):
        if t.dtype != torch.float32 or t.numel() < n or not t.is_contiguous():
            raise GSError(GS_E_ARG, "gs_compact planes must be contiguous float32 of length >= n")
    if seg_begin is not None:
        S = len(seg_begin) - 1
        sb = (c_int64 * (S + 1))(*[int(x) for x in seg_begin])
    else:
        S, sb = 0, None
    ctx.check(lib().gs_compact(ctx.h, ptr(drop), n, k, sa, da, sb, S, ptr(seg_out), ptr(n_out), ptr(ws),
                               ws.numel() * ws.element_size(), _stream(stream)), "gs_compact")


def gs_mlp_features(ctx, views, img, tgt, frame, x, stream=None):
    ctx.check(lib().gs_mlp_features(ctx.h, ctypes.byref(views), ctypes.byref(img), ctypes.byref(tgt),
                                    ctypes.byref(frame), ptr(x), _stream(stream)), "gs_mlp_features")


def gs_mlp_sync(ctx, mlp, stream=None):
    ctx.check(lib().gs_mlp_sync(ctx.h, ctypes.byref(mlp), _stream(stream)), "gs_mlp_sync")


def gs_mlp_fwd(ctx, mlp, x, y, P, stream=None):
    ctx.check(lib().gs_mlp_fwd(ctx.h, ctypes.byref(mlp), ptr(x), ptr(y), int(P), _stream(stream)), "gs_mlp_fwd")


ADAM_MAX_GROUPS = 8


def gs_adam_step(ctx, groups, step, beta1=0.9, beta2=0.999, eps=1e-8, stream=None, advance=False):
    """groups: list of (param, grad, m, v, lr) float32 device tensors of equal
    size; step: the 1-based step count, or an int32 device tensor holding it
    (with advance, the call adds one to it before the step)."""
    arr = (AdamGroup * len(groups))()
    for i, (p_, g_, m_, v_, lr) in enumerate(groups):
        arr[i] = AdamGroup(ptr(p_), ptr(g_), ptr(m_), ptr(v_), p_.numel(), float(lr))
    if isinstance(step, torch.Tensor):
        prm = AdamParams(beta1, beta2, eps, 0, ptr(step), int(bool(advance)))
    else:
        prm = AdamParams(beta1, beta2, eps, int(step), None, 0)
    ctx.check(lib().gs_adam_step(ctx.h, arr, len(groups), ctypes.byref(prm), _stream(stream)), "gs_adam_step")


def gs_pose_update(ctx, views, delta, stream=None):
    """T_cw[v] <- Exp(delta[v]) T_cw[v] in the views' device camera table; delta [V*6] is zeroed."""
    ctx.check(lib().gs_pose_update(ctx.h, views.V, c_void_p(views.cams_dev.data_ptr()), ptr(delta),
                                   _stream(stream)), "gs_pose_update")


def gs_mlp_train_step(ctx, mlp, x, label, P, lr, step, loss, grad, ws, stream=None):
    ctx.check(lib().gs_mlp_train_step(ctx.h, ctypes.byref(mlp), ptr(x), ptr(label), int(P), float(lr), int(step),
                                      ptr(loss), ptr(grad), ptr(ws), ws.numel() * ws.element_size(),
                                      _stream(stream)), "gs_mlp_train_step")


# ---------------------------------------------------------------- host-side helpers
def camera_struct(cam: dict) -> Camera:
    c = Camera()
    c.width, c.height = int(cam["width"]), int(cam["height"])
    c.fx, c.fy, c.cx, c.cy = float(cam["fx"]), float(cam["fy"]), float(cam["cx"]), float(cam["cy"])
    c.z_near = float(cam["z_near"])
    c.T_cw[:] = [float(x) for x in np.asarray(cam["T_cw"], np.float64).reshape(12)]
    return c


class ViewBatch:
    """V cameras over S scenes (packed Gaussians). Holds the host arrays the
    C struct points to and the device copy of the cameras."""

    def __init__(self, cams, n_gaussians, view_scene=None, scene_begin=None, device="cuda"):
        V = len(cams)
        self.V = V
        self.cams = list(cams)
        self._host = (Camera * V)(*[camera_struct(c) for c in cams])
        raw = np.frombuffer(bytes(self._host), dtype=np.uint8).copy()
        self.cams_dev = torch.from_numpy(raw).to(device)
        self._vs = None
        self._sb = None
        S = 1
        if view_scene is not None:
            self._vs = (c_int32 * V)(*[int(s) for s in view_scene])
        if scene_begin is not None:
            S = len(scene_begin) - 1
            self._sb = (c_int64 * (S + 1))(*[int(s) for s in scene_begin])
        self.n_scenes = S
        self.n_gaussians = int(n_gaussians)
        self.s = Views()
        self.s.n_views = V
        self.s.n_scenes = S
        self.s.n_gaussians = self.n_gaussians
        self.s.cams_host = ctypes.cast(self._host, POINTER(Camera))
        self.s.cams_dev = c_void_p(self.cams_dev.data_ptr())
        self.s.view_scene = ctypes.cast(self._vs, POINTER(c_int32)) if self._vs is not None else None
        self.s.scene_begin = ctypes.cast(self._sb, POINTER(c_int64)) if self._sb is not None else None

    def set_pose(self, v, T_cw, stream=None):
        """Update view v's pose in the device camera table (in place, on the stream)."""
        T = torch.as_tensor(np.asarray(T_cw, np.float32).reshape(12))
        off = ctypes.sizeof(Camera) * v + Camera.T_cw.offset
        self.cams_dev[off:off + 48].copy_(T.view(torch.uint8).to(self.cams_dev.device), non_blocking=False)
        self._host[v].T_cw[:] = [float(x) for x in T.tolist()]

    def pose(self, v):
        """View v's T_cw [3, 4] as stored in the device camera table (synchronises)."""
        off = ctypes.sizeof(Camera) * v + Camera.T_cw.offset
        return self.cams_dev[off:off + 48].view(torch.float32).reshape(3, 4).cpu().numpy().astype(np.float64)

    def set_pose_tensor(self, v, T_dev):
        """Copy a float32 [12] device tensor into view v's pose (graph-capturable)."""
        off = ctypes.sizeof(Camera) * v + Camera.T_cw.offset
        self.cams_dev[off:off + 48].view(torch.float32).copy_(T_dev.reshape(12))

    @property
    def rec_count(self):
        return int(lib().gs_rec_count(ctypes.byref(self.s)))

    def rec_offset(self, v):
        return int(lib().gs_rec_offset(ctypes.byref(self.s), v))

    @property
    def tile_count(self):
        return int(lib().gs_tile_count(ctypes.byref(self.s)))

    @property
    def pixel_count(self):
        return int(lib().gs_pixel_count(ctypes.byref(self.s)))


def gaussians_struct(t: dict) -> Gaussians:
    """The C struct of the Gaussian arrays; keeps the tensors alive as long as
    it lives."""
    g = Gaussians()
    g.n = int(t["opacity_logit"].shape[0])
    for k in ("mean", "log_scale", "quat", "opacity_logit", "color", "mp"):
        setattr(g, k, c_void_p(t[k].data_ptr()))
    g._keep = dict(t)
    return g


def to_device(g: dict, device="cuda") -> dict:
    return {k: torch.as_tensor(np.ascontiguousarray(v)).to(device) for k, v in g.items()}


class Pipeline:
    """Buffers and calls of one render + loss + backward iteration for a view
    batch. All buffers are torch tensors on `device`; every kernel runs in
    libgs.so."""

    def __init__(self, ctx: Context, views: ViewBatch, capacity: int, max_rank: int = 0, full_proj=False,
                 device="cuda", bg=(0.0, 0.0, 0.0)):
        self.ctx, self.views, self.device = ctx, views, device
        self.bg = tuple(float(x) for x in bg)
        M, T, P = views.rec_count, views.tile_count, views.pixel_count
        self.M, self.T, self.P = M, T, P
        f32, i32, dev = torch.float32, torch.int32, device
        self.rec = torch.empty(M * 12, dtype=f32, device=dev)
        self.rect = torch.empty(M * 4, dtype=torch.int16, device=dev)
        self.key = torch.empty(M, dtype=i32, device=dev)
        self.full_proj = full_proj
        if full_proj:
            self.mean2d = torch.empty(2 * M, dtype=f32, device=dev)
            self.conic = torch.empty(3 * M, dtype=f32, device=dev)
            self.depth = torch.empty(M, dtype=f32, device=dev)
            self.opacity = torch.empty(M, dtype=f32, device=dev)
            self.radius = torch.empty(M, dtype=i32, device=dev)
        self.proj = Proj()
        self.proj.m = M
        self.proj.rec, self.proj.rect, self.proj.depth_key = ptr(self.rec), ptr(self.rect), ptr(self.key)
        self.key_hist = torch.zeros(views.V * 4096, dtype=i32, device=dev)
        if full_proj:
            for k in ("mean2d", "conic", "depth", "opacity", "radius"):
                setattr(self.proj, k, ptr(getattr(self, k)))
        self.capacity = int(capacity)
        self.ids = torch.empty(max(1, self.capacity), dtype=i32, device=dev)
        self.tile_start = torch.empty(T + 1, dtype=i32, device=dev)
        self.sorted_ids = torch.empty(M, dtype=i32, device=dev)
        # n_instances, overflow, incomplete, the per-view truncation bits
        self.counters = torch.zeros(4, dtype=torch.int64, device=dev)
        self.bins = Bins()
        self.bins.capacity = self.capacity
        self.bins.gauss_id, self.bins.tile_start, self.bins.sorted_ids = ptr(self.ids), ptr(self.tile_start), ptr(
            self.sorted_ids)
        base = self.counters.data_ptr()
        self.bins.n_instances = c_void_p(base)
        self.bins.overflow = c_void_p(base + 8)
        self.bins.incomplete = c_void_p(base + 16)
        self.bins.truncated = c_void_p(base + 24)
        self.set_max_rank(max_rank)
        self.img_color = torch.empty(3 * P, dtype=f32, device=dev)
        self.img_depth = torch.empty(P, dtype=f32, device=dev)
        self.img_mp = torch.empty(P, dtype=f32, device=dev)
        self.img_T = torch.empty(P, dtype=f32, device=dev)
        self.img_nlast = torch.empty(P, dtype=i32, device=dev)
        # tile scheduling state: per-tile work, then the launch order and its
        # marker (zero-filled: no order yet)
        self.img_tile_work = torch.zeros(2 * T + 1, dtype=i32, device=dev)
        self.img = Image(ptr(self.img_color), ptr(self.img_depth), ptr(self.img_mp), ptr(self.img_T),
                         ptr(self.img_nlast), ptr(self.img_tile_work))
        self.dC = torch.empty(3 * P, dtype=f32, device=dev)
        self.dD = torch.empty(P, dtype=f32, device=dev)
        self.dM = torch.zeros(P, dtype=f32, device=dev)
        self.dT = torch.zeros(P, dtype=f32, device=dev)
        self.pg = PixelGrads(ptr(self.dC), ptr(self.dD), ptr(self.dM), ptr(self.dT))
        self.loss = torch.zeros(views.V, dtype=f32, device=dev)
        self.ws_bin = torch.empty(gs_workspace_size(ctx, views.s, GS_OP_BIN_SORT, self.capacity), dtype=torch.uint8,
                                  device=dev)
        self.ws_bwd = torch.zeros(gs_workspace_size(ctx, views.s, GS_OP_RENDER_BWD), dtype=torch.uint8, device=dev)
        self.ws_loss = torch.zeros(gs_workspace_size(ctx, views.s, GS_OP_LOSS), dtype=torch.uint8, device=dev)
        self.lp = LossParams(0.9, 0.1, 1e-6, 0, 0)
        # sticky overflow and incomplete flags (gs_bins.sticky), which the
        # library sets and never clears, kept across iterations while
        # `sticky` is set (the library resets its own flags in every
        # gs_bin_sort)
        self.flags = torch.zeros(2, dtype=torch.int32, device=dev)
        self.sticky = False

    @property
    def sticky(self):
        return self.bins.sticky is not None

    @sticky.setter
    def sticky(self, on):
        self.bins.sticky = ptr(self.flags) if on else None

    def raise_if_failed(self, stream=None):
        """Synchronises and raises GSError when an iteration since the last
        clear_flags() overflowed the list capacity or ran out of a truncated
        prefix list (its images, loss and gradients are then not exact)."""
        over, n_inst, inc = gs_bins_check(self.ctx, self.bins, stream)
        f = self.flags.cpu().tolist() if self.sticky else [0, 0]
        if over or f[0]:
            raise GSError(GS_E_CAPACITY, f"list capacity {self.capacity} exceeded ({n_inst} entries needed)")
        if inc or f[1]:
            raise GSError(GS_E_CAPACITY, f"a tile ran out of its prefix list (max_rank {self.bins.max_rank}): "
                                         "re-bin with a larger rank or full lists")

    def clear_flags(self):
        self.flags.zero_()

    def set_max_rank(self, max_rank: int):
        """Switches between the prefix lists (max_rank > 0: gs_project fills
        the key histogram and gs_bin_sort projects the selected records) and
        the full lists (max_rank <= 0: gs_project writes every record)."""
        self.bins.max_rank = int(max_rank)
        self.key_hist.zero_()
        self.proj.key_hist = ptr(self.key_hist) if max_rank > 0 else None

    def set_loss_params(self, lambda_pho=0.9, lambda_depth=0.1, eps_A=1e-6, weight_mode=0, grad_through_weight=0):
        self.lp = LossParams(lambda_pho, lambda_depth, eps_A, weight_mode, grad_through_weight)

    def forward(self, g: Gaussians, stream=None):
        gs_project(self.ctx, self.views.s, g, self.proj, stream)
        gs_bin_sort(self.ctx, self.views.s, g, self.proj, self.bins, self.ws_bin, stream)
        gs_render_fwd(self.ctx, self.views.s, g, self.proj, self.bins, self.bg, self.img, stream)

    def loss_and_grads(self, target_color, target_depth, stream=None):
        self._tgt_keep = (target_color, target_depth)
        tgt = Target(ptr(target_color), ptr(target_depth))
        gs_loss(self.ctx, self.views.s, self.img, tgt, self.lp, self.loss, self.pg, self.ws_loss, stream)

    def forward_loss(self, g: Gaussians, target_color, target_depth, stream=None):
        """forward and loss_and_grads in one pass (the loss fused into the
        forward's epilogue)."""
        self._tgt_keep = (target_color, target_depth)
        tgt = Target(ptr(target_color), ptr(target_depth))
        gs_project(self.ctx, self.views.s, g, self.proj, stream)
        gs_bin_sort(self.ctx, self.views.s, g, self.proj, self.bins, self.ws_bin, stream)
        gs_render_fwd_loss(self.ctx, self.views.s, g, self.proj, self.bins, self.bg, self.img, tgt, self.lp,
                           self.loss, self.pg, self.ws_loss, stream)

    def backward(self, g: Gaussians, grads: Grads, stream=None):
        gs_render_bwd(self.ctx, self.views.s, g, self.proj, self.bins, self.img, self.pg, self.bg, grads,
                      self.ws_bwd, stream)

    def check(self, stream=None):
        return gs_bins_check(self.ctx, self.bins, stream)

    def image(self):
        P = self.P
        return dict(C=self.img_color.view(3, P), D=self.img_depth, M=self.img_mp, T=self.img_T,
                    n_last=self.img_nlast)


def grads_struct(gr: dict, pose: torch.Tensor, pose_only=False, accumulate=False) -> Grads:
    """The C struct of gradient outputs. It holds raw device addresses, so it
    keeps the tensors alive for as long as it lives (a struct that outlived
    its tensors would let kernels write into freed, possibly unmapped memory)."""
    s = Grads()
    for k in ("mean", "log_scale", "quat", "opacity_logit", "color"):
        setattr(s, k, ptr(gr[k]) if gr is not None and k in gr else None)
    s.pose = ptr(pose)
    s.pose_only = int(pose_only)
    s.accumulate = int(accumulate)
    s._keep = (gr, pose)
    return s


def alloc_grads(n, device="cuda"):
    f = torch.float32
    return dict(mean=torch.zeros(3, n, dtype=f, device=device), log_scale=torch.zeros(3, n, dtype=f, device=device),
                quat=torch.zeros(4, n, dtype=f, device=device), opacity_logit=torch.zeros(n, dtype=f, device=device),
                color=torch.zeros(3, n, dtype=f, device=device))
