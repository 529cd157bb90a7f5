"""Helpers shared by the GPU parity tests (inputs, buffers, comparisons)."""

import numpy as np
import torch

from paper_2602_21644_amd import gs, synth


def make_pipeline(ctx, g_np, cams, capacity=None, max_rank=0, full_proj=True, bg=(0, 0, 0), view_scene=None,
                  scene_begin=None):
    n = synth.n_gaussians(g_np)
    views = gs.ViewBatch(cams, n, view_scene=view_scene, scene_begin=scene_begin)
    if capacity is None:
        capacity = max(1 << 16, 64 * n * len(cams))
    pipe = gs.Pipeline(ctx, views, capacity, max_rank=max_rank, full_proj=full_proj, bg=bg)
    gt = gs.to_device(g_np)
    return views, pipe, gt, gs.gaussians_struct(gt)


def view_slice(views, v, M):
    r0 = views.rec_offset(v)
    return r0


def proj_view(pipe, views, v, n):
    """GPU projection outputs of view v as numpy (first n records)."""
    M = pipe.M
    r0 = views.rec_offset(v)
    s = slice(r0, r0 + n)
    out = dict(mean2d=pipe.mean2d.view(2, M)[:, s].cpu().numpy(), conic=pipe.conic.view(3, M)[:, s].cpu().numpy(),
               depth=pipe.depth[s].cpu().numpy(), opacity=pipe.opacity[s].cpu().numpy(),
               radius=pipe.radius[s].cpu().numpy(),
               rect=pipe.rect.view(M, 4)[s].cpu().numpy().astype(np.int64),
               key=pipe.key[s].cpu().numpy().view(np.uint32))
    return out


def image_view(pipe, views, v):
    P = pipe.P
    off = 0
    for i in range(v):
        off += views.cams[i]["width"] * views.cams[i]["height"]
    W, H = views.cams[v]["width"], views.cams[v]["height"]
    s = slice(off, off + W * H)
    return dict(C=pipe.img_color.view(3, P)[:, s].cpu().numpy().astype(np.float64),
                D=pipe.img_depth[s].cpu().numpy().astype(np.float64),
                M=pipe.img_mp[s].cpu().numpy().astype(np.float64),
                T=pipe.img_T[s].cpu().numpy().astype(np.float64),
                n_last=pipe.img_nlast[s].cpu().numpy())


def oracle_target(orc, g_np, cam, valid_A=0.5):
    pr = orc.project(g_np, cam)
    im = orc.render(pr, g_np, cam)
    td = im["D"].copy()
    td[(1 - im["T"]) < valid_A] = 0.0
    return im["C"].astype(np.float32), td.astype(np.float32)


def assert_image_close(gpu, ref, margin, tol=1e-4, max_excluded=1e-3):
    """Images within `tol` absolute on every pixel whose oracle margin is at
    least 1e-5; at most `max_excluded` of the pixels may be excluded."""
    ok = margin >= 1e-5
    assert (~ok).mean() <= max_excluded, f"excluded {(~ok).sum()} of {ok.size}"
    for k in ("D", "M", "T"):
        err = np.abs(gpu[k] - ref[k])[ok]
        assert err.max() <= tol, (k, err.max(), int((err > tol).sum()),
                                  np.argmax(np.where(ok, np.abs(gpu[k] - ref[k]), 0)))
    err = np.abs(gpu["C"] - ref["C"])[:, ok]
    assert err.max() <= tol, ("C", err.max(), int((err > tol).sum()))


def grads_report(gpu, ref, rel=1e-3):
    """(max abs error / group max, number of elements above 1% of the group
    maximum that miss `rel` relative, worst relative error among them)."""
    gpu = np.asarray(gpu, np.float64)
    ref = np.asarray(ref, np.float64)
    scale = np.abs(ref).max()
    if scale == 0:
        return float(np.abs(gpu).max()), 0, 0.0
    err = np.abs(gpu - ref)
    big = np.abs(ref) > 0.01 * scale
    relerr = err[big] / np.abs(ref[big])
    return float(err.max() / scale), int((relerr > rel).sum()), float(relerr.max()) if relerr.size else 0.0


def assert_grads_close(gpu, ref, rel=1e-3, name=""):
    """The survey's gradient bar: per group, max |g - g_ref| <= rel * max
    |g_ref|, and every element above 1% of the group maximum within `rel`
    relative."""
    gpu = np.asarray(gpu, np.float64)
    ref = np.asarray(ref, np.float64)
    scale = np.abs(ref).max()
    if scale == 0:
        assert np.abs(gpu).max() == 0, name
        return
    err_max, n_bad, worst = grads_report(gpu, ref, rel)
    assert err_max <= rel, (name, "max error / group max", err_max)
    assert n_bad == 0, (name, f"{n_bad} elements above 1% of the group max miss {rel} relative; worst {worst:.3g}")


def bwd_zero_part(pipe, views):
    """The backward scratch, which every call leaves zero-filled."""
    return pipe.ws_bwd


def torch_np(t):
    return t.detach().cpu().numpy()
