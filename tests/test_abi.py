"""CPU checks of the C-ABI library: it loads and exports every symbol that
include/gs.h declares (no compute calls without a GPU), and host-side
argument validation rejects bad input before anything is enqueued."""

import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_symbols():
    src = open(os.path.join(ROOT, "include", "gs.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(gs_[a-z0-9_]+)\s*\(", src)))


def test_header_symbols_exported():
    from paper_2602_21644_amd import gs
    L = gs.lib()
    names = declared_symbols()
    assert len(names) >= 20
    for name in names:
        assert hasattr(L, name), name
    assert set(gs.EXPORTED) == set(names)


def test_status_strings_and_param_validation():
    from paper_2602_21644_amd import gs
    L = gs.lib()
    assert L.gs_status_str(0) == b"ok"
    ctx = gs.Context(0)
    assert ctx.get_param("render_batch") in (64, 128, 256)
    ctx.set_param("bwd_batch", 32)
    assert ctx.get_param("bwd_batch") == 32
    with pytest.raises(gs.GSError):
        ctx.set_param("bwd_batch", 33)
    with pytest.raises(gs.GSError):
        ctx.set_param("nope", 1)
    assert ctx.get_param("tile_order") == 1
    ctx.set_param("tile_order", 0)
    assert ctx.get_param("tile_order") == 0
    with pytest.raises(gs.GSError):
        ctx.set_param("tile_order", 2)
    assert ctx.get_param("n_cu") == 0  # queried by the first backward on a GPU
    assert ctx.get_param("bwd_copies") == 8
    assert ctx.get_param("wave_cull") == 1
    with pytest.raises(gs.GSError):
        ctx.get_param("bwd_mfma")  # the matrix-core backward was removed
    with pytest.raises(gs.GSError):
        ctx.set_param("bwd_copies", 3)


def test_layout_helpers():
    from paper_2602_21644_amd import gs, synth
    cams = [synth.camera(640, 480), synth.camera(320, 240)]
    vb = gs.ViewBatch.__new__(gs.ViewBatch)
    host = (gs.Camera * 2)(*[gs.camera_struct(c) for c in cams])
    sb = (ctypes.c_int64 * 3)(0, 1000, 1100)
    vs = (ctypes.c_int32 * 2)(0, 1)
    v = gs.Views()
    v.n_views, v.n_scenes, v.n_gaussians = 2, 2, 1100
    v.cams_host = ctypes.cast(host, ctypes.POINTER(gs.Camera))
    v.cams_dev = ctypes.c_void_p(1)
    v.view_scene = ctypes.cast(vs, ctypes.POINTER(ctypes.c_int32))
    v.scene_begin = ctypes.cast(sb, ctypes.POINTER(ctypes.c_int64))
    L = gs.lib()
    assert L.gs_rec_count(ctypes.byref(v)) == 1024 + 128
    assert L.gs_rec_offset(ctypes.byref(v), 1) == 1024
    assert L.gs_tile_count(ctypes.byref(v)) == 40 * 30 + 20 * 15
    assert L.gs_pixel_count(ctypes.byref(v)) == 640 * 480 + 320 * 240
    ctx = gs.Context(0)
    for op in (gs.GS_OP_BIN_SORT, gs.GS_OP_RENDER_BWD, gs.GS_OP_LOSS):
        assert gs.gs_workspace_size(ctx, v, op) > 0
    v.n_views = 0
    with pytest.raises(gs.GSError):
        gs.gs_workspace_size(ctx, v, gs.GS_OP_LOSS)
    # an image too large for the binning's LDS tables is rejected, not run
    big = (gs.Camera * 1)(gs.camera_struct(synth.camera(4096, 4096)))
    v.n_views, v.n_scenes, v.n_gaussians = 1, 1, 10
    v.cams_host = ctypes.cast(big, ctypes.POINTER(gs.Camera))
    v.view_scene = None
    v.scene_begin = None
    with pytest.raises(gs.GSError) as e:
        gs.gs_workspace_size(ctx, v, gs.GS_OP_BIN_SORT)
    assert e.value.status == gs.GS_E_UNSUPPORTED


def test_view_count_and_empty_scene_limits():
    """1 .. GS_MAX_VIEWS views per batch; a batch with no Gaussians is valid
    (no records, tiles and workspaces as usual), a negative count is not."""
    from paper_2602_21644_amd import gs, synth
    L = gs.lib()
    ctx = gs.Context(0)
    for V, ok in ((gs.GS_MAX_VIEWS, True), (gs.GS_MAX_VIEWS + 1, False)):
        host = (gs.Camera * V)(*[gs.camera_struct(synth.camera(40, 30)) for _ in range(V)])
        v = gs.Views()
        v.n_views, v.n_scenes, v.n_gaussians = V, 1, 0
        v.cams_host = ctypes.cast(host, ctypes.POINTER(gs.Camera))
        v.cams_dev = ctypes.c_void_p(1)
        if ok:
            assert L.gs_rec_count(ctypes.byref(v)) == 0
            assert L.gs_tile_count(ctypes.byref(v)) == V * 3 * 2
            for op in (gs.GS_OP_BIN_SORT, gs.GS_OP_RENDER_BWD, gs.GS_OP_LOSS):
                assert gs.gs_workspace_size(ctx, v, op) > 0
            v.n_gaussians = -1
        assert L.gs_rec_count(ctypes.byref(v)) == -1
        with pytest.raises(gs.GSError):
            gs.gs_workspace_size(ctx, v, gs.GS_OP_LOSS)


def test_structs_keep_their_tensors_alive():
    """The C structs hold raw addresses: they keep the tensors they point to
    alive, so a captured graph replayed later never writes freed memory."""
    import gc
    import weakref

    import torch
    from paper_2602_21644_amd import gs
    n = 10
    gr = {k: torch.zeros(3, n) for k in ("mean", "log_scale", "color")}
    gr["quat"] = torch.zeros(4, n)
    gr["opacity_logit"] = torch.zeros(n)
    pose = torch.zeros(6)
    refs = [weakref.ref(t) for t in list(gr.values()) + [pose]]
    s = gs.grads_struct(gr, pose)
    g = {k: torch.zeros(3, n) for k in ("mean", "log_scale", "color")}
    g.update(quat=torch.zeros(4, n), opacity_logit=torch.zeros(n), mp=torch.zeros(n))
    grefs = [weakref.ref(t) for t in g.values()]
    gst = gs.gaussians_struct(g)
    del gr, pose, g
    gc.collect()
    assert all(r() is not None for r in refs + grefs)
    del s, gst
    gc.collect()
    assert all(r() is None for r in refs + grefs)


def test_static_forward_loss_rejects_large_batches_on_the_host():
    """The allocation-free forward + loss holds 32768 tiles; a batch with more
    (28 views of 640x480 = 33600 tiles) is refused before any device call,
    so this runs without a GPU."""
    from paper_2602_21644_amd import gs, synth
    L = gs.lib()
    V = 28
    host = (gs.Camera * V)(*[gs.camera_struct(synth.camera(640, 480)) for _ in range(V)])
    v = gs.Views()
    v.n_views, v.n_scenes, v.n_gaussians = V, 1, 10
    v.cams_host = ctypes.cast(host, ctypes.POINTER(gs.Camera))
    v.cams_dev = ctypes.c_void_p(1)
    ctx = gs.Context(0)
    P = ctypes.c_void_p(16)  # never dereferenced: the call stops at the size check
    g = gs.Gaussians(10, P, P, P, P, P, P)
    proj, bins = gs.Proj(), gs.Bins()
    img = gs.Image(P, P, P, P, P, None)
    tgt = gs.Target(P, P)
    pg = gs.PixelGrads(P, P, None, None)
    lp = gs.LossParams(0.9, 0.1, 1e-6, 0, 0)
    bg = (ctypes.c_float * 3)(0, 0, 0)
    st = L.gs_render_fwd_loss_static(ctx.h, ctypes.byref(v), ctypes.byref(g), ctypes.byref(proj),
                                     ctypes.byref(bins), bg, ctypes.byref(img), ctypes.byref(tgt), ctypes.byref(lp),
                                     P, ctypes.byref(pg), None)
    assert st == gs.GS_E_UNSUPPORTED
    assert b"32768" in L.gs_last_error(ctx.h)
