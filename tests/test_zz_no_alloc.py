"""The allocation-free forward + loss (gs_render_fwd_loss_static) against
gs_render_fwd_loss, through the C ABI: two calls in a row, the second with a
smaller batch, each giving the images, pixel adjoints and per-view losses of
the workspace call bit for bit (the per-tile loss partials are summed in the
same fixed order, only their memory differs)."""

import numpy as np
import pytest
import torch

from paper_2602_21644_amd import gs, synth
from tests.gpu_util import make_pipeline

pytestmark = pytest.mark.gpu

OUTS = ("img_color", "img_depth", "img_mp", "img_T", "img_nlast", "dC", "dD", "dM", "dT")


@pytest.fixture(scope="module")
def ctx():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return gs.Context(0)


def _case(ctx, seed, n, W, H, nviews, max_rank, gtw):
    g, cam, tcam, g_t, sl = synth.moving_box_scene(seed, n, W, H)
    cams = [cam, tcam, synth.camera(W, H, synth.perturbed_pose(synth.rng_for(seed + 1)))][:nviews]
    views, pipe, gt, gst = make_pipeline(ctx, g, cams, max_rank=max_rank, bg=(0.1, 0.2, 0.3))
    pipe.set_loss_params(grad_through_weight=gtw)
    rng = np.random.default_rng(seed)
    P = pipe.P
    tc = torch.from_numpy(rng.random(3 * P).astype(np.float32)).cuda()
    td = torch.from_numpy(np.where(rng.random(P) < 0.8, rng.uniform(0.5, 4.0, P), 0.0).astype(np.float32)).cuda()
    return views, pipe, gst, tc, td


def _static_forward_loss(ctx, views, pipe, gst, tc, td, timing):
    gs.gs_project(ctx, views.s, gst, pipe.proj)
    gs.gs_bin_sort(ctx, views.s, gst, pipe.proj, pipe.bins, pipe.ws_bin)
    tgt = gs.Target(gs.ptr(tc), gs.ptr(td))
    ctx.set_param("timing", timing)
    gs.gs_render_fwd_loss_static(ctx, views.s, gst, pipe.proj, pipe.bins, pipe.bg, pipe.img, tgt, pipe.lp,
                                 pipe.loss, pipe.pg)
    ctx.set_param("timing", 0)


@pytest.mark.parametrize("timing", [0, 1])
def test_static_forward_loss_matches_workspace_call(ctx, timing):
    # the second call is smaller in every respect (views, pixels, tiles, Gaussians)
    cases = [(41, 120_000, 640, 480, 3, 2048, 1), (42, 20_000, 320, 240, 1, 0, 0)]
    assert 3 * 40 * 30 > 20 * 15
    for seed, n, W, H, nv, R, gtw in cases:
        views, pipe, gst, tc, td = _case(ctx, seed, n, W, H, nv, R, gtw)
        pipe.forward_loss(gst, tc, td)
        torch.cuda.synchronize()
        ref = {k: getattr(pipe, k).clone() for k in OUTS}
        ref_loss = pipe.loss.clone()
        ref_flags = pipe.check()
        for k in OUTS:  # a value no kernel writes, so a missed element shows
            t = getattr(pipe, k)
            t.fill_(float("nan")) if t.dtype == torch.float32 else t.fill_(0x7FFFFFFF)
        pipe.loss.fill_(float("nan"))
        ctx.kernel_times()
        _static_forward_loss(ctx, views, pipe, gst, tc, td, timing)
        torch.cuda.synchronize()
        assert ctx.kernel_times() == {}  # nothing was timed (no event allocated) inside the call
        assert pipe.check() == ref_flags
        assert not ref_flags[0]
        for k in OUTS:
            assert torch.equal(getattr(pipe, k), ref[k]), k
        assert torch.equal(pipe.loss, ref_loss)
        assert float(ref_loss.abs().min()) > 0
