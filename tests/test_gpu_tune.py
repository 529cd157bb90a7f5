"""GPU test of the knob autotuner: the cache round trip, and that tuned knobs
leave the results unchanged."""

import json

import pytest
import torch

from paper_2602_21644_amd import gs, synth, tune

pytestmark = pytest.mark.gpu


def test_tune_cache_and_invariance(tmp_path):
    ctx = gs.Context(0)
    g, cam, tcam, g_t, sl = synth.moving_box_scene(17, 30000, 160, 120)
    gd = gs.to_device(g)
    # target: the scene with boxes moved, seen from the second camera
    tv = gs.ViewBatch([tcam], synth.n_gaussians(g))
    tp = gs.Pipeline(ctx, tv, capacity=1 << 22)
    tp.forward(gs.gaussians_struct(gs.to_device(g_t)))
    tc = tp.img_color.clone()
    td = tp.img_depth.clone()
    views = gs.ViewBatch([cam], synth.n_gaussians(g))
    # reference image with the default knobs
    ref = gs.Pipeline(ctx, views, capacity=1 << 22)
    gst = gs.gaussians_struct(gd)
    ref.forward(gst)
    ref.loss_and_grads(tc, td)
    img0 = [t.clone() for t in (ref.img_color, ref.img_depth, ref.img_T, ref.img_nlast)]
    loss0 = float(ref.loss[0])
    cache = str(tmp_path / "tune.json")
    ent = tune.tune(ctx, views, gd, tc, td, cache=cache, iters=2)
    assert not ent["cached"] and ent["ms"] > 0
    table = json.load(open(cache))
    key = tune.bucket_key(views, synth.n_gaussians(g))
    assert key in table and table[key]["knobs"] == ent["knobs"]
    for k, v in ent["knobs"].items():
        assert ctx.get_param(k) == v
    again = tune.tune(ctx, views, gd, tc, td, cache=cache)
    assert again["cached"] and again["knobs"] == ent["knobs"]
    # same images and loss with the tuned knobs
    p2 = gs.Pipeline(ctx, views, capacity=1 << 22)
    p2.forward(gst)
    p2.loss_and_grads(tc, td)
    for a, b in zip(img0, (p2.img_color, p2.img_depth, p2.img_T, p2.img_nlast)):
        assert torch.equal(a, b)
    assert float(p2.loss[0]) == loss0
