"""GPU parity of batched calls: several views of one scene (a keyframe
window) and several scenes of different sizes in one call sequence, on the
full-list and the prefix binning paths, plus HIP-graph replays of the whole
iteration against eager runs."""

import numpy as np
import pytest
import torch

from paper_2602_21644_amd import gs, synth
from tests.gpu_util import (assert_grads_close, assert_image_close, bwd_zero_part, image_view, oracle_target,
                            torch_np)

pytestmark = pytest.mark.gpu

KEYS = ("mean", "log_scale", "quat", "opacity_logit", "color")


@pytest.fixture(scope="module")
def ctx():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return gs.Context(0)


def _batch_case(ctx, orc, scenes, views, max_rank=0, bg=(0.1, 0.1, 0.1)):
    """scenes: list of Gaussian dicts; views: list of (scene, camera, target
    camera). Runs project, bin, render, loss and backward once for the whole
    batch and checks every view and every scene against the oracle."""
    sizes = [synth.n_gaussians(g) for g in scenes]
    begin = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)
    g_all = synth.concat_gaussians(scenes)
    n = int(begin[-1])
    cams = [c for _, c, _ in views]
    vb = gs.ViewBatch(cams, n, view_scene=[s for s, _, _ in views], scene_begin=begin.tolist())
    capacity = 64 * sum(sizes[s] for s, _, _ in views) + 4096
    pipe = gs.Pipeline(ctx, vb, capacity, max_rank=max_rank, bg=bg)
    gt = gs.to_device(g_all)
    gst = gs.gaussians_struct(gt)
    # targets and oracle forward per view
    tcs, tds, refs, prs = [], [], [], []
    for s, c, tc in views:
        a, b = oracle_target(orc, scenes[s], tc)
        tcs.append(a)
        tds.append(b)
        pr = orc.project(scenes[s], c)
        prs.append(pr)
        refs.append(orc.render(pr, scenes[s], c, bg=bg))
    tcol = torch.from_numpy(np.concatenate([t.reshape(3, -1) for t in tcs], axis=1).reshape(-1)).cuda()
    tdep = torch.from_numpy(np.concatenate(tds)).cuda()
    pipe.forward(gst)
    over, n_inst, inc = pipe.check()
    assert not over
    if max_rank:
        assert inc == 0, "prefix too short for this batch"
    # forward parity per view
    for v, (s, c, _) in enumerate(views):
        assert_image_close(image_view(pipe, vb, v), refs[v], refs[v]["margin"])
    pipe.loss_and_grads(tcol, tdep)
    # pixel adjoints zeroed on both sides at ambiguous pixels
    keeps, Ls = [], []
    for v, (s, c, _) in enumerate(views):
        im = refs[v]
        L = orc.loss(im, tcs[v], tds[v])
        Ls.append(L)
        amb = (im["margin"] < 1e-5) | (np.abs(im["C"] - tcs[v]).min(axis=0) < 1e-5) | (
            (tds[v] > 0) & (np.abs(im["D"] - tds[v]) < 1e-5))
        keeps.append(~amb)
        assert abs(float(pipe.loss[v]) - L["loss"]) <= 1e-4 * abs(L["loss"]), v
    P = pipe.P
    keep = torch.from_numpy(np.concatenate(keeps)).cuda()
    pipe.dC.view(3, P).mul_(keep)
    pipe.dD.mul_(keep)
    pipe.dM.mul_(keep)
    pipe.dT.mul_(keep)
    grads = gs.alloc_grads(n)
    pose = torch.zeros(6 * len(views), device="cuda")
    pipe.backward(gst, gs.grads_struct(grads, pose))
    torch.cuda.synchronize()
    ref = {k: np.zeros_like(g_all[k], dtype=np.float64) for k in KEYS}
    ref_pose = np.zeros((len(views), 6))
    for v, (s, c, _) in enumerate(views):
        k = keeps[v]
        L = Ls[v]
        g2d = orc.render_backward(prs[v], scenes[s], c, L["dC"] * k, L["dD"] * k, L["dM"] * k, L["dT"] * k, bg=bg)
        rg = orc.project_backward(scenes[s], c, g2d)
        for key in KEYS:
            ref[key][..., begin[s]:begin[s + 1]] += rg[key]
        ref_pose[v] = rg["pose"]
    for s in range(len(scenes)):
        if begin[s + 1] == begin[s]:
            continue  # an empty scene has no gradient
        for key in KEYS:
            assert_grads_close(torch_np(grads[key])[..., begin[s]:begin[s + 1]], ref[key][..., begin[s]:begin[s + 1]],
                               name=f"{key}[scene {s}]")
    got_pose = torch_np(pose).reshape(len(views), 6)
    for v in range(len(views)):
        assert_grads_close(got_pose[v], ref_pose[v], name=f"pose[view {v}]")
    return pipe, vb, gst


def _window(seed, n, W, H, V):
    g, cam, tcam, g_t, sl = synth.moving_box_scene(seed, n, W, H)
    cams = synth.window_cameras(seed, V, W, H, spacing=2)
    rng = synth.rng_for(seed + 100)
    # each target 1 degree and 2 cm away from its view
    tcams = [synth.camera(W, H, synth.perturbed_pose(rng, base=c["T_cw"])) for c in cams]
    return g, [(0, c, tc) for c, tc in zip(cams, tcams)]


@pytest.mark.parametrize("max_rank", [0, 16384])
def test_window_batch_parity(ctx, orc, max_rank):
    """Several keyframes of one scene in one batch: gradients are the sums over
    the views, one pose gradient per view."""
    g, views = _window(21, 12000, 160, 120, 4)
    _batch_case(ctx, orc, [g], views, max_rank=max_rank)


@pytest.mark.parametrize("max_rank", [0, 16384])
def test_uneven_scene_batch_parity(ctx, orc, max_rank):
    """Scenes of different sizes and image shapes (partial edge tiles) in one
    batch, each with its own views."""
    specs = [(31, 3000, 64, 48, 2), (32, 8000, 168, 120, 2), (33, 12000, 200, 150, 1)]
    scenes, views = [], []
    for i, (seed, n, W, H, V) in enumerate(specs):
        g, vv = _window(seed, n, W, H, V)
        scenes.append(g)
        views += [(i, c, tc) for _, c, tc in vv]
    _batch_case(ctx, orc, scenes, views, max_rank=max_rank)


@pytest.mark.parametrize("max_rank", [0, 16384])
def test_max_views_batch_parity(ctx, orc, max_rank):
    """The largest batch one call takes (GS_MAX_VIEWS = 32 views) over four
    scenes, one of them empty: every view's image and loss, every scene's
    gradients and every view's pose twist against the oracle."""
    empty = synth.static_gaussians(synth.rng_for(40), 0, 48, 32)
    scenes, views = [empty], [(0, c, c) for c in synth.window_cameras(40, 2, 48, 32)]
    specs = [(41, 3000, 64, 48, 10), (42, 5000, 96, 72, 10), (43, 2000, 40, 30, 10)]
    for i, (seed, n, W, H, V) in enumerate(specs):
        g, vv = _window(seed, n, W, H, V)
        scenes.append(g)
        views += [(i + 1, c, tc) for _, c, tc in vv]
    assert len(views) == 32
    print(f"\n[batch] 32 views, max_rank={max_rank}", flush=True)
    _batch_case(ctx, orc, scenes, views, max_rank=max_rank)


@pytest.mark.parametrize("fused", [False, True])
def test_graph_replay_matches_eager(ctx, fused):
    """The whole iteration (project, bin, render, loss, backward; the loss
    separate or fused into the forward) captured once and replayed several
    times, with eager work and synchronisations between replays, gives the
    eager results every time."""
    g, views = _window(41, 20000, 160, 120, 3)
    cams = [c for _, c, _ in views]
    vb = gs.ViewBatch(cams, synth.n_gaussians(g))
    pipe = gs.Pipeline(ctx, vb, 64 * 20000 * 3, max_rank=8192)
    gt = gs.to_device(g)
    gst = gs.gaussians_struct(gt)
    P = pipe.P
    tcol = torch.rand(3 * P, device="cuda")
    tdep = torch.rand(P, device="cuda") * 3
    grads = gs.alloc_grads(synth.n_gaussians(g))
    pose = torch.zeros(6 * len(cams), device="cuda")
    gsr = gs.grads_struct(grads, pose)

    def step():
        if fused:
            pipe.forward_loss(gst, tcol, tdep)
        else:
            pipe.forward(gst)
            pipe.loss_and_grads(tcol, tdep)
        pipe.backward(gst, gsr)

    step()
    torch.cuda.synchronize()
    eager = [t.clone() for t in (pipe.img_color, pipe.img_T, pipe.loss, pipe.ids, pipe.tile_start)]
    eager_g = {k: v.clone() for k, v in grads.items()}
    eager_pose = pose.clone()
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        step()  # warm-up on the capture stream
    torch.cuda.current_stream().wait_stream(s)
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        step()
    for rep in range(3):
        for t in (pipe.img_color, pipe.img_T, pipe.loss):
            t.fill_(-1.0)  # eager work between replays
        torch.cuda.synchronize()
        graph.replay()
        torch.cuda.synchronize()
        for a, b in zip(eager, (pipe.img_color, pipe.img_T, pipe.loss, pipe.ids, pipe.tile_start)):
            assert torch.equal(a, b), rep
        for k in grads:
            torch.testing.assert_close(grads[k], eager_g[k], rtol=1e-5,
                                       atol=1e-6 * float(eager_g[k].abs().max()) + 1e-30)
        torch.testing.assert_close(pose, eager_pose, rtol=1e-5, atol=1e-5 * float(eager_pose.abs().max()))
        assert torch.count_nonzero(bwd_zero_part(pipe, vb)) == 0
