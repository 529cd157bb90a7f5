"""GPU parity of the render path (gs_project, gs_bin_sort, gs_render_fwd,
gs_loss, gs_render_bwd) against the FP64 oracle, through the C ABI."""

import numpy as np
import pytest
import torch

from paper_2602_21644_amd import gs, synth
from tests.gpu_util import (assert_grads_close, assert_image_close, bwd_zero_part, image_view, make_pipeline,
                            oracle_target, proj_view, torch_np)

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return gs.Context(0)


def _near_int(x, tol):
    return np.abs(x - np.round(x)) < tol


def test_project_parity(ctx, orc):
    g, cam, tcam = synth.tiny_scene()
    n = synth.n_gaussians(g)
    for c in (cam, tcam):
        views, pipe, gt, gst = make_pipeline(ctx, g, [c])
        gs.gs_project(ctx, views.s, gst, pipe.proj)
        torch.cuda.synchronize()
        got = proj_view(pipe, views, 0, n)
        ref = orc.project(g, c)
        kept = ref["kept"]
        gkept = got["key"] != 0xFFFFFFFF
        assert kept.sum() > 1900
        assert np.array_equal(gkept, kept)  # every kept one of this scene is on screen
        np.testing.assert_allclose(got["mean2d"][:, kept], ref["mean2d"][:, kept], rtol=1e-5, atol=1e-4)
        np.testing.assert_allclose(got["depth"][kept], ref["depth"][kept], rtol=1e-5)
        np.testing.assert_allclose(got["opacity"][kept], ref["opacity"][kept], rtol=1e-5)
        for i in range(3):
            sc = np.abs(ref["conic"][i, kept]).max()
            np.testing.assert_allclose(got["conic"][i, kept], ref["conic"][i, kept], rtol=1e-5, atol=1e-6 * sc)
        # integer radius: equal unless the FP64 extent sits within 1e-4 of an integer
        amb = _near_int(ref["extent"], 1e-4)
        assert np.all((got["radius"][kept] == ref["radius"][kept]) | amb[kept])
        x0, y0, x1, y1, empty = orc.tile_rect(ref["mean2d"], ref["radius"], kept, c["width"], c["height"])
        ambr = amb | _near_int(ref["mean2d"][0], 1e-4) | _near_int(ref["mean2d"][1], 1e-4)
        same = (got["rect"][:, 0] == x0) & (got["rect"][:, 1] == y0) & (got["rect"][:, 2] == x1) & (
            got["rect"][:, 3] == y1)
        assert np.all(same[kept] | ambr[kept])


def _bin_case(ctx, orc, seed, m, W, H, chunk, max_tiles=6):
    rect, key = synth.bin_inputs(seed, m, W, H, max_tiles=max_tiles)
    g = synth.static_gaussians(synth.rng_for(seed), m, W, H)
    cam = synth.camera(W, H)
    ctx.set_param("bin_chunk", chunk)
    views, pipe, gt, gst = make_pipeline(ctx, g, [cam], capacity=max(1024, m * max_tiles * max_tiles))
    M = pipe.M
    rect_full = np.zeros((M, 4), np.int16)
    rect_full[:, 0] = 1
    rect_full[:, 1] = 1
    key_full = np.full(M, 0xFFFFFFFF, np.uint32)
    rect_full[:m] = rect
    key_full[:m] = key
    pipe.rect.copy_(torch.from_numpy(rect_full.reshape(-1)))
    pipe.key.copy_(torch.from_numpy(key_full.view(np.int32)))
    gs.gs_bin_sort(ctx, views.s, gst, pipe.proj, pipe.bins, pipe.ws_bin)
    over, n_inst, _ = pipe.check()
    ids_ref, ranges = orc.bin_reference(rect, key, ((W + 15) // 16, (H + 15) // 16))
    assert not over
    assert n_inst == ids_ref.size
    ts = torch_np(pipe.tile_start).view(np.uint32).astype(np.int64)
    np.testing.assert_array_equal(ts[:-1], ranges[:, 0])
    np.testing.assert_array_equal(ts[1:], ranges[:, 1])
    got = torch_np(pipe.ids[:n_inst]).view(np.uint32)
    np.testing.assert_array_equal(got, ids_ref)


@pytest.mark.parametrize("seed,m,W,H,chunk", [(1, 3000, 64, 48, 256), (2, 20011, 200, 150, 1024),
                                              (3, 70000, 640, 480, 1024), (4, 5000, 640, 480, 2048),
                                              (5, 1, 64, 48, 512)])
def test_bin_sort_bitexact(ctx, orc, seed, m, W, H, chunk):
    _bin_case(ctx, orc, seed, m, W, H, chunk)
    ctx.set_param("bin_chunk", 1024)


def _prefix_selection(key, R):
    """The prefix rule: records with key < theta, theta the first boundary of
    the 4096-bin histogram of key >> 20 with at least R valid keys in front."""
    valid = key != 0xFFFFFFFF
    hist = np.bincount((key[valid] >> 20).astype(np.int64), minlength=4096)
    if hist.sum() <= R:
        return valid, hist
    b = int(np.searchsorted(np.cumsum(hist), R))  # first bin with cum >= R
    theta = (b + 1) << 20
    return valid & (key.astype(np.int64) < theta), hist


@pytest.mark.parametrize("seed,m,W,H,R", [(11, 3000, 64, 48, 500), (12, 70000, 640, 480, 4096),
                                          (13, 12000, 320, 240, 100000), (14, 50000, 1280, 720, 2000),
                                          (15, 20000, 320, 240, 100000), (16, 200000, 640, 480, 6000)])
def test_bin_sort_prefix_bitexact(ctx, orc, seed, m, W, H, R):
    """Prefix path: the lists equal the textbook stable sort restricted to the
    selected records, bit for bit; a selection above the path's cap gives
    empty lists and raises `incomplete`."""
    rect, key = synth.bin_inputs(seed, m, W, H, max_tiles=6)
    # spread depth keys over a realistic range so the selection is partial
    rng = np.random.default_rng(seed)
    z = np.cbrt(0.125 + rng.random(m) * (64 - 0.125)).astype(np.float32)
    z[rng.random(m) < 0.05] = np.float32(1.0)  # exact ties
    key = np.where(key == 0xFFFFFFFF, key, z.view(np.uint32)).astype(np.uint32)
    _prefix_case(ctx, orc, seed, m, W, H, R, rect, key)


@pytest.mark.parametrize("sizes", [(30, 400, 700, 1500), (385, 2000, 4500), (4200, 4300), (9000,)])
def test_bin_sort_prefix_tie_clusters(ctx, orc, sizes):
    """Records at exactly one depth (a surface facing the camera) fill one
    sort bucket: clusters of assorted sizes, below and above the 4096 records
    from which psort sorts a bucket with a network (two such buckets at once
    included), among spread keys and nearly equal ones; the lists must still
    be the stable sort bit for bit."""
    seed, W, H = 31, 320, 240
    m = 20000
    rect, key = synth.bin_inputs(seed, m, W, H, max_tiles=4)
    rng = np.random.default_rng(seed)
    z = np.cbrt(0.125 + rng.random(m) * (64 - 0.125)).astype(np.float32)
    perm = rng.permutation(np.nonzero(key != 0xFFFFFFFF)[0])  # clusters of visible records only
    o = 0
    for c, size in enumerate(sizes):
        zc = np.float32(0.6 + 0.05 * c)
        z[perm[o:o + size]] = zc
        # a few keys one ulp around the cluster
        z[perm[o + size:o + size + 8]] = np.nextafter(zc, np.float32(9), dtype=np.float32)
        o += size + 8
    key = np.where(key == 0xFFFFFFFF, key, z.view(np.uint32)).astype(np.uint32)
    R = int(sum(sizes)) + 600
    _prefix_case(ctx, orc, seed, m, W, H, R, rect, key)


def _prefix_case(ctx, orc, seed, m, W, H, R, rect, key):
    sel, hist = _prefix_selection(key, R)
    g = synth.static_gaussians(synth.rng_for(seed), m, W, H)
    views, pipe, gt, gst = make_pipeline(ctx, g, [synth.camera(W, H)], capacity=m * 36 + 1024, max_rank=R)
    M = pipe.M
    rect_full = np.zeros((M, 4), np.int16)
    rect_full[:, 0] = 1
    rect_full[:, 1] = 1
    key_full = np.full(M, 0xFFFFFFFF, np.uint32)
    rect_full[:m] = rect
    key_full[:m] = key
    pipe.rect.copy_(torch.from_numpy(rect_full.reshape(-1)))
    pipe.key.copy_(torch.from_numpy(key_full.view(np.int32)))
    pipe.key_hist.copy_(torch.from_numpy(hist.astype(np.int32)))
    for rep in range(2):  # the histogram is consumed and cleared by the call
        if rep == 1:
            pipe.key_hist.copy_(torch.from_numpy(hist.astype(np.int32)))
        gs.gs_bin_sort(ctx, views.s, gst, pipe.proj, pipe.bins, pipe.ws_bin)
        over, n_inst, inc = pipe.check()
        assert not over
        assert int(pipe.key_hist.abs().sum()) == 0
        # the view's truncation bit: some visible record was left out
        cap = ctx.get_param("prefix_cap")
        assert int(pipe.counters[3]) == int(sel.sum() < (key != 0xFFFFFFFF).sum() or sel.sum() > cap)
        if sel.sum() > cap:
            assert inc == 1 and n_inst == 0
            continue
        assert inc == 0
        ids_ref, ranges = orc.bin_reference(rect, np.where(sel, key, 0xFFFFFFFF), ((W + 15) // 16, (H + 15) // 16))
        assert n_inst == ids_ref.size
        ts = torch_np(pipe.tile_start).view(np.uint32).astype(np.int64)
        np.testing.assert_array_equal(ts[:-1], ranges[:, 0])
        np.testing.assert_array_equal(ts[1:], ranges[:, 1])
        np.testing.assert_array_equal(torch_np(pipe.ids[:n_inst]).view(np.uint32), ids_ref)


def test_project_key_histogram(ctx, orc):
    """gs_project adds every non-culled record to bin (key >> 20); the keys
    are the float32 camera depths the oracle also orders by."""
    g, cam, tcam = synth.tiny_scene()
    views, pipe, gt, gst = make_pipeline(ctx, g, [tcam], max_rank=100)
    gs.gs_project(ctx, views.s, gst, pipe.proj)
    torch.cuda.synchronize()
    ref = orc.project(g, tcam)
    x0, y0, x1, y1, empty = orc.tile_rect(ref["mean2d"], ref["radius"], ref["kept"], 64, 48)
    zb = ref["zkey"].astype(np.float32).view(np.uint32) >> 20
    expect = np.bincount(zb[~empty].astype(np.int64), minlength=4096)
    np.testing.assert_array_equal(torch_np(pipe.key_hist), expect)


def test_bin_sort_all_culled_and_overflow(ctx, orc):
    g = synth.static_gaussians(synth.rng_for(9), 500, 64, 48)
    g["mean"][2] = -1.0  # everything behind the camera
    views, pipe, gt, gst = make_pipeline(ctx, g, [synth.camera(64, 48)], capacity=16)
    pipe.forward(gst)
    over, n_inst, _ = pipe.check()
    assert not over and n_inst == 0
    im = image_view(pipe, views, 0)
    assert np.all(im["T"] == 1.0) and np.all(im["C"] == 0.0)
    g, cam, tcam = synth.tiny_scene()
    views, pipe, gt, gst = make_pipeline(ctx, g, [cam], capacity=100)
    pipe.forward(gst)
    over, n_inst, _ = pipe.check()
    assert over and n_inst > 100
    # the fused forward and loss under overflow: no image, a defined zero loss
    pipe.loss.fill_(float("nan"))
    tgt = torch.zeros(3 * pipe.P, device="cuda")
    pipe.forward_loss(gst, tgt, tgt[:pipe.P].contiguous())
    over, n_inst, _ = pipe.check()
    assert over and float(pipe.loss[0]) == 0.0


def test_render_fwd_parity_tiny(ctx, orc):
    g, cam, tcam = synth.tiny_scene()
    for c, bg in ((cam, (0, 0, 0)), (tcam, (0.2, 0.5, 0.9))):
        views, pipe, gt, gst = make_pipeline(ctx, g, [c], bg=bg)
        pipe.forward(gst)
        torch.cuda.synchronize()
        got = image_view(pipe, views, 0)
        ref = orc.render(orc.project(g, c), g, c, bg=bg)
        assert_image_close(got, ref, ref["margin"])


def test_render_fwd_deterministic(ctx):
    g, cam, tcam = synth.moving_box_scene(2, 20000, 320, 240)[:3]
    views, pipe, gt, gst = make_pipeline(ctx, g, [cam])
    pipe.forward(gst)
    a = [t.clone() for t in (pipe.img_color, pipe.img_depth, pipe.img_T, pipe.ids)]
    pipe.forward(gst)
    b = [pipe.img_color, pipe.img_depth, pipe.img_T, pipe.ids]
    for x, y in zip(a, b):
        assert torch.equal(x, y)


def test_render_fwd_parity_640(ctx, orc):
    g, cam, tcam, g_t, sl = synth.moving_box_scene(2, 30000, 640, 480)
    views, pipe, gt, gst = make_pipeline(ctx, g, [tcam])
    pipe.forward(gst)
    torch.cuda.synchronize()
    got = image_view(pipe, views, 0)
    ref = orc.render(orc.project(g, tcam), g, tcam)
    assert_image_close(got, ref, ref["margin"])


def _loss_bwd_case(ctx, orc, g, cam, tcam, weight_mode=0, gtw=0, bg=(0, 0, 0)):
    """GPU loss + backward against the oracle. Pixels where the forward sits
    within the margin of a discontinuity, or where a residual is within 1e-5
    of zero (sign of the L1 adjoint ambiguous), get zero pixel adjoints on
    both sides, so the comparison covers the continuous part of the adjoint."""
    tc, td = oracle_target(orc, g, tcam)
    n = synth.n_gaussians(g)
    views, pipe, gt, gst = make_pipeline(ctx, g, [cam], bg=bg)
    pipe.set_loss_params(weight_mode=weight_mode, grad_through_weight=gtw)
    pipe.forward(gst)
    tcd, tdd = torch.from_numpy(tc.reshape(-1)).cuda(), torch.from_numpy(td).cuda()
    pipe.loss_and_grads(tcd, tdd)
    pr = orc.project(g, cam)
    im = orc.render(pr, g, cam, bg=bg)
    L = orc.loss(im, tc, td, weight_mode=weight_mode, grad_through_weight=bool(gtw))
    amb = (im["margin"] < 1e-5) | (np.abs(im["C"] - tc).min(axis=0) < 1e-5) | (
        (td > 0) & (np.abs(im["D"] - td) < 1e-5))
    P = amb.size
    keep = torch.from_numpy(~amb).cuda()
    pipe.dC.view(3, P).mul_(keep)
    pipe.dD.mul_(keep)
    pipe.dM.mul_(keep)
    pipe.dT.mul_(keep)
    grads = gs.alloc_grads(n)
    pose = torch.zeros(6, device="cuda")
    pipe.backward(gst, gs.grads_struct(grads, pose))
    torch.cuda.synchronize()
    k = ~amb
    g2d = orc.render_backward(pr, g, cam, L["dC"] * k, L["dD"] * k, L["dM"] * k, L["dT"] * k, bg=bg)
    rg = orc.project_backward(g, cam, g2d)
    return pipe, views, grads, pose, L, im, rg


@pytest.mark.parametrize("weight_mode,gtw", [(0, 0), (1, 0), (0, 1)])
def test_loss_and_backward_parity_tiny(ctx, orc, weight_mode, gtw):
    g, cam, tcam = synth.tiny_scene()
    pipe, views, grads, pose, L, im, rg = _loss_bwd_case(ctx, orc, g, cam, tcam, weight_mode, gtw)
    assert abs(float(pipe.loss[0]) - L["loss"]) <= 1e-4 * abs(L["loss"])
    for k in ("mean", "log_scale", "quat", "opacity_logit", "color"):
        assert_grads_close(torch_np(grads[k]), rg[k], name=k)
    assert_grads_close(torch_np(pose), rg["pose"], name="pose")


def test_backward_parity_640(ctx, orc):
    g, cam, tcam, g_t, sl = synth.moving_box_scene(3, 20000, 640, 480)
    pipe, views, grads, pose, L, im, rg = _loss_bwd_case(ctx, orc, g, cam, tcam, bg=(0.1, 0.1, 0.1))
    assert abs(float(pipe.loss[0]) - L["loss"]) <= 1e-4 * abs(L["loss"])
    for k in ("mean", "log_scale", "quat", "opacity_logit", "color"):
        assert_grads_close(torch_np(grads[k]), rg[k], name=k)
    assert_grads_close(torch_np(pose), rg["pose"], name="pose")


def test_backward_zero_ws_invariant_and_pose_only(ctx, orc):
    """Two backward calls in a row agree (the scratch is left zero-filled);
    pose-only mode gives the same pose gradient."""
    g, cam, tcam = synth.tiny_scene(seed=4)
    tc, td = oracle_target(orc, g, tcam)
    n = synth.n_gaussians(g)
    views, pipe, gt, gst = make_pipeline(ctx, g, [cam])
    pipe.forward(gst)
    pipe.loss_and_grads(torch.from_numpy(tc.reshape(-1)).cuda(), torch.from_numpy(td).cuda())
    outs = []
    for pose_only in (False, False, True):
        grads = gs.alloc_grads(n)
        pose = torch.zeros(6, device="cuda")
        pipe.backward(gst, gs.grads_struct(None if pose_only else grads, pose, pose_only=pose_only))
        torch.cuda.synchronize()
        outs.append((grads, pose.clone()))
    # float atomics make the summation order (and the last bits) vary
    for k in outs[0][0]:
        torch.testing.assert_close(outs[0][0][k], outs[1][0][k], rtol=1e-5, atol=1e-6 * float(outs[0][0][k].abs().max()))
    torch.testing.assert_close(outs[0][1], outs[2][1], rtol=1e-5, atol=1e-5 * float(outs[0][1].abs().max()))
    assert torch.count_nonzero(bwd_zero_part(pipe, views)) == 0  # the scratch is left zero-filled


def _host_tile_work_bounds(nlast, W, H, tile_len):
    """Bounds on the per-tile work (the entries the tile's four 16x4 pixel
    groups evaluated): each group evaluates at least the entry each of its
    pixels composited last (distinct nonzero n_last values), and at most its
    whole list in groups of four per staged batch."""
    gx, gy = (W + 15) // 16, (H + 15) // 16
    pad = np.zeros((gy * 16, gx * 16), np.int64)
    pad[:H, :W] = nlast.reshape(H, W)
    grp = pad.reshape(gy, 4, 4, gx, 16).transpose(0, 3, 1, 2, 4).reshape(gy * gx, 4, 64)
    lo = np.array([sum(len(set(g[g > 0].tolist())) for g in t) for t in grp], np.int64)
    hi = 4 * (tile_len + 3 * ((tile_len + 63) // 64))  # batches of at least 64 entries
    return lo, hi


def test_backward_tile_order(ctx, orc):
    """The forward's per-tile work lies within the bounds its definition
    implies; the backward run heaviest-tile-first, and with 1, 2 or 8
    accumulator copies, gives the gradients of the plain tile order."""
    g, cam, tcam, g_t, sl = synth.moving_box_scene(8, 30000, 640, 480)
    cam2 = synth.camera(320, 240, cam["T_cw"])
    views, pipe, gt, gst = make_pipeline(ctx, g, [cam, cam2], bg=(0.1, 0.2, 0.3))
    pipe.forward(gst)
    tc0, td0 = pipe.img_color.clone(), pipe.img_depth.clone()
    tc, td = (tc0 * 0.9).contiguous(), (td0 * 1.05).contiguous()
    nl = torch_np(pipe.img_nlast).view(np.uint32).astype(np.int64)
    work = torch_np(pipe.img_tile_work).view(np.uint32).astype(np.int64)[:views.tile_count]
    ts = torch_np(pipe.tile_start).view(np.uint32).astype(np.int64)[:views.tile_count + 1]
    tlen = np.diff(ts)
    nt0 = 40 * 30
    lo0, hi0 = _host_tile_work_bounds(nl[:640 * 480], 640, 480, tlen[:nt0])
    lo1, hi1 = _host_tile_work_bounds(nl[640 * 480:], 320, 240, tlen[nt0:])
    lo, hi = np.concatenate([lo0, lo1]), np.concatenate([hi0, hi1])
    assert np.all(work >= lo) and np.all(work <= hi)
    assert work.sum() > lo.sum()
    host = work
    # the forward dealt the backward's order: a permutation with its marker,
    # heaviest first (by log-scale bucket of the work) round by round
    T = views.tile_count
    tw = torch_np(pipe.img_tile_work).view(np.uint32).astype(np.int64)
    assert tw[2 * T] == T + 1
    order = tw[T:2 * T]
    np.testing.assert_array_equal(np.sort(order), np.arange(T))
    k = (host.astype(np.float32).view(np.uint32).astype(np.int64) >> 19) - (127 << 4) + 1
    bucket = 2047 - np.clip(k, 0, 2047)  # smaller = heavier
    ncu = ctx.get_param("n_cu")
    rounds = [bucket[order[r:r + ncu]] for r in range(0, T, ncu)]
    for a_, b_ in zip(rounds, rounds[1:]):
        assert a_.max() <= b_.min()
    pipe.loss_and_grads(tc, td)
    n = synth.n_gaussians(g)
    outs = []
    # (tile order, accumulator copies); the scratch was sized for 8 copies
    for order, copies in ((1, 8), (0, 8), (1, 8), (1, 1), (0, 2)):
        ctx.set_param("tile_order", order)
        ctx.set_param("bwd_copies", copies)
        grads = gs.alloc_grads(n)
        pose = torch.zeros(12, device="cuda")
        pipe.backward(gst, gs.grads_struct(grads, pose))
        torch.cuda.synchronize()
        outs.append((grads, pose))
        if copies == 8:
            assert torch.count_nonzero(bwd_zero_part(pipe, views)) == 0
    ctx.set_param("tile_order", 1)
    ctx.set_param("bwd_copies", 8)
    assert ctx.get_param("n_cu") > 0
    # only the order of the float atomics differs: agreement far inside the
    # 1e-3 gradient tolerance
    for other in outs[1:]:
        for k in outs[0][0]:
            assert_grads_close(torch_np(other[0][k]), torch_np(outs[0][0][k]), rel=1e-4, name=k)
        assert_grads_close(torch_np(other[1]), torch_np(outs[0][1]), rel=1e-4, name="pose")
    assert float(outs[0][0]["color"].abs().sum()) > 0


@pytest.mark.parametrize("seed,n,W,H,max_rank", [(21, 20000, 640, 480, 0), (22, 200000, 320, 240, 8192),
                                                 (23, 3000, 100, 75, 0)])
def test_wave_cull_exact(ctx, seed, n, W, H, max_rank):
    """Skipping, per 16x4 pixel strip, the entries whose alpha >= 1/255 region
    misses the strip (forward and backward) leaves every image bit-identical,
    and so does the forward's launch order (the first forward runs in natural
    order, the later ones in the order the last one dealt); the gradients
    agree up to the order of their float atomics. The per-tile work (entries
    evaluated) shrinks with the skipping and repeats exactly without a
    change."""
    g, cam, tcam, g_t, sl = synth.moving_box_scene(seed, n, W, H)
    views, pipe, gt, gst = make_pipeline(ctx, g, [cam], max_rank=max_rank, bg=(0.2, 0.1, 0.0))
    outs, grads, works = [], [], []
    tc = td = None
    for cull in (1, 0, 1):
        ctx.set_param("wave_cull", cull)
        pipe.forward(gst)
        if tc is None:
            tc, td = (pipe.img_color * 0.8).contiguous(), (pipe.img_depth * 1.1).contiguous()
        pipe.loss_and_grads(tc, td)
        gr = gs.alloc_grads(n)
        pose = torch.zeros(6, device="cuda")
        pipe.backward(gst, gs.grads_struct(gr, pose))
        torch.cuda.synchronize()
        outs.append([t.clone() for t in (pipe.img_color, pipe.img_depth, pipe.img_mp, pipe.img_T, pipe.img_nlast)])
        works.append(pipe.img_tile_work[:views.tile_count].clone())
        grads.append((gr, pose))
    ctx.set_param("wave_cull", 1)
    over, n_inst, inc = pipe.check()
    assert not over and n_inst > 0
    for other in outs[1:]:
        for a, b in zip(outs[0], other):
            assert torch.equal(a, b)
    assert torch.equal(works[0], works[2])
    assert int(works[0].sum()) <= int(works[1].sum())
    for other in grads[1:]:
        for k in grads[0][0]:
            assert_grads_close(torch_np(other[0][k]), torch_np(grads[0][0][k]), rel=1e-4, name=k)
        assert_grads_close(torch_np(other[1]), torch_np(grads[0][1]), rel=1e-4, name="pose")


def test_max_rank_prefix_lists(ctx, orc):
    """Binning only the records in front of the rank-R threshold gives exact
    prefixes of the full lists (every tile checked). At the smallest exact
    rank (no tile runs out of its prefix) the image is identical to the
    full-list image and matches the oracle."""
    from paper_2602_21644_amd import optim
    g, cam, tcam, g_t, sl = synth.moving_box_scene(5, 200000, 320, 240)
    views, pipe, gt, gst = make_pipeline(ctx, g, [cam])
    pipe.forward(gst)
    full_ids = torch_np(pipe.ids).view(np.uint32).copy()
    full_ts = torch_np(pipe.tile_start).view(np.uint32).astype(np.int64)
    full_img = [t.clone() for t in (pipe.img_color, pipe.img_depth, pipe.img_mp, pipe.img_T, pipe.img_nlast)]
    R_exact, _ = optim.choose_rank(ctx, views, gst, synth.n_gaussians(g))
    assert R_exact > 0
    R_short = R_exact // 2 if R_exact > 256 else 64
    for R in (R_short, R_exact):
        views2, pipe2, gt2, gst2 = make_pipeline(ctx, g, [cam], max_rank=R)
        pipe2.forward(gst2)
        over, n_inst, inc = pipe2.check()
        assert not over
        ts = torch_np(pipe2.tile_start).view(np.uint32).astype(np.int64)
        ids = torch_np(pipe2.ids).view(np.uint32)
        assert 0 < n_inst < full_ts[-1]
        for t in range(len(ts) - 1):
            mine = ids[ts[t]:ts[t + 1]]
            full = full_ids[full_ts[t]:full_ts[t + 1]]
            np.testing.assert_array_equal(mine, full[:len(mine)])
        if R == R_exact:
            assert inc == 0
            for a, b in zip(full_img, (pipe2.img_color, pipe2.img_depth, pipe2.img_mp, pipe2.img_T,
                                       pipe2.img_nlast)):
                assert torch.equal(a, b)
            ref = orc.render(orc.project(g, cam), g, cam)
            assert_image_close(image_view(pipe2, views2, 0), ref, ref["margin"])
        elif R_exact > 256:
            assert inc == 1  # R_exact is the smallest exact power of two from 256


@pytest.mark.parametrize("prefix", [True, False])
def test_rank_above_visible_count_is_exact(ctx, orc, prefix):
    """max_rank below the record count but above the visible count: the
    lists keep every visible record, so they are the full lists and no tile
    raises `incomplete`, though most pixels are unsaturated; a rank below the
    visible count does raise it. Both on the prefix path and on the
    rank-limited full path (key_hist NULL)."""
    g, cam, _ = synth.tiny_scene(seed=6)
    n = synth.n_gaussians(g)
    g["mean"][2, 500:] = -1.0  # 500 of 2000 in front of the camera
    views, pipe, gt, gst = make_pipeline(ctx, g, [cam])
    pipe.forward(gst)
    full = [t.clone() for t in (pipe.img_color, pipe.img_depth, pipe.img_mp, pipe.img_T, pipe.img_nlast)]
    n_full = pipe.check()[1]
    assert float((pipe.img_T > 0.5).float().mean()) > 0.1  # unsaturated pixels
    ref = orc.render(orc.project(g, cam), g, cam)
    for R, inc_want in ((1024, 0), (64, 1)):
        print(f"\n[rank] prefix={prefix} R={R} (n={n})", flush=True)
        views2, pipe2, gt2, gst2 = make_pipeline(ctx, g, [cam], max_rank=R, full_proj=not prefix)
        if not prefix:
            pipe2.proj.key_hist = None  # rank-limited full lists
        pipe2.forward(gst2)
        over, n_inst, inc = pipe2.check()
        assert not over and inc == inc_want, (R, inc)
        if inc_want == 0:
            assert n_inst == n_full
            for a, b in zip(full, (pipe2.img_color, pipe2.img_depth, pipe2.img_mp, pipe2.img_T, pipe2.img_nlast)):
                assert torch.equal(a, b)
            assert_image_close(image_view(pipe2, views2, 0), ref, ref["margin"])


def test_full_size_full_lists(ctx, orc):
    """1M Gaussians at 640x480 on the full-list path: the ~45M list entries
    equal the stable sort of the (tile, depth) keys bit for bit (built from
    the GPU's rects and keys), and every pixel matches the oracle."""
    g, cam, tcam, g_t, sl = synth.moving_box_scene(7, 1_000_000, 640, 480)
    n = synth.n_gaussians(g)
    views, pipe, gt, gst = make_pipeline(ctx, g, [cam], capacity=80_000_000, full_proj=False)
    pipe.forward(gst)
    over, n_inst, inc = pipe.check()
    assert not over and inc == 0
    print(f"\n[full lists] {n_inst} list entries")
    assert n_inst > 30_000_000
    rect = torch_np(pipe.rect).reshape(-1, 4)[:n]
    key = torch_np(pipe.key).view(np.uint32)[:n]
    ids_ref, ranges = orc.bin_reference_np(rect, key, (40, 30))
    assert n_inst == ids_ref.size
    ts = torch_np(pipe.tile_start).view(np.uint32).astype(np.int64)
    np.testing.assert_array_equal(ts[:-1], ranges[:, 0])
    np.testing.assert_array_equal(ts[1:], ranges[:, 1])
    np.testing.assert_array_equal(torch_np(pipe.ids[:n_inst]).view(np.uint32), ids_ref)
    del ids_ref, ranges
    got = image_view(pipe, views, 0)
    T = got["T"]
    # the kernel stops before T drops below the float32 threshold 1e-4f,
    # which is a little under the double 1e-4
    assert T.min() >= np.float32(1e-4) and T.max() <= 1.0
    assert np.all(got["M"] <= 1 - T + 1e-5)
    ref = orc.render(orc.project(g, cam), g, cam)
    assert_image_close(got, ref, ref["margin"])


@pytest.mark.parametrize("seed,n,W,H,weight_mode,gtw,max_rank,nviews", [
    (21, 3000, 64, 48, 0, 0, 0, 1), (22, 60000, 333, 250, 1, 1, 0, 1), (23, 200000, 640, 480, 0, 1, 1024, 1),
    (24, 40000, 320, 240, 0, 0, 0, 3)])
def test_render_fwd_loss_fused(ctx, seed, n, W, H, weight_mode, gtw, max_rank, nviews):
    """gs_render_fwd_loss writes the images and pixel adjoints of gs_render_fwd
    followed by gs_loss bit for bit; the loss differs only in the order of its
    float64 sum."""
    g, cam, tcam, g_t, sl = synth.moving_box_scene(seed, n, W, H)
    cams = [cam, tcam, cam][:nviews]
    views, pipe, gt, gst = make_pipeline(ctx, g, cams, max_rank=max_rank, bg=(0.1, 0.2, 0.3))
    pipe.set_loss_params(weight_mode=weight_mode, grad_through_weight=gtw)
    pipe.forward(gst)
    rng = np.random.default_rng(seed)
    tc = (pipe.img_color * 0.8 + 0.05).contiguous()
    mask = torch.from_numpy(rng.random(pipe.P) < 0.7).cuda()
    td = torch.where(mask, pipe.img_depth * 1.1, torch.zeros_like(pipe.img_depth)).contiguous()
    pipe.loss_and_grads(tc, td)
    torch.cuda.synchronize()
    inc_ref = pipe.check()[2]
    outs = ("img_color", "img_depth", "img_mp", "img_T", "img_nlast", "dC", "dD", "dM", "dT")
    ref = {k: getattr(pipe, k).clone() for k in outs}
    ref_loss = pipe.loss.clone()
    for k in outs:  # a value no kernel writes, so a missed pixel shows
        t = getattr(pipe, k)
        if t.dtype == torch.float32:
            t.fill_(float("nan"))
        else:
            t.fill_(0x7FFFFFFF)
    pipe.loss.fill_(float("nan"))
    pipe.forward_loss(gst, tc, td)
    torch.cuda.synchronize()
    over, n_inst, inc = pipe.check()
    assert not over and inc == inc_ref  # same lists, same flag
    for k in outs:
        assert torch.equal(getattr(pipe, k), ref[k]), k
    torch.testing.assert_close(pipe.loss, ref_loss, rtol=1e-6, atol=0)
    assert float(ref_loss.abs().min()) > 0


def _thin_gaussians_on_strip_edges(seed, n, W, H):
    """Gaussians that test the strip test's edges: one long and one very short
    axis at every angle, projected means a fraction of a pixel from 16x4 strip
    and 16x16 tile boundaries, opacities from just below to well above
    1/255."""
    rng = synth.rng_for(seed)
    fx, fy, cx, cy = synth.intrinsics(W, H)
    gx, gy = W // 16, H // 16
    px = rng.integers(0, gx, n) * 16 + rng.choice([-0.4, -0.01, 0.0, 0.01, 0.4, 7.5], n)
    py = rng.integers(0, gy * 4, n) * 4 + rng.choice([-0.6, -0.02, 0.0, 0.02, 0.6, 1.5], n)
    z = rng.uniform(1.0, 3.0, n)
    mean = np.stack([z * (px - cx) / fx, z * (py - cy) / fy, z])
    log_scale = np.stack([rng.uniform(-2.5, -1.0, n), rng.uniform(-7.0, -5.0, n), rng.uniform(-7.0, -5.0, n)])
    ang = rng.uniform(0.0, np.pi, n)  # rotation about the optical axis
    quat = np.stack([np.cos(ang / 2), np.zeros(n), np.zeros(n), np.sin(ang / 2)])
    opl = np.log(1.0 / 255.0 / (1.0 - 1.0 / 255.0)) + rng.choice([-0.05, 0.02, 0.3, 2.0, 6.0], n)
    g = synth._pack(mean, log_scale, quat, opl, rng.random((3, n)), rng.random(n))
    return g, synth.camera(W, H)


@pytest.mark.parametrize("seed", [31, 32])
def test_wave_cull_exact_thin_edges(ctx, seed):
    """The strip test keeps every strip in which some pixel reaches alpha >=
    1/255, also for needle-like Gaussians at every angle whose means sit on
    strip and tile edges and whose opacities straddle 1/255: the images are
    bit-identical with and without culling, and so are the colour and opacity
    gradients up to the order of their float atomics. (The geometry
    gradients of needles are ill-conditioned: per-tile conic adjoints of
    opposite sign meet in the atomic sums and the chain through the inverse
    covariance amplifies their rounding, so that two runs with the same
    settings already differ by percents; they are not compared here.)"""
    n, W, H = 4000, 320, 240
    g, cam = _thin_gaussians_on_strip_edges(seed, n, W, H)
    views, pipe, gt, gst = make_pipeline(ctx, g, [cam], bg=(0.3, 0.2, 0.1))
    outs, grads = [], []
    tc = td = None
    for cull in (1, 0):
        ctx.set_param("wave_cull", cull)
        pipe.forward(gst)
        if tc is None:
            tc, td = (pipe.img_color * 0.7).contiguous(), (pipe.img_depth * 1.2).contiguous()
        pipe.loss_and_grads(tc, td)
        gr = gs.alloc_grads(n)
        pose = torch.zeros(6, device="cuda")
        pipe.backward(gst, gs.grads_struct(gr, pose))
        torch.cuda.synchronize()
        outs.append([t.clone() for t in (pipe.img_color, pipe.img_depth, pipe.img_mp, pipe.img_T, pipe.img_nlast)])
        grads.append((gr, pose))
    ctx.set_param("wave_cull", 1)
    over, n_inst, inc = pipe.check()
    assert not over and n_inst > 0
    assert float((1.0 - outs[0][3]).sum()) > 0.05 * W * H  # the needles cover the image
    for a, b in zip(outs[0], outs[1]):
        assert torch.equal(a, b)
    for k in ("color", "opacity_logit"):
        assert_grads_close(torch_np(grads[1][0][k]), torch_np(grads[0][0][k]), rel=1e-5, name=k)
    for k in grads[0][0]:
        assert np.isfinite(torch_np(grads[1][0][k])).all() and np.isfinite(torch_np(grads[0][0][k])).all()


@pytest.mark.parametrize("seed,n,W,H", [(71, 200000, 320, 240), (72, 1_000_000, 640, 480), (73, 3000, 64, 48)])
def test_keys_only_projection(ctx, orc, seed, n, W, H):
    """On the prefix path without planar outputs gs_project writes depth keys
    from its cheap screen test: every Gaussian the full projection keys gets
    the same key (the test never drops one it keeps), and the lists binned
    from those keys are exact prefixes of the full lists; at an exact rank the
    images equal the full-list images bit for bit."""
    from paper_2602_21644_amd import optim
    g, cam, tcam, g_t, sl = synth.moving_box_scene(seed, n, W, H)
    for c in (cam, tcam):
        views, full, gt, gst = make_pipeline(ctx, g, [c], capacity=max(1 << 16, 60 * n))
        full.forward(gst)
        over, _, _ = full.check()
        assert not over
        ex_key = torch_np(full.key).view(np.uint32)[:n].copy()
        full_ids = torch_np(full.ids).view(np.uint32).copy()
        full_ts = torch_np(full.tile_start).view(np.uint32).astype(np.int64)
        R, _ = optim.choose_rank(ctx, views, gst, n)
        if R == 0:
            R = 256  # sparse scene: a truncated prefix still has to be exact
        ko = gs.Pipeline(ctx, views, capacity=max(1 << 16, 60 * n), max_rank=R)
        ko.forward(gst)
        assert ko.proj.keys_only == 1
        over, n_inst, inc = ko.check()
        assert not over
        sk = torch_np(ko.key).view(np.uint32)[:n]
        kept = ex_key != 0xFFFFFFFF
        np.testing.assert_array_equal(sk[kept], ex_key[kept])
        print(f"\n[keys only] {kept.sum()} keyed exactly, {int((sk != 0xFFFFFFFF).sum())} by the screen test, "
              f"rank {R}, incomplete {inc}")
        ts = torch_np(ko.tile_start).view(np.uint32).astype(np.int64)
        ids = torch_np(ko.ids).view(np.uint32)
        for t in range(len(ts) - 1):
            mine = ids[ts[t]:ts[t + 1]]
            np.testing.assert_array_equal(mine, full_ids[full_ts[t]:full_ts[t] + len(mine)])
        if inc == 0:
            for a, b in zip((full.img_color, full.img_depth, full.img_mp, full.img_T, full.img_nlast),
                            (ko.img_color, ko.img_depth, ko.img_mp, ko.img_T, ko.img_nlast)):
                assert torch.equal(a, b)
