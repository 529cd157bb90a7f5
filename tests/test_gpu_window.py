"""The mapping window at full size: 1M Gaussians, 8 keyframes at 640x480 in
one batch.

* The window's gradient (the sum over the keyframes, to every Gaussian
  parameter) against central finite differences of the FP64 oracle's forward
  on a 5k-Gaussian subset: 16 random directions restricted to the subset, and
  single coordinates of 64 of its Gaussians.
* The whole chain of one frame (iterations of the window on the full
  objective of Eq. (27), then the MP update
  of the newest keyframe in log-odds mode, the prune flag at MP > 0.8 and the
  compaction of parameters, MP and Adam moments) captured in one HIP graph:
  the replay keeps its invariants, and the compaction equals removing the
  flagged Gaussians.
"""

import numpy as np
import pytest
import torch

from paper_2602_21644_amd import gs, optim, synth
from tests.gpu_util import torch_np

pytestmark = pytest.mark.gpu

N, W, H, V = 1_000_000, 640, 480, 8
P = W * H
GROUPS = ("mean", "log_scale", "quat", "opacity_logit", "color")
NDIR = 16


@pytest.fixture(scope="module")
def ctx():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return gs.Context(0)


@pytest.fixture(scope="module")
def window(orc):
    """The scene, 8 keyframes 5 frames apart, and each keyframe's observed
    frame: the oracle's render at a pose 0.5 degree / 1 cm away (at this
    density the static Gaussians in front hide the boxes, so the residual
    comes from the camera motion)."""
    g, cam, tcam, g_t, sl = synth.moving_box_scene(3, N, W, H)
    cams = synth.window_cameras(4, V, W, H, spacing=5)
    rng = synth.rng_for(5)
    tcams = [synth.camera(W, H, synth.perturbed_pose(rng, deg=0.5, trans=0.01, base=c["T_cw"])) for c in cams]
    tc, td = [], []
    for c in tcams:
        it = orc.render(orc.project(g, c), g, c)
        tc.append(it["C"])
        td.append(np.where(1.0 - it["T"] >= 0.5, it["D"], 0.0))
    return dict(g=g, cams=cams, tc=tc, td=td, slices=sl)


def _gpu_window_grads(ctx, orc, w):
    """GPU window gradients with the pixel adjoints zeroed where the oracle's
    compositing decisions sit within the margin of a threshold or a residual
    lies within 1e-5 of zero; returns (grads, oracle data per view)."""
    g, cams = w["g"], w["cams"]
    views = gs.ViewBatch(cams, N)
    gt = gs.to_device(g)
    gst = gs.gaussians_struct(gt)
    R, n_inst = optim.choose_rank(ctx, views, gst, N)
    pipe = gs.Pipeline(ctx, views, capacity=int(n_inst * 1.25) + 4096, max_rank=R)
    tcd = torch.from_numpy(np.concatenate(w["tc"], axis=1).astype(np.float32).reshape(-1)).cuda()
    tdd = torch.from_numpy(np.concatenate(w["td"]).astype(np.float32)).cuda()
    pipe.forward_loss(gst, tcd, tdd)
    over, _, inc = pipe.check()
    assert not over and inc == 0
    per_view, keep = [], []
    for v, c in enumerate(cams):
        pr = orc.project(g, c)
        im = orc.render(pr, g, c)
        L = orc.loss(im, w["tc"][v], w["td"][v])
        td = w["td"][v]
        amb = (im["margin"] < 1e-5) | (np.abs(im["C"] - w["tc"][v]).min(axis=0) < 1e-5) | (
            (td > 0) & (np.abs(im["D"] - td) < 1e-5))
        per_view.append(dict(pr=pr, im=im, L=L, ok=~amb))
        keep.append(~amb)
    k = torch.from_numpy(np.concatenate(keep)).cuda()
    pipe.dC.view(3, -1).mul_(k)
    pipe.dD.mul_(k)
    grads = gs.alloc_grads(N)
    pose = torch.zeros(6 * V, device="cuda")
    pipe.backward(gst, gs.grads_struct(grads, pose))
    torch.cuda.synchronize()
    return {k_: torch_np(grads[k_]).astype(np.float64) for k_ in GROUPS}, per_view


def _loss_restricted(orc, gp, c, tc, td, wv, pix, sub=None):
    """The loss over the pixel list `pix` with the weight held at wv. With
    `sub`, only those Gaussians are rendered: exact when they include every
    Gaussian whose tile rect reaches a pixel of the list."""
    if sub is not None:
        gp = {k: np.ascontiguousarray(x[..., sub]) for k, x in gp.items()}
    im = orc.render(orc.project(gp, c), gp, c, pixels=pix)
    return orc.loss(im, tc[:, pix], td[pix], w_fixed=wv[pix])["loss"]


def test_window_gradients_finite_differences(ctx, orc, window):
    grads, pv = _gpu_window_grads(ctx, orc, window)
    check_window_gradients(orc, window, grads, pv)


def check_window_gradients(orc, w, grads, pv):
    g64 = {k: np.asarray(v, np.float64) for k, v in w["g"].items()}
    # the subset: every Gaussian the oracle's window gradient touches, filled
    # up to 5,000 with untouched ones that some keyframe keeps
    touched = np.zeros(N, bool)
    for v, c in enumerate(w["cams"]):
        L = pv[v]["L"]
        ok = pv[v]["ok"]
        g2d = orc.render_backward(pv[v]["pr"], g64, c, L["dC"] * ok, L["dD"] * ok)
        touched |= np.abs(g2d).sum(axis=0) > 0
    rng = np.random.default_rng(17)
    kept_any = np.zeros(N, bool)
    for p in pv:
        kept_any |= p["pr"]["kept"]
    T = np.nonzero(touched)[0]
    fill = rng.choice(np.nonzero(kept_any & ~touched)[0], size=max(0, 5000 - T.size), replace=False)
    S = np.sort(np.concatenate([T, fill]))
    print(f"\n[window fd] touched {T.size}, subset {S.size}")
    assert S.size == 5000 and T.size > 500
    # untouched members get no gradient on the GPU either
    for k in GROUPS:
        assert np.all(grads[k].reshape(-1, N)[:, fill] == 0)

    def window_loss(gp):
        tot = 0.0
        for v, c in enumerate(w["cams"]):
            pix = np.nonzero(pv[v]["ok"])[0]
            tot += _loss_restricted(orc, gp, c, w["tc"][v], w["td"][v], pv[v]["L"]["w"], pix)
        return tot

    # 16 directions on the subset. The step is tiny so that no alpha or stop
    # threshold among the millions of (pixel, Gaussian) pairs is crossed; a
    # direction whose difference quotient changes with the step crossed one
    # and is not used.
    accepted = 0
    for i in range(NDIR):
        d = {k: np.zeros_like(g64[k]) for k in GROUPS}
        for k in GROUPS:
            d[k].reshape(-1, N)[:, S] = rng.normal(size=(d[k].reshape(-1, N).shape[0], S.size))
        an = sum(float((grads[k] * d[k]).sum()) for k in GROUPS)

        def quotient(h):
            vals = [window_loss({k: g64[k] + s * h * d[k] if k in d else g64[k] for k in g64}) for s in (1, -1)]
            return (vals[0] - vals[1]) / (2 * h)

        fd = quotient(1e-10)
        if abs(fd - an) > 1e-3 * abs(fd):
            fd2 = quotient(3e-11)
            assert abs(fd2 - fd) > 1e-4 * abs(fd), (i, "gradient mismatch", an, fd, fd2)
            print(f"[window fd] direction {i}: a threshold was crossed ({fd:.6g} vs {fd2:.6g}); not used")
            continue
        accepted += 1
        print(f"[window fd] direction {i}: GPU {an:.8g} FD {fd:.8g} rel {abs(fd - an) / abs(fd):.2e}")
    assert accepted >= min(12, NDIR)

    # single coordinates of the 64 touched Gaussians with the smallest
    # footprints: the loss restricted to the pixels of the Gaussian's rect,
    # rendered from the Gaussians whose rects reach them
    rects = []
    for v, c in enumerate(w["cams"]):
        pr = pv[v]["pr"]
        rects.append(orc.tile_rect(pr["mean2d"], pr["radius"], pr["kept"], W, H, tile=1))
    area = np.zeros(T.size)
    for r in rects:
        area += np.where(r[4][T], 0, (r[2][T] - r[0][T] + 1) * (r[3][T] - r[1][T] + 1))
    chosen = T[np.argsort(area)[:64]]
    print(f"[window fd] footprints of the 64 coordinates: {int(area[np.argsort(area)[:64]].max())} px at most "
          f"(over the keyframes)")
    names = [(k, c_) for k in GROUPS for c_ in range(g64[k].reshape(-1, N).shape[0])]
    checked = 0
    for gi in chosen:
        k, c_ = names[rng.integers(len(names))]
        an = grads[k].reshape(-1, N)[c_, gi]
        plans = []
        for v, c in enumerate(w["cams"]):
            x0, y0, x1, y1, empty = rects[v]
            if empty[gi]:
                continue
            yy, xx = np.mgrid[y0[gi]:y1[gi] + 1, x0[gi]:x1[gi] + 1]
            pix = (yy * W + xx).ravel()
            pix = pix[pv[v]["ok"][pix]]
            sub = np.nonzero(~empty & (x1 >= x0[gi]) & (x0 <= x1[gi]) & (y1 >= y0[gi]) & (y0 <= y1[gi]))[0]
            plans.append((v, c, pix, sub))

        def coord_loss(gp):
            return sum(_loss_restricted(orc, gp, c, w["tc"][v], w["td"][v], pv[v]["L"]["w"], pix, sub)
                       for v, c, pix, sub in plans)

        x0_ = g64[k].reshape(-1, N)[c_, gi]

        def coord_quotient(h):
            vals = []
            for s in (1, -1):
                g64[k].reshape(-1, N)[c_, gi] = x0_ + s * h
                vals.append(coord_loss(g64))
            g64[k].reshape(-1, N)[c_, gi] = x0_
            # with the float64 rounding of the restricted loss over the step
            return (vals[0] - vals[1]) / (2 * h), 1e-14 * abs(vals[0]) / h

        fd, noise = coord_quotient(1e-9)
        if abs(an - fd) > 1e-3 * abs(fd) + 2 * noise:
            fd2, noise2 = coord_quotient(3e-10)
            # a crossing changes the quotient with the step; a wrong gradient does not
            assert abs(fd2 - fd) > 1e-5 * abs(fd) + 2 * (noise + noise2), (gi, k, c_, an, fd, fd2)
            continue
        checked += 1
    print(f"[window fd] {checked} of 64 single coordinates checked")
    assert checked >= 48


def test_window_chain_in_one_graph(ctx, orc, window):
    """Iterations of the window, the newest keyframe's MP update (log-odds)
    with the prune flag at MP > 0.8, and the compaction, captured once and
    replayed: the state after the replay is exact (no overflow, no
    incomplete prefix), the prune flag is MP > 0.8 on the observed
    Gaussians, unobserved ones keep their MP, and the compacted map is the
    map without the flagged Gaussians, Adam moments included."""
    w = window
    g, cams = w["g"], w["cams"]
    gd = gs.to_device(g)
    mw = optim.MappingWindow(ctx, gd, cams)  # the smallest exact prefix rank, chosen again after the prune
    tcd = torch.from_numpy(np.concatenate(w["tc"], axis=1).astype(np.float32).reshape(-1)).cuda()
    tdd = torch.from_numpy(np.concatenate(w["td"]).astype(np.float32)).cuda()
    # the newest keyframe's frame: its observation and the boxes' screen
    # rectangles as the instance masks (the segmentation prior)
    ntc = tcd.view(3, V * P)[:, (V - 1) * P:].contiguous().view(-1)
    ntd = tdd[(V - 1) * P:].contiguous()
    inst = np.zeros((H, W), np.int32)
    c = cams[-1]
    Rm, t = np.asarray(c["T_cw"], np.float64)[:, :3], np.asarray(c["T_cw"], np.float64)[:, 3]
    for b, sl in enumerate(w["slices"]):
        pc = Rm @ g["mean"][:, sl].astype(np.float64) + t[:, None]
        u = c["fx"] * pc[0] / pc[2] + c["cx"]
        vv = c["fy"] * pc[1] / pc[2] + c["cy"]
        x0, x1 = int(np.clip(u.min(), 0, W - 1)), int(np.clip(u.max(), 0, W - 1))
        y0, y1 = int(np.clip(vv.min(), 0, H - 1)), int(np.clip(vv.max(), 0, H - 1))
        inst[y0:y1 + 1, x0:x1 + 1] = b + 1
    instd = torch.from_numpy(inst.reshape(-1)).cuda()
    prior = torch.tensor([0.05] + [0.9] * len(w["slices"]), device="cuda")
    conf = torch.tensor([0.1] + [0.9] * len(w["slices"]), device="cuda")

    def chain():
        for _ in range(3):
            mw.iterate(tcd, tdd)
        mw.frame_end(ntc, ntd, instd, prior, conf)

    mp0 = gd["mp"].clone()
    # warm up on a side stream (loads every kernel), restore, capture, replay
    state = {k: v.clone() for k, v in gd.items()}
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        chain()
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    for k in gd:
        gd[k].copy_(state[k])
    mw.adam.reset()
    mw.pipe.clear_flags()
    mw.mp_pipe.clear_flags()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        chain()
    for k in gd:
        gd[k].copy_(state[k])
    mw.adam.reset()
    torch.cuda.synchronize()
    graph.replay()
    torch.cuda.synchronize()
    terms = mw.objective()
    print(f"\n[window chain] L_G terms after the replay: render {terms['render'].sum():.4g}, "
          f"l3 L_MP {terms['mp']:.4g}, l4 L_edge {terms['edge'].sum():.4g}")
    assert terms["mp"] > 0 and np.all(np.isfinite(terms["edge"]))  # the means moved off the previous frame's
    mp = gd["mp"].cpu().numpy()
    observed = torch_np(mw.alpha) > 0
    prune = torch_np(mw.prune).astype(bool)
    print(f"[window chain] observed {observed.sum()}, pruned {prune.sum()}")
    assert observed.sum() > 1000 and 0 < prune.sum() < N
    np.testing.assert_array_equal(prune, mp > 0.8)
    np.testing.assert_array_equal(mp[~observed], mp0.cpu().numpy()[~observed])
    assert mp[observed].min() >= 0.01 - 1e-6 and mp[observed].max() <= 0.99 + 1e-6  # log-odds clip
    keep = torch.from_numpy(~prune).cuda()
    k_out = int(mw.n_out.item())
    assert k_out == int((~prune).sum())
    for src, dst in zip(mw.src_planes, mw.dst_planes):
        assert torch.equal(dst[:k_out], src[keep])
    rank0 = mw.rank
    n_new = mw.commit()
    assert n_new == k_out and mw.n == k_out
    print(f"[window chain] prefix rank {rank0} -> {mw.rank} after the prune")
    # the smaller map iterates on, exactly
    mw.iterate(tcd, tdd)
    mw.pipe.raise_if_failed()
