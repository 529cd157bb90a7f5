"""GPU parity at the benchmarked configuration: 1M Gaussians, one 640x480 view,
the prefix lists of the smallest exact rank, the forward with the loss fused
into it, and the backward to every Gaussian parameter and the pose, compared
element by element with the FP64 oracle (every pixel, the loss, the four
pixel-adjoint planes, all five gradient groups and the pose twist)."""

import numpy as np
import pytest
import torch

from paper_2602_21644_amd import gs, optim, synth
from tests.gpu_util import assert_grads_close, assert_image_close, grads_report, image_view, torch_np

pytestmark = pytest.mark.gpu

N, W, H, SEED = 1_000_000, 640, 480, 11
GROUPS = ("mean", "log_scale", "quat", "opacity_logit", "color")


@pytest.fixture(scope="module")
def ctx():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return gs.Context(0)


@pytest.fixture(scope="module")
def case(orc):
    """The benchmark's scene; its observed frame is the oracle's render of the
    moved boxes at the target pose (depth 0 where A < 0.5)."""
    g, cam, tcam, g_t, sl = synth.moving_box_scene(SEED, N, W, H)
    pt = orc.project(g_t, tcam)
    it = orc.render(pt, g_t, tcam)
    tc = it["C"].astype(np.float32)
    td = np.where(1.0 - it["T"] >= 0.5, it["D"], 0.0).astype(np.float32)
    pr = orc.project(g, cam)
    im = orc.render(pr, g, cam)
    L = orc.loss(im, tc, td)
    return dict(g=g, cam=cam, tc=tc, td=td, pr=pr, im=im, L=L)


@pytest.mark.parametrize("render_batch,bwd_batch", [(256, 64), (128, 32)])
def test_bench_config_parity(ctx, orc, case, render_batch, bwd_batch):
    g, cam, tc, td, pr, im, L = (case[k] for k in ("g", "cam", "tc", "td", "pr", "im", "L"))
    views = gs.ViewBatch([cam], N)
    gt = gs.to_device(g)
    gst = gs.gaussians_struct(gt)
    R, n_inst = optim.choose_rank(ctx, views, gst, N)
    assert R > 0, "the benchmark runs the prefix path"
    ctx.set_param("render_batch", render_batch)
    ctx.set_param("bwd_batch", bwd_batch)
    try:
        pipe = gs.Pipeline(ctx, views, capacity=int(n_inst * 1.25) + 4096, max_rank=R)
        tcd = torch.from_numpy(tc.reshape(-1)).cuda()
        tdd = torch.from_numpy(td).cuda()
        pipe.forward_loss(gst, tcd, tdd)
        over, n_i, inc = pipe.check()
        assert not over and inc == 0 and n_i == n_inst
        got = image_view(pipe, views, 0)
        margin = im["margin"]
        print(f"\n[bench-config] rank {R}, {n_i} list entries, margin-excluded pixels "
              f"{int((margin < 1e-5).sum())} of {margin.size}")
        assert_image_close(got, im, margin)
        loss = float(pipe.loss[0])
        assert abs(loss - L["loss"]) <= 1e-4 * abs(L["loss"]), (loss, L["loss"])

        # pixel adjoints: where the margin is small, or a residual lies within
        # the measured image error of 0 (sign(0) = 0 makes the L1 adjoint
        # discontinuous there, so either side may take either sign), both
        # sides are set to zero
        P = W * H
        rc = np.abs(im["C"] - tc) <= np.abs(got["C"] - im["C"]) + 1e-7
        rd = (td > 0) & (np.abs(im["D"] - td) <= np.abs(got["D"] - im["D"]) + 1e-7)
        amb = (margin < 1e-5) | rc.any(axis=0) | rd
        print(f"[bench-config] pixels with a zeroed adjoint: {int(amb.sum())}")
        k = ~amb
        dC = torch_np(pipe.dC).reshape(3, P)
        dD = torch_np(pipe.dD)
        assert np.abs(dC[:, k] - L["dC"][:, k]).max() <= 1e-4
        assert np.abs(dD[k] - L["dD"][k]).max() <= 1e-4
        assert np.all(torch_np(pipe.dM) == 0) and np.all(torch_np(pipe.dT) == 0)  # w detached
        keep = torch.from_numpy(k).cuda()
        pipe.dC.view(3, P).mul_(keep)
        pipe.dD.mul_(keep)
        grads = gs.alloc_grads(N)
        pose = torch.zeros(6, device="cuda")
        pipe.backward(gst, gs.grads_struct(grads, pose))
        torch.cuda.synchronize()
        g2d = orc.render_backward(pr, g, cam, L["dC"] * k, L["dD"] * k)
        rg = orc.project_backward(g, cam, g2d)
        touched = int((np.abs(rg["color"]).sum(axis=0) > 0).sum())
        report = {name: grads_report(torch_np(grads[name]), rg[name]) for name in GROUPS}
        report["pose"] = grads_report(torch_np(pose), rg["pose"])
        print(f"[bench-config] Gaussians with a gradient: {touched}; (max err / group max, n bad, worst rel): "
              + ", ".join(f"{k_}={v[0]:.2e}/{v[1]}/{v[2]:.2e}" for k_, v in report.items()))
        for name in GROUPS:
            assert_grads_close(torch_np(grads[name]), rg[name], name=name)
        assert_grads_close(torch_np(pose), rg["pose"], name="pose")
    finally:
        ctx.set_param("render_batch", 128)
        ctx.set_param("bwd_batch", 64)
