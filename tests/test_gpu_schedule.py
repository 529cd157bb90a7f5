"""GPU parity of MP sequences under the semantic-on-demand scheduler (Sec.
IV-B, Eq. (13)-(17)): the library's scheduler and gs_mp_update frame after
frame against the reference scheduler and the FP64 MP reference, for the
three scheduling policies."""

import numpy as np
import pytest
import torch

from oracle import scheduler as osch
from paper_2602_21644_amd import gs, schedule, synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return gs.Context(0)


def _gpu_sequence(ctx, frames, policy, n_fixed=10):
    W, H = frames[0]["width"], frames[0]["height"]
    n, P = frames[0]["mp"].shape[0], W * H
    views = gs.ViewBatch([synth.camera(W, H)], n)
    M = views.rec_count
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()
    sched = schedule.PriorScheduler(P, policy=policy, n_fixed=n_fixed)
    mp = t(frames[0]["mp"].astype(np.float32))
    Ut, al = torch.zeros(n, device="cuda"), torch.zeros(n, device="cuda")
    dyn, pr = torch.zeros(n, dtype=torch.uint8, device="cuda"), torch.zeros(n, dtype=torch.uint8, device="cuda")
    stats = torch.zeros(8, device="cuda")
    out = gs.MPOut(gs.ptr(Ut), gs.ptr(al), gs.ptr(dyn), gs.ptr(pr), None, None, gs.ptr(stats))
    ws = torch.zeros(gs.gs_workspace_size(ctx, views.s, gs.GS_OP_MP_UPDATE), dtype=torch.uint8, device="cuda")
    pp = gs.MPParams(*[gs.MP_DEFAULTS[k] for k in gs.MP_PARAM_NAMES], 0, 0)
    res = []
    for fr in frames:
        mean2d = np.zeros((2, M), np.float32)
        mean2d[:, :n] = fr["mean2d"]
        key = np.full(M, 0xFFFFFFFF, np.uint32)
        key[:n] = np.where(fr["culled"], 0xFFFFFFFF, np.float32(1.0).view(np.uint32))
        m2d, keyd = t(mean2d.reshape(-1)), t(key.view(np.int32))
        proj = gs.Proj()
        proj.m = M
        proj.mean2d, proj.depth_key = gs.ptr(m2d), gs.ptr(keyd)
        Dd, Cd = t(fr["depth"]), t(fr["color"].reshape(-1))
        img = gs.Image(gs.ptr(Cd), gs.ptr(Dd), None, None, None)
        Dg, Cg = t(fr["target_depth"]), t(fr["target_color"].reshape(-1))
        tgt = gs.Target(gs.ptr(Cg), gs.ptr(Dg))
        go = sched.decide(fr["dbar"], fr["epi_state"])
        masks = sched.prior(t(fr["instance_id"]))
        prior, conf = t(fr["inst_prior"]), t(fr["inst_conf"])
        frame = gs.MPFrame(gs.ptr(masks), len(fr["inst_prior"]) - 1, gs.ptr(prior), gs.ptr(conf), int(go), None)
        gs.gs_mp_update(ctx, views.s, proj, img, tgt, frame, pp, mp, out, ws)
        torch.cuda.synchronize()
        sched.observe(stats)
        res.append(dict(refresh=go, S=sched.state.S, mp=mp.cpu().numpy(), dynamic=dyn.cpu().numpy().astype(bool),
                        U_bar=float(stats[0]), tau=float(stats[1])))
    return res, sched


@pytest.mark.parametrize("policy", ["on_demand", "always", "fixed"])
def test_mp_sequence_parity(ctx, orc, policy):
    frames = synth.mp_sequence_inputs(21, 6000, 96, 72, 16)
    got, sched = _gpu_sequence(ctx, frames, policy, n_fixed=10)
    ref = osch.run_mp_sequence(frames, policy=policy, n_fixed=10)
    flips = 0
    for k, (g, r) in enumerate(zip(got, ref)):
        rr = r["result"]
        assert g["refresh"] == r["refresh"], (k, g["S"], r["S"])
        if policy == "on_demand":
            assert abs(g["S"] - r["S"]) < 1e-5
        np.testing.assert_allclose(g["mp"], rr["mp"], atol=2e-5)
        np.testing.assert_allclose(g["U_bar"], rr["stats"]["U_bar"], atol=2e-5)
        far = np.abs(rr["mp"] - rr["stats"]["tau"]) > 1e-4
        np.testing.assert_array_equal(g["dynamic"][far], rr["dynamic"][far])
        if k:
            flips += int((got[k]["dynamic"] != got[k - 1]["dynamic"]).sum())
    n_ref = sum(r["refresh"] for r in ref)
    print(f"\n[schedule] {policy}: {n_ref} refreshes over {len(frames)} frames, {flips} label flips")
    assert sched.refreshes == n_ref
    if policy == "always":
        assert n_ref == len(frames)
    if policy == "fixed":
        assert n_ref == 2
    if policy == "on_demand":
        # the bursts of large epipolar distances trigger refreshes the fixed
        # interval would not make
        assert 2 < n_ref < len(frames)
