"""GPU parity of the learned MP surrogate kernels (features, bfloat16 sync,
inference, training step) against the FP64 oracle, through the C ABI."""

import numpy as np
import pytest
import torch

from paper_2602_21644_amd import gs, synth

pytestmark = pytest.mark.gpu

NAMES = ("W1", "b1", "W2", "b2", "W3", "b3")


@pytest.fixture(scope="module")
def ctx():
    assert torch.cuda.is_available()
    return gs.Context(0)


def pack(params):
    return np.concatenate([np.asarray(params[k], np.float32).reshape(-1) for k in NAMES])


def unpack(v):
    out, o = {}, 0
    for k, shp in (("W1", (32, 8)), ("b1", (32,)), ("W2", (32, 32)), ("b2", (32,)), ("W3", (1, 32)), ("b3", (1,))):
        s = int(np.prod(shp))
        out[k] = np.asarray(v[o:o + s], np.float64).reshape(shp)
        o += s
    return out


def make_mlp(params):
    master = torch.from_numpy(pack(params)).cuda()
    wq = torch.zeros(gs.GS_MLP_WEIGHTS, dtype=torch.int16, device="cuda")
    m = torch.zeros(gs.GS_MLP_PARAMS, device="cuda")
    v = torch.zeros(gs.GS_MLP_PARAMS, device="cuda")
    s = gs.MLP(gs.ptr(master), gs.ptr(wq), gs.ptr(m), gs.ptr(v))
    return s, (master, wq, m, v)


def test_sync_bf16_bitexact(ctx, orc):
    x, lab, params = synth.mlp_inputs(0, 10)
    s, (master, wq, m, v) = make_mlp(params)
    gs.gs_mlp_sync(ctx, s)
    got = wq.cpu().numpy().view(np.uint16)
    ref = np.concatenate([orc.mlp.bf16_round(params[k]).reshape(-1) for k in ("W1", "W2", "W3")])
    np.testing.assert_array_equal(got, (ref.view(np.uint32) >> 16).astype(np.uint16))


@pytest.mark.parametrize("P", [1, 1000, 307200])
def test_forward_parity(ctx, orc, P):
    x, lab, params = synth.mlp_inputs(1, P)
    s, keep = make_mlp(params)
    gs.gs_mlp_sync(ctx, s)
    xd = torch.from_numpy(x.reshape(-1)).cuda()
    y = torch.zeros(P, device="cuda")
    gs.gs_mlp_fwd(ctx, s, xd, y, P)
    ref, _ = orc.mlp.forward(params, x)
    np.testing.assert_allclose(y.cpu().numpy(), ref, atol=1e-4)


@pytest.mark.parametrize("P", [300, 65537])
def test_train_step_parity(ctx, orc, P):
    x, lab, params = synth.mlp_inputs(2, P)
    s, (master, wq, m, v) = make_mlp(params)
    gs.gs_mlp_sync(ctx, s)
    xd = torch.from_numpy(x.reshape(-1)).cuda()
    ld = torch.from_numpy(lab).cuda()
    loss = torch.zeros(1, device="cuda")
    grad = torch.zeros(gs.GS_MLP_PARAMS, device="cuda")
    ws = torch.empty(gs.gs_workspace_size(ctx, _views(P), gs.GS_OP_MLP_TRAIN), dtype=torch.uint8, device="cuda")
    lr = 1e-3
    gs.gs_mlp_train_step(ctx, s, xd, ld, P, lr, 1, loss, grad, ws)
    torch.cuda.synchronize()
    L, g, _ = orc.mlp.loss_and_grads(params, x, lab)
    np.testing.assert_allclose(float(loss[0]), L, rtol=1e-5)
    gg = unpack(grad.cpu().numpy())
    for k in NAMES:
        sc = np.abs(g[k]).max()
        assert np.abs(gg[k] - g[k]).max() <= 1e-3 * sc + 1e-9, k
    # one Adam step: the oracle's update from the oracle gradient
    zeros = {k: np.zeros_like(np.asarray(params[k], np.float64)) for k in NAMES}
    newp, _, _ = orc.mlp.adam_step({k: np.asarray(params[k], np.float64) for k in NAMES}, g, zeros, zeros, 1, lr)
    got = unpack(master.cpu().numpy())
    for k in NAMES:
        big = np.abs(g[k]) > 1e-3 * np.abs(g[k]).max()
        np.testing.assert_allclose(got[k][big], newp[k][big], atol=2e-6 + 1e-6)


def _views(P):
    cam = synth.camera(256, (P + 255) // 256)
    return gs.ViewBatch([cam], 1).s


def test_features_parity(ctx, orc):
    inp = synth.mp_frame_inputs(4, 100, 64, 48)
    P = 64 * 48
    rng = np.random.default_rng(1)
    Mimg = rng.random(P).astype(np.float32)
    Timg = rng.random(P).astype(np.float32)
    views = gs.ViewBatch([synth.camera(64, 48)], 1)
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()
    C, D, Mt, Tt = t(inp["color"].reshape(-1)), t(inp["depth"]), t(Mimg), t(Timg)
    img = gs.Image(gs.ptr(C), gs.ptr(D), gs.ptr(Mt), gs.ptr(Tt), None)
    Cg, Dg = t(inp["target_color"].reshape(-1)), t(inp["target_depth"])
    tgt = gs.Target(gs.ptr(Cg), gs.ptr(Dg))
    inst, prior, conf = t(inp["instance_id"]), t(inp["inst_prior"]), t(inp["inst_conf"])
    fr = gs.MPFrame(gs.ptr(inst), 3, gs.ptr(prior), gs.ptr(conf), 1, None)
    x = torch.zeros(8 * P, device="cuda")
    gs.gs_mlp_features(ctx, views.s, img, tgt, fr, x)
    mp_ins = inp["inst_prior"][inp["instance_id"]]
    ref = orc.mlp.features(inp["color"], inp["depth"], Mimg, Timg, inp["target_color"], inp["target_depth"], mp_ins)
    np.testing.assert_allclose(x.cpu().numpy().reshape(8, P), ref, atol=1e-5)
