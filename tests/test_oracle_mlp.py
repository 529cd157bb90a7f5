"""Pins of the FP64 MLP-surrogate oracle (CPU only): zero weights, a closed
form, finite differences, bfloat16 rounding against torch's conversion and the
Adam step against torch.optim.Adam."""

import numpy as np
import torch

from paper_2602_21644_amd import synth


def test_zero_weights_half(orc):
    x, lab, params = synth.mlp_inputs(0, 50)
    z = {k: np.zeros_like(v) for k, v in params.items()}
    y, _ = orc.mlp.forward(z, x)
    np.testing.assert_allclose(y, 0.5)


def test_single_path_closed_form(orc):
    """Only W1[0,0], W2[0,0], W3[0,0] nonzero (bfloat16-exact values):
    y = sigmoid(c * relu(b * relu(a x0)))."""
    x, lab, params = synth.mlp_inputs(1, 64)
    z = {k: np.zeros_like(v) for k, v in params.items()}
    z["W1"][0, 0], z["W2"][0, 0], z["W3"][0, 0] = 1.5, -0.75, 2.0
    y, _ = orc.mlp.forward(z, x)
    ref = 1 / (1 + np.exp(-2.0 * np.maximum(-0.75 * np.maximum(1.5 * x[0].astype(float), 0), 0)))
    np.testing.assert_allclose(y, ref, rtol=1e-14)


def test_bf16_round_matches_torch(orc):
    v = np.random.default_rng(3).normal(size=4096).astype(np.float32) * 10
    v[:4] = [1.00390625, 1.01171875, -2.0078125, 3.0]  # exact ties
    ref = torch.from_numpy(v).to(torch.bfloat16).to(torch.float32).numpy()
    np.testing.assert_array_equal(orc.mlp.bf16_round(v), ref)


def test_gradients_fd(orc):
    x, lab, params = synth.mlp_inputs(2, 40)
    L, g, _ = orc.mlp.loss_and_grads(params, x, lab)
    w = orc.mlp.used_weights(params)
    rng = np.random.default_rng(0)
    for name in orc.mlp.PARAM_NAMES:
        for _ in range(4):
            idx = tuple(rng.integers(0, s) for s in w[name].shape)
            h = 1e-6
            vals = []
            for sgn in (1, -1):
                ww = {k: v.copy() for k, v in w.items()}
                ww[name][idx] += sgn * h
                # evaluate with the float64 values directly (no re-rounding)
                z1 = ww["W1"] @ x + ww["b1"][:, None]
                h1 = np.maximum(z1, 0)
                z2 = ww["W2"] @ h1 + ww["b2"][:, None]
                h2 = np.maximum(z2, 0)
                y = 1 / (1 + np.exp(-(ww["W3"] @ h2 + ww["b3"][:, None])[0]))
                vals.append(orc.mlp.bce(y, lab))
            fd = (vals[0] - vals[1]) / (2 * h)
            assert abs(fd - g[name][idx]) <= 1e-6 * max(1.0, abs(fd)), (name, idx, fd, g[name][idx])


def test_adam_matches_torch(orc):
    rng = np.random.default_rng(5)
    p = {"W1": rng.normal(size=(4, 3))}
    m = {"W1": np.zeros((4, 3))}
    v = {"W1": np.zeros((4, 3))}
    tp = torch.tensor(p["W1"], dtype=torch.float64, requires_grad=True)
    opt = torch.optim.Adam([tp], lr=1e-2)
    for step in range(1, 4):
        gr = {"W1": rng.normal(size=(4, 3))}
        tp.grad = torch.tensor(gr["W1"])
        opt.step()
        names = ("W1",)
        b1c, b2c = 1 - 0.9 ** step, 1 - 0.999 ** step
        mk = 0.9 * m["W1"] + 0.1 * gr["W1"]
        vk = 0.999 * v["W1"] + 0.001 * gr["W1"] ** 2
        full_p, full_m, full_v = orc.mlp.adam_step(
            {k: (p[k] if k in names else np.zeros(1)) for k in orc.mlp.PARAM_NAMES},
            {k: (gr[k] if k in names else np.zeros(1)) for k in orc.mlp.PARAM_NAMES},
            {k: (m[k] if k in names else np.zeros(1)) for k in orc.mlp.PARAM_NAMES},
            {k: (v[k] if k in names else np.zeros(1)) for k in orc.mlp.PARAM_NAMES}, step, 1e-2)
        p["W1"], m["W1"], v["W1"] = full_p["W1"], full_m["W1"], full_v["W1"]
        np.testing.assert_allclose(p["W1"], tp.detach().numpy(), rtol=1e-12, atol=1e-14)
        np.testing.assert_allclose(m["W1"], mk, rtol=1e-12)
