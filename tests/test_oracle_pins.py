"""More pins of the FP64 oracle (CPU only), each against something other than
the oracle's own formula:

* the adjoint of the loss with the static weight differentiated (both weight
  modes) and the adjoints of the rendered MP channel and final transmittance,
  against central finite differences of the forward;
* the log-odds state update against Bayes' rule for two independent
  probabilities (rate 1) and against the power law of the odds (prior 1/2),
  with its clip;
* the fixed normalisation of the uncertainty (u_norm = 1) against its
  maximum (binary entropy ln 2 plus lambda_u times the largest variance of
  values in [0, 1], 1/4) and against the binary entropy in bits;
* thresholds, labels, the frame uncertainty and the prune flag on hand-worked
  frames (lower median of an even count, the 0.5 floor of tau, strict ">");
* the photometric share of the residual cue against an equivalent depth
  residual;
* the surrogate's input features on a hand-worked pixel.
"""

import math

import numpy as np
import pytest
from scipy.stats import entropy

from paper_2602_21644_amd import synth


# ---------------------------------------------------------------- adjoints
def _scene(orc, seed=1, n=800):
    g, cam, tcam = synth.tiny_scene(seed=seed, n=n)
    pr_t = orc.project(g, tcam)
    tgt = orc.render(pr_t, g, tcam)
    td = tgt["D"].copy()
    td[(1 - tgt["T"]) < 0.5] = 0.0
    return {k: np.asarray(v, np.float64) for k, v in g.items()}, cam, tgt["C"], td


def _fd_check(orc, g64, grads, f, rng, n_per_group=6, min_checked=12, groups=None):
    """Central differences of the scalar f(gaussians) against `grads` on
    coordinates with large gradients; a coordinate counts only when two step
    sizes agree (no threshold crossed between them)."""
    checked = 0
    for name in groups or ("mean", "log_scale", "quat", "opacity_logit", "color"):
        G = grads[name] if grads[name].ndim > 1 else grads[name][None]
        flat = np.abs(G).ravel()
        cand = np.argsort(flat)[::-1][:40]
        cand = rng.choice(cand, size=n_per_group, replace=False)
        for idx in cand:
            row, k = np.unravel_index(idx, G.shape)
            ests = []
            for h in (1e-5, 1e-6):
                vals = []
                for sgn in (1, -1):
                    gp = {kk: v.copy() for kk, v in g64.items()}
                    arr = gp[name] if gp[name].ndim > 1 else gp[name][None]
                    scale = max(1.0, abs(arr[row, k]))
                    arr[row, k] += sgn * h * scale
                    vals.append(f(gp))
                ests.append((vals[0] - vals[1]) / (2 * h * scale))
            if abs(ests[0] - ests[1]) > 1e-6 * max(abs(ests[0]), 1e-9) + 1e-9:
                continue
            an = G[row, k]
            assert abs(an - ests[1]) <= 1e-5 * abs(ests[1]) + 1e-7, (name, row, k, an, ests)
            checked += 1
    assert checked >= min_checked, checked


@pytest.mark.parametrize("weight_mode", [0, 1])
def test_gradient_through_weight_finite_differences(orc, weight_mode):
    """With the static weight w differentiated (w = 1 - M/A, or A - M), the
    adjoint of the loss, chained through the MP channel M and the
    transmittance T of the render, equals central differences of the loss
    recomputed with w recomputed at every step."""
    g64, cam, tc, td = _scene(orc, seed=3)
    kw = dict(weight_mode=weight_mode, grad_through_weight=True)
    L, im, grads, pr, _ = orc.full_backward(g64, cam, tc, td, **kw)
    assert np.abs(L["dM"]).max() > 0 and np.abs(L["dT"]).max() > 0

    def f(gp):
        return orc.forward_loss(gp, cam, tc, td, **kw)

    _fd_check(orc, g64, grads, f, np.random.default_rng(weight_mode))
    # the weight's share of the gradient is not negligible here: detaching it
    # changes the gradients
    Ld, _, gd, _, _ = orc.full_backward(g64, cam, tc, td, weight_mode=weight_mode)
    assert np.abs(gd["opacity_logit"] - grads["opacity_logit"]).max() > 1e-3 * np.abs(grads["opacity_logit"]).max()


def test_mp_channel_and_transmittance_adjoints(orc):
    """For a linear upstream L = sum_u a(u) M(u) + b(u) T(u) (+ a background
    colour term), the render adjoint fed with gM = a, gT = b matches central
    differences of L."""
    g64, cam, tc, td = _scene(orc, seed=5, n=600)
    P = 64 * 48
    rng = np.random.default_rng(7)
    a, b = rng.normal(size=P), rng.normal(size=P)
    gC = rng.normal(size=(3, P))
    bg = (0.3, 0.1, 0.6)
    pr = orc.project(g64, cam)
    g2d = orc.render_backward(pr, g64, cam, gC, np.zeros(P), a, b, bg=bg)
    grads = orc.project_backward(g64, cam, g2d)

    def f(gp):
        im = orc.render(orc.project(gp, cam), gp, cam, bg=bg)
        return float((a * im["M"]).sum() + (b * im["T"]).sum() + (gC * im["C"]).sum())

    _fd_check(orc, g64, grads, f, rng, groups=("mean", "log_scale", "quat", "opacity_logit"))
    # gM alone (no colour, no T): the colour adjoint is zero, the opacity one is not
    g2d = orc.render_backward(pr, g64, cam, np.zeros((3, P)), np.zeros(P), a, None)
    assert np.all(g2d[6:9] == 0) and np.abs(g2d[5]).max() > 0


# ---------------------------------------------------------------- MP update, hand-built frames
def _blocks_frame(values, prev, width_per=5, height=5):
    """A frame of len(values) side-by-side blocks of width_per x height pixels,
    every pixel observed, one Gaussian at each block centre (windows of
    radius 2 stay inside their block), surrogate M_p = values[block]."""
    nb = len(values)
    W, H = nb * width_per, height
    P = W * H
    xx = np.tile(np.arange(W), H)
    mp_px = np.asarray(values, np.float64)[xx // width_per]
    cx = np.arange(nb) * width_per + width_per // 2
    inp = dict(width=W, height=H, depth=np.full(P, 1.0, np.float32), target_depth=np.full(P, 1.0, np.float32),
               color=np.zeros((3, P), np.float32), target_color=np.zeros((3, P), np.float32),
               instance_id=np.zeros(P, np.int32), inst_prior=np.array([0.05], np.float32),
               inst_conf=np.array([0.1], np.float32),
               mean2d=np.stack([cx, np.full(nb, height // 2)]).astype(np.float32),
               culled=np.zeros(nb, bool), mp=np.asarray(prev, np.float32))
    return inp, mp_px


def _H(p, eps):
    return -p * math.log(p + eps) - (1 - p) * math.log(1 - p + eps)


def test_labels_tau_floor_even_median_and_ubar(orc):
    """Rate 1 (M^t = window mean of a constant M_p): M^t = (0.2, 0.3, 0.45,
    0.9). The lower median of the even count is 0.3, so tau = max(0.3, 0.5)
    = 0.5 and only 0.9 is dynamic. U = binary entropy of the previous state
    (zero window variance): previous states (0.5, 0.1, 0.2, 0.3) normalise to
    (1, 0, u2, u3) and the frame uncertainty is the lower median u2. The prune
    flag at 0.8 marks the 0.9 one."""
    vals, prev = [0.2, 0.3, 0.45, 0.9], [0.5, 0.1, 0.2, 0.3]
    inp, mp_px = _blocks_frame(vals, prev)
    prm = dict(alpha_min=1.0, alpha_max=1.0, prune_above=0.8)
    r = orc.mp.mp_update(inp, prm, mlp_mp=mp_px)
    assert r["observed"].all()
    np.testing.assert_allclose(r["mp"], vals, atol=1e-15)
    assert r["stats"]["tau"] == 0.5
    assert r["stats"]["median"] == pytest.approx(0.3, abs=1e-15)
    assert r["dynamic"].tolist() == [False, False, False, True]
    assert r["prune"].tolist() == [False, False, False, True]
    eps = orc.mp.DEFAULTS["eps"]
    Hs = [_H(float(np.float32(p)), eps) for p in prev]
    u2 = (Hs[2] - Hs[1]) / (Hs[0] - Hs[1])
    assert r["stats"]["U_bar"] == pytest.approx(u2, rel=1e-12)
    np.testing.assert_allclose(r["U_tilde"], [1.0, 0.0, u2, (Hs[3] - Hs[1]) / (Hs[0] - Hs[1])], rtol=1e-12, atol=1e-15)
    # the prune flag has its own threshold, independent of tau
    r = orc.mp.mp_update(inp, dict(prm, prune_above=0.4), mlp_mp=mp_px)
    assert r["prune"].tolist() == [False, False, True, True]
    assert r["dynamic"].tolist() == [False, False, False, True]
    assert r["stats"]["n_prune"] == 2


def test_labels_strict_threshold_and_odd_median(orc):
    """M^t = (0.6, 0.7, 0.8, 0.9): lower median 0.7 is tau itself, and the
    Gaussian at tau is not dynamic (strict '>'); with a fifth one at 0.65 the
    median of the odd count is 0.7 as well."""
    for vals in ([0.6, 0.7, 0.8, 0.9], [0.6, 0.7, 0.8, 0.9, 0.65]):
        inp, mp_px = _blocks_frame(vals, [0.5] * len(vals))
        r = orc.mp.mp_update(inp, dict(alpha_min=1.0, alpha_max=1.0), mlp_mp=mp_px)
        assert r["stats"]["tau"] == pytest.approx(0.7, abs=1e-15)
        assert r["dynamic"].tolist() == [v > 0.7 for v in vals]
        assert r["stats"]["n_dyn"] == 2


def test_logodds_rate_one_is_bayes_rule(orc):
    """Log-odds mode at rate 1: the new state is the posterior of two
    independent probabilities p (previous state) and q (window estimate),
    p q / (p q + (1 - p)(1 - q)), clipped to [0.01, 0.99] in probability."""
    ps = [0.5, 0.2, 0.7, 0.9, 0.95, 0.05]
    qs = [0.8, 0.6, 0.3, 0.9, 0.95, 0.4]
    inp, mp_px = _blocks_frame(qs, ps)
    r = orc.mp.mp_update(inp, dict(alpha_min=1.0, alpha_max=1.0, mode=1), mlp_mp=mp_px)
    p = np.asarray(ps, np.float32).astype(np.float64)
    q = np.asarray(qs, np.float64)
    bayes = p * q / (p * q + (1 - p) * (1 - q))
    np.testing.assert_allclose(r["mp"], np.clip(bayes, 0.01, 0.99), rtol=1e-12)
    assert r["mp"][4] == pytest.approx(0.99, abs=1e-14)  # 0.95 twice: clipped


def test_logodds_half_prior_power_law(orc):
    """Log-odds mode from the uninformative state 1/2 with rate a: the odds of
    the new state are the a-th power of the odds of the window estimate
    (a = rho alpha = 0.5 without a prior refresh)."""
    qs = [0.8, 0.3, 0.6, 0.97]
    inp, mp_px = _blocks_frame(qs, [0.5] * 4)
    r = orc.mp.mp_update(inp, dict(alpha_min=1.0, alpha_max=1.0, mode=1), seg_updated=False, mlp_mp=mp_px)
    q = np.clip(np.asarray(qs, np.float64), 0.01, 0.99)
    odds = (q / (1 - q)) ** 0.5
    np.testing.assert_allclose(r["mp"], odds / (1 + odds), rtol=1e-12)


def _popoviciu_frame():
    """5x5 frame, one Gaussian at the centre pixel; of its radius-2 window
    (13 pixels) the centre is unobserved and the 12 others carry residuals 0
    (six) and e1 (six); every pixel outside the window is unobserved."""
    W = H = 5
    P = W * H
    yy, xx = np.mgrid[0:H, 0:W]
    d2 = (xx - 2) ** 2 + (yy - 2) ** 2
    win = (d2 <= 4) & (d2 > 0)
    idx = np.nonzero(win.ravel())[0]
    assert idx.size == 12
    depth = np.full(P, 1.0)
    tdepth = np.zeros(P)
    tdepth[idx[:6]] = 1.0
    tdepth[idx[6:]] = 1.1
    return dict(width=W, height=H, depth=depth, target_depth=tdepth, color=np.zeros((3, P)),
                target_color=np.zeros((3, P)), instance_id=np.zeros(P, np.int32), inst_prior=np.array([0.05]),
                inst_conf=np.array([0.0]), mean2d=np.array([[2.0], [2.0]], np.float32), culled=np.zeros(1, bool),
                mp=np.array([0.5], np.float32))


def test_fixed_uncertainty_bound_is_reached(orc):
    """u_norm = 1 divides U = H(M) + lambda_u Var by its largest value: the
    binary entropy peaks at ln 2 (M = 1/2) and values in [0, 1] have variance
    at most 1/4 (half of them 0, half 1). With lambda_e = 0 the window's M_p
    is exactly half 0, half 1, and the normalised uncertainty is 1; with
    min-max normalisation a lone Gaussian gets 0."""
    inp = _popoviciu_frame()
    prm = dict(lambda_e=0.0, eps=1e-15, lambda_u=1.0)
    r = orc.mp.mp_update(inp, dict(prm, u_norm=1))
    assert r["nobs"][0] == 12
    assert r["var"][0] == pytest.approx(0.25, abs=1e-15)
    assert r["U_tilde"][0] == pytest.approx(1.0, abs=1e-12)
    r0 = orc.mp.mp_update(inp, dict(prm, u_norm=0))
    assert r0["U_tilde"][0] == 0.0
    # a smaller variance weight lowers the bound and the value alike
    r = orc.mp.mp_update(inp, dict(prm, u_norm=1, lambda_u=3.0))
    assert r["U_tilde"][0] == pytest.approx(1.0, abs=1e-12)


def test_fixed_uncertainty_is_entropy_in_bits(orc):
    """u_norm = 1 with lambda_u = 0 is the binary entropy of the previous
    state in bits."""
    prev = [0.5, 0.1, 0.25, 0.9, 0.7]
    inp, mp_px = _blocks_frame([0.3] * 5, prev)
    r = orc.mp.mp_update(inp, dict(u_norm=1, lambda_u=0.0, eps=1e-15), mlp_mp=mp_px)
    ref = [entropy([p, 1 - p], base=2) for p in np.asarray(prev, np.float32).astype(np.float64)]
    np.testing.assert_allclose(r["U_tilde"], ref, rtol=1e-12)


def test_photometric_residual_share(orc):
    """e = |D - D_obs| + beta |C - C_obs|_1: a frame whose only residual is a
    colour one, with beta, gives the same update as the frame whose only
    residual is a depth one of beta times the colour residual."""
    base = synth.mp_frame_inputs(21, 300, 32, 24, n_inst=2)
    P = 32 * 24
    rng = np.random.default_rng(3)
    D = base["depth"].astype(np.float64)
    valid = base["target_depth"] > 0
    C = rng.random((3, P))
    dC = rng.normal(0, 0.05, size=(3, P))
    for beta in (1.0, 2.5):
        a = dict(base, depth=D, target_depth=np.where(valid, D, 0.0), color=C, target_color=C + dC)
        r_col = np.abs(dC).sum(axis=0)
        b = dict(base, depth=D, target_depth=np.where(valid, D + beta * r_col, 0.0), color=C, target_color=C)
        ra = orc.mp.mp_update(a, dict(beta_color=beta))
        rb = orc.mp.mp_update(b, dict(beta_color=beta))
        np.testing.assert_allclose(ra["e"][valid], rb["e"][valid], rtol=1e-9)
        for k in ("M_p", "mp", "U_tilde", "alpha"):
            np.testing.assert_allclose(ra[k], rb[k], rtol=1e-7, atol=1e-9)
        assert np.array_equal(ra["dynamic"], rb["dynamic"])
        # without the colour share the colour-only frame has no residual at all
        rz = orc.mp.mp_update(a, dict(beta_color=0.0))
        assert np.abs(rz["e"][valid]).max() == 0.0


def test_mlp_features_hand_worked(orc):
    """One observed pixel and one unobserved pixel: colour residual as is,
    depth residual per 0.1 m (0 where unobserved), depth per 4 m."""
    C = np.array([[0.5, 0.5], [0.2, 0.2], [0.1, 0.1]])
    Cg = np.array([[0.4, 0.4], [0.4, 0.4], [0.1, 0.1]])
    x = orc.mlp.features(C, [2.0, 3.0], [0.3, 0.1], [0.25, 0.5], Cg, [1.95, 0.0], [0.9, 0.05])
    np.testing.assert_allclose(x[:, 0], [0.1, -0.2, 0.0, 0.5, 0.3, 0.25, 0.5, 0.9], atol=1e-12)
    np.testing.assert_allclose(x[:, 1], [0.1, -0.2, 0.0, 0.0, 0.1, 0.5, 0.75, 0.05], atol=1e-12)


# ---------------------------------------------------------------- depth-order precision
def _order_effect(orc, g, cam):
    pr = orc.project(g, cam)
    a = orc.render(pr, g, cam)
    b = orc.render(pr, g, cam, order="f64")
    diff = np.maximum.reduce([np.abs(a["C"] - b["C"]).max(0), np.abs(a["D"] - b["D"]), np.abs(a["M"] - b["M"]),
                              np.abs(a["T"] - b["T"])])
    return diff, a["margin"], b["margin"]


@pytest.mark.parametrize("seed", [1, 2, 3])
def test_depth_order_precision_tiny(orc, seed):
    """The order of the composited Gaussians is decided on their float32
    camera depth (the precision the GPU decides it in). Ordering by the
    float64 depth instead changes no pixel of the tiny scenes at either
    pose."""
    g, cam, tcam = synth.tiny_scene(seed=seed)
    for c in (cam, tcam):
        diff, m32, m64 = _order_effect(orc, g, c)
        assert diff.max() == 0.0


def test_depth_order_precision_full_size(orc):
    """The same at 1M Gaussians over the whole 640x480 image at the rotated
    pose: no pixel changes. The survey's depth-gap exclusion term (relative
    gap below 1e-5 between consecutive contributors) would have excluded
    about a third of these pixels, mostly exact ties (Gaussians on box faces
    level with the image plane), which both precisions order by id; the
    thresholds of the compositing exclude under 0.1%."""
    g, cam, tcam, g_t, sl = synth.moving_box_scene(7, 1_000_000, 640, 480)
    diff, m32, m64 = _order_effect(orc, g, tcam)
    assert diff.max() == 0.0
    assert (m32 < 1e-5).mean() <= 1e-3
    assert (m64 < 1e-5).mean() > 0.2
