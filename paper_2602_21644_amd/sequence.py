"""A sequence of frames through tracking, epipolar verification, the
semantic-on-demand scheduler and the temporal MP update: the synthetic
analogue of the ablations on temporal MP (instant / fixed / adaptive rate),
MP fusion (MP_ins only K = 0, MP_geo only K = 1, fusion) and scheduling
(always / fixed interval / on demand).

Per frame t >= 1 of a moving-box sequence (the map is the scene at frame 0;
the observed frames have the boxes moved):
  1. the observed colour and depth are rendered from the true scene at the
     true pose (depth 0 where the accumulated opacity is below 0.5);
  2. tracking: pose-only optimisation of the MP-weighted loss from the
     previous estimate (optim.Tracker, full lists);
  3. epipolar verification (gs_epipolar_verify) with synthetic matches
     between frames t - 1 and t (true geometry, pixel noise, outliers) under
     the estimated poses, of k_cand candidates: half drawn from the Gaussians
     the last update labelled dynamic (the ambiguous ones the verification is
     meant for), half from all; suppressed candidates whose median distance
     is below 1 px are restored as static (MP 0), unless the variant turns
     the recovery off;
  4. the scheduler decides from the last U_bar and the verification whether
     the instance prior (a synthetic detector's box masks at frame t) is
     refreshed; otherwise the last masks are reused with alpha' = rho alpha;
  5. gs_mp_update at the estimated pose updates MP in place; its labels and
     frame statistics feed the metrics and the next decision.
Metrics: prior refreshes, label flip ratio between consecutive frames over
the Gaussians observed in both, mean |MP - truth| and label error over the
Gaussians observed in the last frame, camera-centre RMSE and mean rotation
error of the tracked poses, and milliseconds per frame.
"""

from __future__ import annotations

import time

import numpy as np
import torch

from . import gs, optim, schedule, synth

VARIANTS = {
    # Ablation I: temporal MP (with fusion and the on-demand scheduler)
    "instant": dict(mp=dict(alpha_min=1.0, alpha_max=1.0)),
    "fixed_rate": dict(mp=dict(alpha_min=0.45, alpha_max=0.45)),
    "adaptive": dict(),
    # Ablation II: MP fusion
    "ins_only": dict(mp=dict(sigma_g=1e-30)),
    "geo_only": dict(conf_zero=True),
    # Ablation III: scheduling (adaptive rate, fusion)
    "always": dict(policy="always"),
    "fixed_interval": dict(policy="fixed"),
    # without the epipolar static recovery
    "no_recovery": dict(recover=False),
}
PRIOR = (0.05, 0.9)  # mu(background), mu(box)
CONF = (0.1, 0.9)


def _observe(ctx, cam, g_dev, n):
    views = gs.ViewBatch([cam], n)
    gst = gs.gaussians_struct(g_dev)
    pipe = gs.Pipeline(ctx, views, capacity=max(1 << 20, 48 * n))
    pipe.forward(gst)
    over, _, _ = pipe.check()
    if over:
        raise gs.GSError(gs.GS_E_CAPACITY, "observation render overflowed")
    A = 1.0 - pipe.img_T
    return pipe.img_color.clone(), torch.where(A >= 0.5, pipe.img_depth, torch.zeros_like(A)).contiguous()


def _pose_errors(T, T_ref):
    dR = T[:, :3] @ T_ref[:, :3].T
    ang = np.degrees(np.arccos(np.clip((np.trace(dR) - 1) / 2, -1, 1)))
    c = -T[:, :3].T @ T[:, 3]
    c_ref = -T_ref[:, :3].T @ T_ref[:, 3]
    return float(ang), float(np.linalg.norm(c - c_ref))


def run(ctx, seq, variant="adaptive", track_iters=20, k_cand=2000, per=(4, 16), noise_px=0.3, outlier_frac=0.1,
        n_fixed=10, seed=0):
    """One pass over `seq` (synth.box_sequence) with the variant's settings;
    returns the metrics (see the module docstring)."""
    cfg = VARIANTS[variant]
    policy = cfg.get("policy", "on_demand")
    g0 = seq["map"]
    cams, obs, slices, truth = seq["cams"], seq["obs"], seq["slices"], seq["dynamic"]
    n = synth.n_gaussians(g0)
    W, H = cams[0]["width"], cams[0]["height"]
    P = W * H
    rng = np.random.default_rng(seed)
    gd = gs.to_device(g0)
    gd["mp"].fill_(0.5)
    gst = gs.gaussians_struct(gd)
    # MP update inputs at the estimated pose
    views = gs.ViewBatch([cams[0]], n)
    pipe = gs.Pipeline(ctx, views, capacity=max(1 << 20, 48 * n), full_proj=True)
    mpp = dict(gs.MP_DEFAULTS)
    mpp.update(cfg.get("mp", {}))
    params = gs.MPParams(*[mpp[k] for k in gs.MP_PARAM_NAMES], 0, 0)
    K = len(slices)
    prior = torch.tensor([PRIOR[0]] + [PRIOR[1]] * K, dtype=torch.float32, device="cuda")
    conf = torch.tensor([CONF[0]] + [CONF[1]] * K, dtype=torch.float32, device="cuda")
    if cfg.get("conf_zero"):
        conf.zero_()
    Ut, al = torch.zeros(n, device="cuda"), torch.zeros(n, device="cuda")
    dyn = torch.zeros(n, dtype=torch.uint8, device="cuda")
    pr = torch.zeros(n, dtype=torch.uint8, device="cuda")
    stats = torch.zeros(8, device="cuda")
    out = gs.MPOut(gs.ptr(Ut), gs.ptr(al), gs.ptr(dyn), gs.ptr(pr), None, None, gs.ptr(stats))
    ws = torch.zeros(gs.gs_workspace_size(ctx, views.s, gs.GS_OP_MP_UPDATE), dtype=torch.uint8, device="cuda")
    sched = schedule.PriorScheduler(P, policy=policy, n_fixed=n_fixed)
    # verification buffers
    pair = gs.ViewBatch([cams[0], cams[0]], n)
    mp_scratch = torch.empty_like(gd["mp"])
    tracker = optim.Tracker(ctx, gd, cams[0], max_rank=0, use_graph=True)
    T_est = [np.asarray(cams[0]["T_cw"], np.float64)]
    errs, flips, ms = [], [], []
    prev_dyn = prev_obs = None
    exact = True
    restored = 0
    for t in range(1, len(cams)):
        tc, td = _observe(ctx, cams[t], gs.to_device(obs[t]), n)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        T, _, ex = tracker.run(tc.reshape(-1).contiguous(), td, iters=track_iters, T_init=T_est[-1])
        exact = exact and ex
        T_est.append(T)
        # epipolar verification between frames t - 1 and t under the estimates
        amb = np.nonzero(prev_dyn)[0] if prev_dyn is not None else np.zeros(0, np.int64)
        half = min(k_cand // 2, amb.size)
        ids = np.unique(np.concatenate([rng.choice(amb, size=half, replace=False) if half else amb[:0],
                                        rng.choice(n, size=min(k_cand - half, n), replace=False)])).astype(np.int32)
        p1, p2, seg = synth.frame_matches(rng, obs[t - 1], obs[t], cams[t - 1], cams[t], ids, per, noise_px,
                                          outlier_frac)
        pair.set_pose(0, T_est[-2])
        pair.set_pose(1, T_est[-1])
        target_mp = gd["mp"] if cfg.get("recover", True) else mp_scratch
        if target_mp is mp_scratch:
            mp_scratch.copy_(gd["mp"])
        dev = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()
        d = torch.empty(max(p1.shape[1], 1), device="cuda")
        dbar = torch.empty(len(ids), device="cuda")
        est = torch.empty(len(ids), dtype=torch.uint8, device="cuda")
        gs.gs_epipolar_verify(ctx, pair.s, 0, 1, dev(p1), dev(p2), dev(ids), dev(seg), target_mp, d, dbar, est)
        if target_mp is not mp_scratch:
            restored += int((est == gs.GS_EPI_RESTORED).sum())
        go = sched.decide(dbar.cpu().numpy(), est.cpu().numpy())
        masks = sched.prior(dev(synth.box_masks(cams[t], obs[t], slices)))
        # the MP update at the estimated pose
        views.set_pose(0, T)
        pipe.forward(gst)
        frame = gs.MPFrame(gs.ptr(masks), K, gs.ptr(prior), gs.ptr(conf), int(go), None)
        tgt = gs.Target(gs.ptr(tc), gs.ptr(td))
        gs.gs_mp_update(ctx, views.s, pipe.proj, pipe.img, tgt, frame, params, gd["mp"], out, ws)
        torch.cuda.synchronize()
        sched.observe(stats)
        ms.append(1000.0 * (time.perf_counter() - t0))
        errs.append(_pose_errors(T, np.asarray(cams[t]["T_cw"], np.float64)))
        cur_dyn = dyn.cpu().numpy().astype(bool)
        cur_obs = al.cpu().numpy() > 0
        if prev_dyn is not None:
            both = cur_obs & prev_obs
            flips.append(float((cur_dyn[both] != prev_dyn[both]).mean()) if both.any() else 0.0)
        prev_dyn, prev_obs = cur_dyn, cur_obs
    mp = gd["mp"].cpu().numpy()
    seen = prev_obs
    ang = np.array([e[0] for e in errs])
    dist = np.array([e[1] for e in errs])
    return dict(variant=variant, policy=policy, frames=len(cams) - 1, refreshes=sched.refreshes,
                flip_ratio_pct=round(100.0 * float(np.mean(flips)) if flips else 0.0, 3),
                mp_abs_error=round(float(np.abs(mp[seen] - truth[seen]).mean()), 4),
                label_error_pct=round(100.0 * float((prev_dyn[seen] != truth[seen]).mean()), 3),
                ate_cm=round(100.0 * float(np.sqrt(np.mean(dist ** 2))), 4),
                rot_err_deg=round(float(ang.mean()), 4), ms_per_frame=round(float(np.median(ms)), 3),
                restored=restored, exact=bool(exact))


def ablation(ctx, seed=31, n=100_000, W=320, H=240, frames=40, variants=None, **kw):
    """Every variant on one sequence; a list of metric dicts."""
    seq = synth.box_sequence(seed, n, W, H, frames, box_frac=0.08, zmin=1.5, zmax=5.0)
    return [run(ctx, seq, v, **kw) for v in (variants or VARIANTS)]
