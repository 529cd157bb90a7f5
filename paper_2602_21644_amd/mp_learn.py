"""The per-frame MP loop and the learned MP surrogate (the surrogate is not
in the paper).

MPFrame      one view of one scene: renders the map at the frame's pose
             (gs_project with the planar projection, gs_bin_sort,
             gs_render_fwd) and runs the temporal MP update (gs_mp_update,
             Eq. (1)-(13), (17)) against the observed frame, with the plain
             residual cue or the surrogate's per-pixel M_p.
MPSurrogate  the 8 -> 32 -> 32 -> 1 per-pixel network: float32 masters,
             bfloat16 copies and Adam state on the device; trained with
             gs_mlp_train_step on (gs_mlp_features, plain M_p) pairs.
observe      renders an observed frame (colour, depth with holes where the
             accumulated opacity is below 0.5, instance map of the moving
             boxes) with the library, as the synthetic stand-in for an RGB-D
             frame and its segmentation.
train_c5 / evaluate_c5
             the learned-MP protocol at scale: the surrogate trained on the
             plain cue's M_p over 20 sequences of 100 frames, then five
             held-out sequences tracked and MP-updated with the plain cue and
             with the surrogate, which falls back to the plain cue for a few
             frames whenever its mean disagreement with the plain cue (the
             error judge gs_mp_update forms beside it) exceeds a bound.

Every kernel runs in libgs.so; torch holds the buffers.
"""

from __future__ import annotations

import numpy as np
import torch

from . import gs, synth

MLP_SHAPES = (("W1", (32, 8)), ("b1", (32,)), ("W2", (32, 32)), ("b2", (32,)), ("W3", (1, 32)), ("b3", (1,)))


def _render(ctx, g_dev, cam, capacity=None):
    n = int(g_dev["opacity_logit"].shape[0])
    views = gs.ViewBatch([cam], n)
    pipe = gs.Pipeline(ctx, views, capacity or max(1 << 20, 64 * n))
    pipe.forward(gs.gaussians_struct(g_dev))
    over, _, _ = pipe.check()
    if over:
        raise RuntimeError("binning capacity exceeded")
    return pipe


def observe(ctx, g_obs_dev, cam, slices, valid_A=0.5):
    """Observed frame of the scene state g_obs_dev: colour [3P], depth [P]
    (0 where A < valid_A), instance ids [P] (box k + 1 where its rendered
    indicator covers more than half of the accumulated opacity)."""
    pipe = _render(ctx, g_obs_dev, cam)
    A = 1.0 - pipe.img_T
    tc = pipe.img_color.clone()
    td = torch.where(A >= valid_A, pipe.img_depth, torch.zeros_like(A)).contiguous()
    inst = torch.zeros_like(pipe.img_nlast, dtype=torch.int32)
    ind = dict(g_obs_dev)
    for k, sl in enumerate(slices):
        m = torch.zeros_like(g_obs_dev["mp"])
        m[sl] = 1.0
        ind["mp"] = m
        pk = _render(ctx, ind, cam)
        Ak = (1.0 - pk.img_T).clamp_min(1e-12)
        inst = torch.where((pk.img_mp / Ak > 0.5) & (Ak > 1e-6), torch.full_like(inst, k + 1), inst)
    return tc, td, inst.contiguous()


class MPSurrogate:
    """Per-pixel MP network with its device state."""

    def __init__(self, ctx, seed=0, device="cuda"):
        self.ctx = ctx
        rng = np.random.default_rng(seed)
        parts = []
        for name, shp in MLP_SHAPES:
            if name.startswith("W"):
                fan_in = shp[1]
                parts.append(rng.normal(0, np.sqrt(2.0 / fan_in), size=shp).astype(np.float32).reshape(-1))
            else:
                parts.append(np.zeros(int(np.prod(shp)), np.float32))
        self.master = torch.from_numpy(np.concatenate(parts)).to(device)
        self.w_bf16 = torch.zeros(gs.GS_MLP_WEIGHTS, dtype=torch.int16, device=device)
        self.m = torch.zeros(gs.GS_MLP_PARAMS, device=device)
        self.v = torch.zeros(gs.GS_MLP_PARAMS, device=device)
        self.s = gs.MLP(gs.ptr(self.master), gs.ptr(self.w_bf16), gs.ptr(self.m), gs.ptr(self.v))
        self.steps = 0
        self.loss = torch.zeros(1, device=device)
        self._ws = {}
        gs.gs_mlp_sync(ctx, self.s)

    def _workspace(self, views):
        P = views.pixel_count
        if P not in self._ws:
            self._ws[P] = torch.zeros(gs.gs_workspace_size(self.ctx, views.s, gs.GS_OP_MLP_TRAIN), dtype=torch.uint8,
                                      device=self.master.device)
        return self._ws[P]

    def train_step(self, views, x, label, lr=3e-3):
        """One Adam step on the mean BCE against label [P]; returns the loss
        before the step (device tensor [1])."""
        self.steps += 1
        P = views.pixel_count
        gs.gs_mlp_train_step(self.ctx, self.s, x, label, P, lr, self.steps, self.loss, None, self._workspace(views))
        return self.loss

    def predict(self, x, y):
        gs.gs_mlp_fwd(self.ctx, self.s, x, y, y.numel())


class MPFrame:
    """Temporal MP update of one scene seen by one camera, frame by frame."""

    def __init__(self, ctx, g_dev, cam, params=None):
        self.ctx = ctx
        self.g = g_dev
        self.gst = gs.gaussians_struct(g_dev)
        n = int(g_dev["opacity_logit"].shape[0])
        self.n = n
        self.views = gs.ViewBatch([cam], n)
        self.pipe = gs.Pipeline(ctx, self.views, max(1 << 20, 64 * n), full_proj=True)
        dev = g_dev["mean"].device
        P = self.pipe.P
        self.P = P
        self.Ut = torch.zeros(n, device=dev)
        self.alpha = torch.zeros(n, device=dev)
        self.dyn = torch.zeros(n, dtype=torch.uint8, device=dev)
        self.prune = torch.zeros(n, dtype=torch.uint8, device=dev)
        self.Mp = torch.zeros(P, device=dev)
        self.e = torch.zeros(P, device=dev)
        self.stats = torch.zeros(8, device=dev)
        self.judge = torch.zeros(2, device=dev)
        self.out = gs.MPOut(gs.ptr(self.Ut), gs.ptr(self.alpha), gs.ptr(self.dyn), gs.ptr(self.prune),
                            gs.ptr(self.Mp), gs.ptr(self.e), gs.ptr(self.stats), gs.ptr(self.judge))
        self.ws = torch.zeros(gs.gs_workspace_size(ctx, self.views.s, gs.GS_OP_MP_UPDATE), dtype=torch.uint8,
                              device=dev)
        self.x = torch.zeros(8 * P, device=dev)
        self.y = torch.zeros(P, device=dev)
        p = dict(gs.MP_DEFAULTS)
        if params:
            p.update(params)
        self.params = gs.MPParams(*[p[k] for k in gs.MP_PARAM_NAMES], int(p["mode"]), int(p["u_norm"]))

    def _frame(self, inst, prior, conf, seg_updated, mlp_mp=None):
        return gs.MPFrame(gs.ptr(inst), int(prior.numel()) - 1, gs.ptr(prior), gs.ptr(conf), int(seg_updated),
                          gs.ptr(mlp_mp))

    def step(self, cam_T, tc, td, inst, prior, conf, seg_updated=True, surrogate=None):
        """Renders the map at pose cam_T and updates the scene's MP in place.
        With a surrogate, its M_p replaces the plain residual cue. Leaves the
        features of the frame in self.x and the M_p used in self.Mp."""
        self.views.set_pose(0, cam_T)
        self.pipe.forward(self.gst)
        tgt = gs.Target(gs.ptr(tc), gs.ptr(td))
        fr = self._frame(inst, prior, conf, seg_updated)
        gs.gs_mlp_features(self.ctx, self.views.s, self.pipe.img, tgt, fr, self.x)
        mlp_mp = None
        if surrogate is not None:
            surrogate.predict(self.x, self.y)
            mlp_mp = self.y
        fr = self._frame(inst, prior, conf, seg_updated, mlp_mp)
        gs.gs_mp_update(self.ctx, self.views.s, self.pipe.proj, self.pipe.img, tgt, fr, self.params, self.g["mp"],
                        self.out, self.ws)


def instance_tables(n_boxes, device="cuda", prior_box=0.9, conf_box=0.9, prior_bg=0.05, conf_bg=0.1):
    """Instance prior mu and confidence c of the background and the boxes
    (the values this library takes where the paper gives none)."""
    prior = torch.tensor([prior_bg] + [prior_box] * n_boxes, dtype=torch.float32, device=device)
    conf = torch.tensor([conf_bg] + [conf_box] * n_boxes, dtype=torch.float32, device=device)
    return prior, conf


def run_sequence(ctx, seq, surrogate=None, train=False, lr=3e-3, steps_per_frame=4, params=None):
    """MP updates over a box_sequence with the plain cue (training the
    surrogate on its M_p when train=True) or with the surrogate's M_p. At
    frame t the map holds the scene state of frame t - 1.
    Returns (final MP [n] host, observed [n] host: updated at least once,
    training losses [frames, steps_per_frame] host or None)."""
    g = gs.to_device(seq["map"])
    cam0 = seq["cams"][0]
    mpf = MPFrame(ctx, g, cam0, params=params)
    prior, conf = instance_tables(len(seq["slices"]))
    observed = torch.zeros(mpf.n, dtype=torch.bool, device=g["mp"].device)
    losses = []
    prev = [seq["map"]] + seq["obs"][:-1]
    for cam, g_obs, g_prev in zip(seq["cams"], seq["obs"], prev):
        # the map holds the boxes where they were one frame earlier
        g["mean"].copy_(torch.from_numpy(g_prev["mean"]))
        tc, td, inst = observe(ctx, gs.to_device(g_obs), cam, seq["slices"])
        mpf.step(cam["T_cw"], tc, td, inst, prior, conf, surrogate=None if train else surrogate)
        observed |= mpf.alpha > 0
        if train:
            label = mpf.Mp.clone()
            for _ in range(steps_per_frame):
                losses.append(surrogate.train_step(mpf.views, mpf.x, label, lr).clone())
    torch.cuda.synchronize()
    mp = g["mp"].cpu().numpy().astype(np.float64)
    tl = torch.cat(losses).view(-1, steps_per_frame).cpu().numpy() if losses else None
    return mp, observed.cpu().numpy(), tl


def mp_error(mp, dynamic, observed=None):
    """Mean |MP - flag| against the ground-truth dynamic flags."""
    err = np.abs(mp - dynamic.astype(np.float64))
    return float(err[observed].mean()) if observed is not None else float(err.mean())


class DeviceSequence:
    """A box sequence (synth.box_sequence, materialize=False) on the device:
    the map's parameters once, and frame states made by moving the box slices
    of a mean plane in place."""

    def __init__(self, seq, device="cuda"):
        self.seq = seq
        self.base = gs.to_device(seq["map"], device=device)
        self.mean0 = self.base["mean"].clone()
        self.deltas = [torch.tensor(np.stack(d).T if d else np.zeros((3, 0)), dtype=torch.float32,
                                    device=self.mean0.device) for d in seq["deltas"]]

    def frames(self):
        return len(self.seq["cams"])

    def set_state(self, mean, t):
        """mean <- the scene's means at frame t (t < 0: the map as built)."""
        mean.copy_(self.mean0)
        if t >= 0:
            for k, sl in enumerate(self.seq["slices"]):
                mean[:, sl] += self.deltas[t][:, k:k + 1]

    def view(self, mean=None, mp=None):
        """A Gaussian dict sharing the map's planes, with its own mean/mp
        tensors when given."""
        g = dict(self.base)
        if mean is not None:
            g["mean"] = mean
        if mp is not None:
            g["mp"] = mp
        return g


def c5_sequence(seed, n, width, height, frames):
    """A C5-protocol sequence: 1-5 moving boxes (5% of the Gaussians) in front
    of a static layer 3-6 m away, so that the boxes are seen."""
    return synth.box_sequence(seed, n, width, height, frames, n_boxes=1 + seed % 5, box_frac=0.05, zmin=3.0,
                              zmax=6.0, materialize=False)


def train_c5(ctx, seeds=range(1000, 1020), n=1_000_000, width=640, height=480, frames=100, steps_per_frame=2,
             lr=3e-3, surrogate=None, log=None):
    """Trains a surrogate on the plain cue's M_p of every frame of the
    training sequences (true poses; the map holds each box where it was one
    frame earlier). Returns (surrogate, frames used, mean BCE of the first and
    the last 100 steps)."""
    sur = surrogate or MPSurrogate(ctx, seed=0)
    losses = []
    used = 0
    for seed in seeds:
        ds = DeviceSequence(c5_sequence(seed, n, width, height, frames))
        obs_mean = torch.empty_like(ds.mean0)
        map_mean = torch.empty_like(ds.mean0)
        mp = torch.full_like(ds.base["mp"], 0.5)
        g_map = ds.view(map_mean, mp)
        g_obs = ds.view(obs_mean)
        mpf = MPFrame(ctx, g_map, ds.seq["cams"][0])
        prior, conf = instance_tables(len(ds.seq["slices"]))
        for t in range(ds.frames()):
            ds.set_state(map_mean, t - 1)
            ds.set_state(obs_mean, t)
            cam = ds.seq["cams"][t]
            tc, td, inst = observe(ctx, g_obs, cam, ds.seq["slices"])
            mpf.step(cam["T_cw"], tc, td, inst, prior, conf)
            label = mpf.Mp.clone()
            for _ in range(steps_per_frame):
                losses.append(sur.train_step(mpf.views, mpf.x, label, lr).clone())
            used += 1
        if log:
            log(f"trained on sequence {seed}: {used} frames")
        del mpf, ds
        torch.cuda.empty_cache()
    tl = torch.cat(losses).cpu().numpy()
    k = min(100, tl.size)
    return sur, used, float(tl[:k].mean()), float(tl[-k:].mean())


def evaluate_c5(ctx, surrogate, seeds=range(5000, 5005), n=1_000_000, width=640, height=480, frames=100,
                track_iters=10, judge_max=0.15, fallback_frames=5):
    """Held-out sequences tracked from the first frame's true pose (pose-only
    tracking of the MP-weighted loss, full lists) and MP-updated at the
    tracked pose, once with the plain cue and once with the surrogate under
    the fallback rule. Returns per form: MP abs error and label error over
    the Gaussians observed at least once, camera-centre RMSE (cm), mean
    rotation error (deg), the MP source's milliseconds per frame, and for the
    surrogate the share of frames it served and its mean disagreement."""
    from . import optim
    res = {}
    for form in ("plain", "learned"):
        mp_err, lab_err, dists, angs, ms_src, served, dev = [], [], [], [], [], [], []
        for seed in seeds:
            ds = DeviceSequence(c5_sequence(seed, n, width, height, frames))
            obs_mean = torch.empty_like(ds.mean0)
            map_mean = torch.empty_like(ds.mean0)
            mp = torch.full_like(ds.base["mp"], 0.5)
            g_map = ds.view(map_mean, mp)
            g_obs = ds.view(obs_mean)
            cams = ds.seq["cams"]
            ds.set_state(map_mean, -1)
            mpf = MPFrame(ctx, g_map, cams[0])
            trk = optim.Tracker(ctx, g_map, cams[0], max_rank=0, capacity=64 * n + (1 << 16), use_graph=True)
            prior, conf = instance_tables(len(ds.seq["slices"]))
            observed = torch.zeros(mpf.n, dtype=torch.bool, device=mp.device)
            T_prev = np.asarray(cams[0]["T_cw"], np.float64)
            cool = 0
            for t in range(1, ds.frames()):
                ds.set_state(map_mean, t - 1)
                ds.set_state(obs_mean, t)
                tc, td, inst = observe(ctx, g_obs, cams[t], ds.seq["slices"])
                T, _, _ = trk.run(tc.reshape(-1).contiguous(), td, iters=track_iters, T_init=T_prev)
                T_prev = T
                use = form == "learned" and cool == 0
                torch.cuda.synchronize()
                e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                e0.record()
                mpf.step(T, tc, td, inst, prior, conf, surrogate=surrogate if use else None)
                e1.record()
                e1.synchronize()
                ms_src.append(e0.elapsed_time(e1))
                observed |= mpf.alpha > 0
                if form == "learned":
                    served.append(use)
                    if use:
                        j = mpf.judge.cpu().numpy()
                        d = float(j[0] / max(j[1], 1.0))
                        dev.append(d)
                        if d > judge_max:
                            cool = fallback_frames
                    elif cool > 0:
                        cool -= 1
                R_ref = np.asarray(cams[t]["T_cw"], np.float64)
                dR = T[:, :3] @ R_ref[:, :3].T
                angs.append(float(np.degrees(np.arccos(np.clip((np.trace(dR) - 1) / 2, -1, 1)))))
                c = -T[:, :3].T @ T[:, 3]
                c_ref = -R_ref[:, :3].T @ R_ref[:, 3]
                dists.append(float(np.linalg.norm(c - c_ref)))
            ob = observed.cpu().numpy()
            dyn = ds.seq["dynamic"]
            mpv = mp.cpu().numpy().astype(np.float64)
            mp_err.append(mp_error(mpv, dyn, ob))
            lab = mpf.dyn.cpu().numpy().astype(bool)
            lab_err.append(float((lab[ob] != dyn[ob]).mean()))
            del trk, mpf, ds
            torch.cuda.empty_cache()
        r = dict(mp_abs_error=round(float(np.mean(mp_err)), 4), label_error_pct=round(100 * float(np.mean(lab_err)), 3),
                 ate_cm=round(100 * float(np.sqrt(np.mean(np.square(dists)))), 4),
                 rot_err_deg=round(float(np.mean(angs)), 4), ms_per_frame_mp=round(float(np.median(ms_src)), 4))
        if form == "learned":
            r["surrogate_frames_pct"] = round(100 * float(np.mean(served)), 2)
            r["mean_disagreement"] = round(float(np.mean(dev)), 4) if dev else None
        res[form] = r
    return res
