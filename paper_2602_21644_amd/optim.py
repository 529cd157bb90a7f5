"""Optimisation around the library calls: the joint optimisation of Gaussian
parameters and camera poses (Sec. IV-D). Every kernel runs in libgs.so; torch
holds the buffers and the stream.

RenderLoss     torch.autograd.Function: forward = gs_project, gs_bin_sort,
               gs_render_fwd and gs_loss (one loss per view); backward =
               gs_render_bwd (the Gaussian parameter gradients, and the
               gradient of the left pose twist of every view at its current
               pose).
Adam           device state of a list of tensors, stepped by gs_adam_step.
track          pose-only tracking of one frame: Adam steps on the left twist,
               each retracted onto SE(3) by gs_pose_update; the iteration is
               captured once in a HIP graph and replayed.
map_gaussians  Adam steps on the Gaussian parameters against a batch of views.

(The paper refines poses with Levenberg-Marquardt; these loops take
first-order steps on the same gradients.)
"""

from __future__ import annotations

import numpy as np
import torch

from . import gs

PARAMS = ("mean", "log_scale", "quat", "opacity_logit", "color")


class RenderLoss(torch.autograd.Function):
    """loss[V] = RenderLoss.apply(pipe, mp, target_color, target_depth,
    mean, log_scale, quat, opacity_logit, color, pose)

    `pipe` is a gs.Pipeline over the views; `pose` a [V, 6] zero tensor that
    stands for the left twist (rho, phi) of every view at its current pose
    (its gradient is the pose gradient). MP is a state, not a parameter: it
    gets no gradient.

    A forward whose lists overflowed their capacity, or whose tiles ran out of
    a truncated prefix list, is not exact: outside graph capture the forward
    synchronises and raises GSError then; under capture the pipeline's sticky
    flags record it and pipe.raise_if_failed() raises after the replays."""

    @staticmethod
    def forward(ctx, pipe, mp, target_color, target_depth, mean, log_scale, quat, opacity_logit, color, pose):
        g = dict(mean=mean.contiguous(), log_scale=log_scale.contiguous(), quat=quat.contiguous(),
                 opacity_logit=opacity_logit.contiguous(), color=color.contiguous(), mp=mp.contiguous())
        gst = gs.gaussians_struct(g)
        pipe.sticky = True
        pipe.forward_loss(gst, target_color.contiguous(), target_depth.contiguous())
        if not torch.cuda.is_current_stream_capturing():
            pipe.raise_if_failed()
        ctx.pipe, ctx.gst, ctx.keep = pipe, gst, g
        ctx.n = int(opacity_logit.shape[0])
        return pipe.loss.clone()

    @staticmethod
    def backward(ctx, gloss):
        pipe = ctx.pipe
        # each view's pixel adjoints enter the backward scaled by the incoming
        # gradient of its loss
        w = gloss.to(torch.float32).contiguous()
        pipe.pg.view_weight = gs.ptr(w)
        grads = gs.alloc_grads(ctx.n)
        pose = torch.zeros(6 * pipe.views.V, dtype=torch.float32, device=gloss.device)
        try:
            pipe.backward(ctx.gst, gs.grads_struct(grads, pose))
        finally:
            pipe.pg.view_weight = None
        return (None, None, None, None, grads["mean"], grads["log_scale"], grads["quat"], grads["opacity_logit"],
                grads["color"], pose.view(-1, 6))


class Adam:
    """Adam state (first and second moments, device step count) for a list of
    (tensor, lr); step() applies gs_adam_step with the given gradients."""

    def __init__(self, ctx, params, betas=(0.9, 0.999), eps=1e-8):
        self.ctx = ctx
        self.params = [(p, float(lr)) for p, lr in params]
        self.m = [torch.zeros_like(p) for p, _ in self.params]
        self.v = [torch.zeros_like(p) for p, _ in self.params]
        dev = self.params[0][0].device
        self.count = torch.zeros(1, dtype=torch.int32, device=dev)
        self.betas, self.eps = betas, eps

    def reset(self):
        for t in self.m + self.v:
            t.zero_()
        self.count.zero_()

    def step(self, grads, stream=None):
        """Graph-capturable: the step count advances on the device."""
        groups = [(p, g, m, v, lr) for (p, lr), g, m, v in zip(self.params, grads, self.m, self.v)]
        for i in range(0, len(groups), gs.ADAM_MAX_GROUPS):
            # the first call advances the count, the rest read the advanced one
            gs.gs_adam_step(self.ctx, groups[i:i + gs.ADAM_MAX_GROUPS], self.count, self.betas[0], self.betas[1],
                            self.eps, stream, advance=i == 0)


def choose_rank(ctx, views, gst, n, start=256):
    """Smallest power-of-two prefix rank (from `start`) whose prefix lists let
    every tile of the views saturate at their current poses, with the instance
    count it gives; (0, count) when none does (full lists)."""
    R = start
    cap = max(1 << 20, 16 * n)
    while True:
        probe = gs.Pipeline(ctx, views, capacity=cap, max_rank=R)
        probe.forward(gst)
        over, n_inst, inc = probe.check()
        del probe
        if over:
            # the library reports the count it needed: retry this rank with room for it
            if n_inst >= (1 << 32) - 1:
                raise RuntimeError("more list entries than 32-bit offsets hold")
            cap = int(n_inst * 1.1) + (1 << 16)
            continue
        if inc == 0 or R == 0:
            return R, n_inst
        R = R * 2 if R * 2 <= ctx.get_param("prefix_cap") else 0


class Tracker:
    """Pose-only tracking of one view against an observed frame.

    Every iteration renders at the current pose, takes the MP-weighted loss
    and its pose gradient (gs_render_bwd in pose-only mode), one Adam step on
    the left twist and the retraction T <- Exp(delta) T (gs_pose_update), all
    on the device. The iteration is captured once as a HIP graph."""

    def __init__(self, ctx, gaussians, cam, lr_rho=2e-3, lr_phi=2e-3, max_rank=-1, capacity=None, use_graph=True,
                 slack=4.0):
        self.ctx = ctx
        self.g = gaussians
        self.gst = gs.gaussians_struct(gaussians)
        n = int(gaussians["opacity_logit"].shape[0])
        self.views = gs.ViewBatch([cam], n)
        if max_rank < 0:
            R, n_inst = choose_rank(ctx, self.views, self.gst, n)
            # the pose moves during tracking: keep margin on the rank
            R = min(R * 2, ctx.get_param("prefix_cap")) if R else 0
        else:
            R, n_inst = max_rank, 64 * n
        self.rank = R
        cap = capacity or int(slack * max(n_inst, 1)) + (1 << 16)
        self.pipe = gs.Pipeline(ctx, self.views, cap, max_rank=R)
        dev = gaussians["mean"].device
        self.delta = torch.zeros(6, dtype=torch.float32, device=dev)
        self.dpose = torch.zeros(6, dtype=torch.float32, device=dev)
        self.adam = Adam(ctx, [(self.delta[:3], lr_rho), (self.delta[3:], lr_phi)])
        self.grs = gs.grads_struct(None, self.dpose, pose_only=True)
        self.pipe.sticky = True  # the library records overflow / incomplete across the replays
        self.flags = self.pipe.flags
        self.use_graph = use_graph
        self.graph = None
        self.tc = self.td = None

    def _iteration(self):
        p = self.pipe
        p.forward_loss(self.gst, self.tc, self.td)
        p.backward(self.gst, self.grs)
        self.adam.step([self.dpose[:3], self.dpose[3:]])
        gs.gs_pose_update(self.ctx, self.views, self.delta)

    def run(self, target_color, target_depth, iters=100, T_init=None):
        """Tracks from T_init (default: the current pose) for `iters`
        iterations; returns (T_cw [3, 4], final loss, exact) where `exact` is
        False when some iteration overflowed or ran out of its prefix lists."""
        if self.tc is None:
            self.tc = torch.empty_like(target_color)
            self.td = torch.empty_like(target_depth)
        self.tc.copy_(target_color)
        self.td.copy_(target_depth)
        if T_init is not None:
            self.views.set_pose(0, T_init)
        self.adam.reset()
        self.delta.zero_()
        self.flags.zero_()
        if self.use_graph and self.graph is None:
            # one eager iteration first (loads every kernel), then restore the
            # start and capture
            T0 = self.views.pose(0)
            self._iteration()
            torch.cuda.synchronize()
            self.views.set_pose(0, T0)
            self.adam.reset()
            self.delta.zero_()
            self.flags.zero_()
            s = torch.cuda.Stream()
            s.wait_stream(torch.cuda.current_stream())
            torch.cuda.synchronize()
            self.graph = torch.cuda.CUDAGraph()
            with torch.cuda.graph(self.graph, stream=s):
                self._iteration()
            torch.cuda.synchronize()
        for _ in range(iters):
            if self.graph is not None:
                self.graph.replay()
            else:
                self._iteration()
        # loss at the final pose
        self.pipe.forward_loss(self.gst, self.tc, self.td)
        torch.cuda.synchronize()
        exact = int(self.flags.sum()) == 0
        return self.views.pose(0), float(self.pipe.loss[0]), exact


def map_gaussians(ctx, gaussians, cams, target_color, target_depth, iters=50, lrs=None, max_rank=0,
                  view_scene=None, scene_begin=None):
    """Adam steps on the Gaussian parameters (in place) against a batch of
    views at fixed poses; returns the per-iteration total loss (host). Raises
    GSError when any iteration overflowed the list capacity or ran out of a
    truncated prefix list (max_rank > 0)."""
    lrs = lrs or dict(mean=1e-4, log_scale=5e-3, quat=1e-3, opacity_logit=2e-2, color=5e-3)
    n = int(gaussians["opacity_logit"].shape[0])
    views = gs.ViewBatch(cams, n, view_scene=view_scene, scene_begin=scene_begin)
    gst = gs.gaussians_struct(gaussians)
    pipe = gs.Pipeline(ctx, views, capacity=max(1 << 20, 64 * n * len(cams)), max_rank=max_rank)
    pipe.sticky = True
    grads = gs.alloc_grads(n)
    pose = torch.zeros(6 * len(cams), dtype=torch.float32, device=gaussians["mean"].device)
    grs = gs.grads_struct(grads, pose)
    adam = Adam(ctx, [(gaussians[k], lrs[k]) for k in PARAMS])
    losses = torch.zeros(iters, dtype=torch.float32, device=gaussians["mean"].device)
    for it in range(iters):
        pipe.forward_loss(gst, target_color, target_depth)
        losses[it] = pipe.loss.sum()
        pipe.backward(gst, grs)
        adam.step([grads[k] for k in PARAMS])
    pipe.raise_if_failed()
    return losses.cpu().numpy().astype(np.float64)


class MappingWindow:
    """The mapping window of one scene: V keyframes rendered and
    back-propagated together (one call sequence over the view batch), Adam on
    every Gaussian parameter; once per frame the MP update of the newest
    keyframe (gs_mp_update, log-odds mode by default) whose prune flag
    (MP > prune_above) drops Gaussians from the map: gs_compact moves the
    parameters, the MP state and the Adam moments of the kept ones into the
    second set of buffers. Both iterate() and frame_end() only enqueue work,
    so a caller can capture them in one HIP graph; commit() then reads the
    kept count (synchronising) and swaps the buffers, after which the
    pipelines are rebuilt for the smaller map (and a graph must be captured
    again).

    Sec. IV-D (joint optimisation over keyframes), Sec. IV-A Eq. (1)-(13) and
    Sec. IV-B Eq. (17) (the MP update); the prune and the log-odds form are
    this library's options, not the paper's (which suppresses dynamic
    Gaussians and recovers them later)."""

    PLANES = (("mean", 3), ("log_scale", 3), ("quat", 4), ("opacity_logit", 1), ("color", 3), ("mp", 1))

    def __init__(self, ctx, gaussians, cams, max_rank=-1, capacity=None, lrs=None, mp_params=None,
                 full_objective=True, lambda_mp=500.0, lambda_edge=300.0, edge_params=None):
        """max_rank < 0: the smallest exact prefix rank (choose_rank), chosen
        again whenever the map changes; capacity then 1.5x its list entries.
        full_objective: the iterations minimise the whole of Eq. (27), adding
        lambda_mp L_MP (against the means at the end of the previous frame)
        and lambda_edge L_edge over consecutive keyframes (i, i + 1) to the
        photometric and depth terms."""
        self.full = bool(full_objective)
        self.lambda_mp, self.lambda_edge = float(lambda_mp), float(lambda_edge)
        self.edge_params = dict(delta=0.05, edge_thresh=0.05, eps_A=1e-6)
        if edge_params:
            self.edge_params.update(edge_params)
        self.ctx = ctx
        self.cams = list(cams)
        self.lrs = lrs or dict(mean=1e-4, log_scale=5e-3, quat=1e-3, opacity_logit=2e-2, color=5e-3)
        p = dict(gs.MP_DEFAULTS, mode=1, prune_above=0.8)
        if mp_params:
            p.update(mp_params)
        self.mp_params = gs.MPParams(*[p[k] for k in gs.MP_PARAM_NAMES], int(p["mode"]), int(p["u_norm"]))
        self.max_rank = max_rank
        self.capacity = capacity
        self._build(gaussians, None)

    def _build(self, gaussians, adam_state):
        ctx = self.ctx
        self.g = gaussians
        n = int(gaussians["opacity_logit"].shape[0])
        self.n = n
        dev = gaussians["mean"].device
        self.gst = gs.gaussians_struct(gaussians)
        self.views = gs.ViewBatch(self.cams, n)
        if self.max_rank < 0:
            self.rank, n_inst = choose_rank(ctx, self.views, self.gst, n)
            cap = int(1.5 * n_inst) + (1 << 16)
        else:
            self.rank = self.max_rank
            cap = self.capacity or max(1 << 20, 64 * n * len(self.cams))
        self.pipe = gs.Pipeline(ctx, self.views, cap, max_rank=self.rank)
        self.pipe.sticky = True
        self.grads = gs.alloc_grads(n, device=dev)
        self.pose = torch.zeros(6 * len(self.cams), dtype=torch.float32, device=dev)
        self.grs = gs.grads_struct(self.grads, self.pose)
        self.adam = Adam(ctx, [(gaussians[k], self.lrs[k]) for k in PARAMS])
        if adam_state is not None:
            for dst, src in zip(self.adam.m + self.adam.v, adam_state[0] + adam_state[1]):
                dst.copy_(src)
            self.adam.count.copy_(adam_state[2])
        # the MP update of the newest keyframe needs its own projection with
        # the planar means
        self.mp_views = gs.ViewBatch([self.cams[-1]], n)
        self.mp_pipe = gs.Pipeline(ctx, self.mp_views, max(1 << 20, 64 * n), full_proj=True)
        self.mp_pipe.sticky = True
        self.Ut = torch.zeros(n, device=dev)
        self.alpha = torch.zeros(n, device=dev)
        self.dyn = torch.zeros(n, dtype=torch.uint8, device=dev)
        self.prune = torch.zeros(n, dtype=torch.uint8, device=dev)
        self.stats = torch.zeros(8, device=dev)
        self.mp_out = gs.MPOut(gs.ptr(self.Ut), gs.ptr(self.alpha), gs.ptr(self.dyn), gs.ptr(self.prune), None, None,
                               gs.ptr(self.stats))
        self.mp_ws = torch.zeros(gs.gs_workspace_size(ctx, self.mp_views.s, gs.GS_OP_MP_UPDATE), dtype=torch.uint8,
                                 device=dev)
        # compaction: every per-Gaussian plane (parameters, MP, Adam moments)
        self.src_planes = self._planes(gaussians, self.adam)
        self.dst = {k: torch.empty_like(v) for k, v in gaussians.items()}
        self.dst_m = [torch.empty_like(t) for t in self.adam.m]
        self.dst_v = [torch.empty_like(t) for t in self.adam.v]
        self.dst_planes = self._planes(self.dst, None, self.dst_m, self.dst_v)
        self.n_out = torch.zeros(1, dtype=torch.int64, device=dev)
        self.cp_ws = torch.empty(gs.gs_workspace_size(ctx, None, gs.GS_OP_COMPACT, n), dtype=torch.uint8, device=dev)
        # the further terms: the means at the end of the previous frame, the
        # keyframe pairs of the edge term, their losses and scratch
        V = len(self.cams)
        self.mean_prev = gaussians["mean"].clone()
        self.pairs = [(v, v + 1) for v in range(V - 1)]
        self.loss_mp = torch.zeros(1, device=dev)
        self.loss_edge = torch.zeros(max(1, len(self.pairs)), device=dev)
        self.pose_edge = torch.zeros(6 * V, device=dev)
        self.mp_reg_ws = torch.empty(gs.gs_workspace_size(ctx, None, gs.GS_OP_MP_REG, n), dtype=torch.uint8,
                                     device=dev)
        self.edge_ws = torch.empty(max(1, gs.gs_workspace_size(ctx, self.views.s, gs.GS_OP_EDGE_WARP,
                                                                len(self.pairs))), dtype=torch.uint8, device=dev)

    def _planes(self, g, adam, m=None, v=None):
        out = []
        for k, c in self.PLANES:
            out += [g[k].view(c, -1)[i] for i in range(c)] if c > 1 else [g[k].view(-1)]
        for lst in ((adam.m if adam else m), (adam.v if adam else v)):
            for t, (k, c) in zip(lst, self.PLANES[:-1]):
                out += [t.view(c, -1)[i] for i in range(c)] if c > 1 else [t.view(-1)]
        return out

    def iterate(self, target_color, target_depth):
        """One iteration over the window: render + loss + backward of every
        keyframe (with the edge-warp and motion-consistency terms when the
        full objective is on), one Adam step on every Gaussian parameter."""
        p = self.pipe
        p.forward_loss(self.gst, target_color, target_depth)
        if self.full and self.pairs:
            tgt = gs.Target(gs.ptr(target_color), gs.ptr(target_depth))
            self._tgt_keep = (target_color, target_depth)
            gs.gs_edge_warp(self.ctx, self.views.s, p.img, tgt, self.pairs, self.loss_edge, p.dD, self.pose_edge,
                            self.edge_ws, lam=self.lambda_edge, **self.edge_params)
        p.backward(self.gst, self.grs)
        if self.full:
            gs.gs_mp_regularizer(self.ctx, self.g["mean"], self.mean_prev, self.g["mp"], self.loss_mp,
                                 self.grads["mean"], self.mp_reg_ws, lam=self.lambda_mp)
        self.adam.step([self.grads[k] for k in PARAMS])

    def objective(self):
        """The last iteration's L_G terms (synchronises): photometric + depth
        per keyframe, l3 L_MP, l4 L_edge per keyframe pair."""
        return dict(render=self.pipe.loss.cpu().numpy(), mp=float(self.loss_mp[0]),
                    edge=self.loss_edge[:len(self.pairs)].cpu().numpy())

    def frame_end(self, target_color, target_depth, instance_id, prior, conf, seg_updated=True):
        """The newest keyframe's MP update against its observed frame (colour,
        depth, instance ids, prior and confidence tables), then the map
        compacted by the prune flag into the second buffers."""
        self.mp_pipe.forward(self.gst)
        tgt = gs.Target(gs.ptr(target_color), gs.ptr(target_depth))
        fr = gs.MPFrame(gs.ptr(instance_id), int(prior.numel()) - 1, gs.ptr(prior), gs.ptr(conf), int(seg_updated),
                        None)
        gs.gs_mp_update(self.ctx, self.mp_views.s, self.mp_pipe.proj, self.mp_pipe.img, tgt, fr, self.mp_params,
                        self.g["mp"], self.mp_out, self.mp_ws)
        gs.gs_compact(self.ctx, self.prune, self.src_planes, self.dst_planes, self.n_out, self.cp_ws)

    def commit(self):
        """Makes the compacted map current (synchronises); raises if any
        iteration since the last commit was not exact. Returns the new count."""
        self.pipe.raise_if_failed()
        self.mp_pipe.raise_if_failed()
        k = int(self.n_out.item())
        g = {key: (t.view(-1, self.n)[:, :k] if t.dim() > 1 else t[:k]).contiguous() for key, t in self.dst.items()}
        m = [(t.view(-1, self.n)[:, :k] if t.dim() > 1 else t[:k]).contiguous() for t in self.dst_m]
        v = [(t.view(-1, self.n)[:, :k] if t.dim() > 1 else t[:k]).contiguous() for t in self.dst_v]
        self._build(g, (m, v, self.adam.count.clone()))
        return k
