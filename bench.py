#!/usr/bin/env python
"""Benchmark of one MP-weighted render + loss + backward iteration.

Workload: 1,000,000 Gaussians (95% static, uniform in the 0.5-4 m frustum
volume; 5% on three moving boxes), one 640x480 view, full gradients to every
Gaussian parameter and the pose twist. The target RGB-D frame is rendered by
the same library at a camera 0.5 degree / 1 cm away with the boxes moved.

A step is gs_project -> gs_bin_sort -> gs_render_fwd_loss (the MP-weighted
loss fused into the forward) -> gs_render_bwd: one optimisation iteration
(the per-frame MP update is timed beside it). The prefix rank is the smallest
exact one and the launch knobs are autotuned first. The timed region replays
a hip graph of the step K times (inputs resident in HBM); a second timed
region runs K eager steps with every kernel bracketed by HIP events, which
gives per-kernel durations for the roofline entries: `roofline` for the
kernel that takes the most time, `roofline_iteration` for the whole step's
algorithmic HBM bytes against the HBM peak. The oracle is timed on the host
over whole iterations (every pixel, every Gaussian) for about 10 seconds.

Prints one JSON line.
"""

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "MP-weighted render+backward iters/s @640×480, 1M Gaussians; % HBM roofline"
HBM_PEAK_GBS = 8000.0
FP32_VECTOR_PEAK_TFS = 157.3  # 256 CUs x 4 SIMDs x 2.4 GHz x 64 FP32 FLOP/clk (packed FP32)
# FP32 FLOPs per (pixel, composited entry) pair of the compositing kernels
FLOPS_PER_PAIR = {"render_fwd_kernel": 28, "render_bwd_kernel": 54}
# HBM traffic per launch from rocprofv3 --pmc (FETCH_SIZE, WRITE_SIZE in KiB) at
# this workload, valid while the kernel source hashes to the recorded value;
# the counters are scaled by what they read for a 256 MiB device copy
# (FETCH_SIZE x 2.0, WRITE_SIZE x 1.0)
PMC_TRAFFIC = {
    "render_bwd_kernel<64>": {"fetch_kib": 10424.3, "write_kib": 60458.2,
                              "sha256": "84df235f5b401b14f8f7c6a538a2265db34bf945b90f94389e674129150004c9"},
    "render_bwd_kernel<32>": {"fetch_kib": 10374.1, "write_kib": 60464.9,
                              "sha256": "84df235f5b401b14f8f7c6a538a2265db34bf945b90f94389e674129150004c9"},
}
PMC_SCALE = {"fetch": 2.0, "write": 1.0}


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--n", type=int, default=1_000_000)
    ap.add_argument("--width", type=int, default=640)
    ap.add_argument("--height", type=int, default=480)
    ap.add_argument("--seed", type=int, default=11)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-graph", action="store_true")
    ap.add_argument("--max-rank", type=int, default=-1,
                    help="prefix rank for binning (-1: smallest power of two >= 256 that is exact; 0: full lists)")
    ap.add_argument("--no-tune", action="store_true", help="keep the default launch knobs")
    ap.add_argument("--knobs", default="",
                    help="comma-separated name=value context knobs set before tuning (e.g. bwd_batch=64)")
    ap.add_argument("--profile-tracking", type=int, default=0,
                    help="only run the tracking configuration for this many graph-replayed iterations (after the "
                         "capture's two), for a profiler")
    ap.add_argument("--oracle-timing", action="store_true",
                    help="only time the FP64 oracle (C1, C2, the metric workload, one window view) on the host, "
                         "on all threads and on one, and print the table as JSON")
    ap.add_argument("--no-extras", action="store_true",
                    help="skip the batched-window, uneven-batch and learned-MP forms reported beside the step")
    ap.add_argument("--profile-steps", type=int, default=0,
                    help="run only this many eager steps (for rocprofv3) and exit")
    ap.add_argument("--copy-bytes", type=int, default=0,
                    help="with --profile-steps: first copy this many bytes device to device once (a plain copy "
                         "kernel of known size that calibrates the HBM byte counters)")
    return ap.parse_args()


def kernel_bytes(name, st):
    """Algorithmic HBM bytes of one launch of `name` for this workload."""
    N, I, P, T, Mrec = st["n"], st["instances"], st["pixels"], st["tiles"], st["records"]
    if name.startswith("project_kernel"):
        return N * 44 + Mrec * (8 + 4)
    if name.startswith("psel_kernel"):
        return Mrec * 4 + st["selected"] * (60 + 48 + 8 + 16)
    if name.startswith("psort_kernel"):
        return st["selected"] * (16 + 12)
    if name.startswith("ptiles_kernel"):
        return st["selected"] * 12 + I * 4
    if name.startswith("radix_hist_kernel"):
        return Mrec * 4
    if name.startswith("radix_scatter_kernel"):
        return Mrec * 16
    if name.startswith("bin_count_kernel"):
        return st["nlim"] * 16 + st["cm"] * 4
    if name.startswith("bin_scatter_kernel"):
        return st["nlim"] * 16 + st["cm"] * 4 + I * 4
    if name.startswith("render_fwd_kernel"):
        # with the loss fused in: targets read (16 B) and adjoints written (24 B) per pixel
        return st["loaded_fwd"] * 52 + P * (28 + (40 if st.get("fused_loss") else 0))
    if name.startswith("loss_kernel"):
        return P * 68
    if name.startswith("render_bwd_kernel"):
        # list entries and pixel state read, the 2D adjoint of touched records
        # accumulated, and the dense gradient planes cleared (14 floats each)
        return st["loaded_bwd"] * 52 + P * 32 + st["touched"] * 40 + N * 56
    if name.startswith("bwd_project_kernel"):
        # per listed Gaussian: parameters, list entry and flag, the 2D adjoint
        # copies read and cleared, the gradients written
        return st["touched"] * (44 + 8 + 80 * st.get("copies", 1) + 56)
    return None


def main():
    a = parse()
    if a.oracle_timing:
        print(json.dumps(oracle_timing()), flush=True)
        return
    if a.profile_tracking > 0:
        from paper_2602_21644_amd import gs
        ctx = gs.Context(0)
        for kv in filter(None, a.knobs.split(",")):
            name, val = kv.split("=")
            ctx.set_param(name.strip(), int(val))
        tracking_run(ctx, iters=a.profile_tracking)
        return
    if a.gpus != 1:
        print(json.dumps({"error": "mpsplat runs on one GPU; --gpus must be 1 (sharding the views over "
                                   "several GPUs is not implemented)"}))
        sys.exit(2)
    import torch

    from paper_2602_21644_amd import gs, synth

    dev = "cuda"
    torch.cuda.set_device(0)
    CLOCKS["start"] = rocm_smi_clocks()
    log(f"[bench] workload: {a.n} Gaussians, {a.width}x{a.height}")
    g, cam, tcam, g_t, sl = synth.moving_box_scene(a.seed, a.n, a.width, a.height)
    ctx = gs.Context(0)
    # target frame rendered by the library at the target pose, boxes moved
    tv = gs.ViewBatch([tcam], a.n)
    tp = gs.Pipeline(ctx, tv, capacity=a.n * 128)
    gtt = gs.to_device(g_t)
    tp.forward(gs.gaussians_struct(gtt))
    over, n_t, _ = tp.check()
    assert not over
    tc = tp.img_color.clone()
    A = 1.0 - tp.img_T
    td = torch.where(A >= 0.5, tp.img_depth, torch.zeros_like(tp.img_depth)).contiguous()
    del tp, gtt
    # the iteration under test; choose the smallest power-of-two prefix rank
    # whose prefix lists let every tile saturate (exact result), full lists
    # when none does
    views = gs.ViewBatch([cam], a.n)
    gt = gs.to_device(g)
    gst = gs.gaussians_struct(gt)
    from paper_2602_21644_amd import optim, tune
    if a.max_rank >= 0:
        R = a.max_rank
        probe = gs.Pipeline(ctx, views, capacity=a.n * 64, max_rank=R)
        probe.forward(gst)
        over, n_inst, inc = probe.check()
        del probe
        assert not over and inc == 0, "the given prefix rank is not exact for this workload"
    else:
        R, n_inst = optim.choose_rank(ctx, views, gst, a.n)
    log(f"[bench] prefix rank {R} ({'full lists' if R == 0 else 'prefix lists'}), {n_inst} list entries")
    knobs = None
    for kv in filter(None, a.knobs.split(",")):
        name, val = kv.split("=")
        ctx.set_param(name.strip(), int(val))
    if not a.no_tune:
        import tempfile
        ent = tune.tune(ctx, views, gt, tc, td, cache=os.path.join(tempfile.gettempdir(), "gs_bench_tune.json"),
                        force=True)
        knobs = ent["knobs"]
        log(f"[bench] tuned knobs {knobs} ({ent['ms']:.4f} ms/iteration while tuning)")
    cap = int(n_inst * 1.25) + 4096
    pipe = gs.Pipeline(ctx, views, capacity=cap, max_rank=R)
    grads = gs.alloc_grads(a.n)
    pose = torch.zeros(6, device=dev)
    grs = gs.grads_struct(grads, pose)

    def step():
        pipe.forward_loss(gst, tc, td)
        pipe.backward(gst, grs)

    if a.profile_steps > 0:
        if a.copy_bytes > 0:
            src = torch.ones(a.copy_bytes // 4, dtype=torch.float32, device=dev)
            dst = torch.empty_like(src)
            torch.cuda.synchronize()
            dst.copy_(src)
            torch.cuda.synchronize()
            del src, dst
            log(f"[bench] calibration copy of {a.copy_bytes} bytes done")
        for _ in range(a.profile_steps):
            step()
        torch.cuda.synchronize()
        log("[bench] profile steps done")
        return

    for _ in range(max(1, a.warmup)):
        step()
    torch.cuda.synchronize()
    over, n_inst, inc = pipe.check()
    assert not over and n_inst > 0 and inc == 0
    # workload statistics for the byte model
    P = a.width * a.height
    nl = pipe.img_nlast.view(a.height, a.width)
    Hp, Wp = (a.height + 15) // 16 * 16, (a.width + 15) // 16 * 16
    nlp = torch.zeros(Hp, Wp, dtype=torch.int32, device=dev)
    nlp[:a.height, :a.width] = nl
    tile_max = nlp.view(Hp // 16, 16, Wp // 16, 16).amax(dim=(1, 3)).to(torch.int64)
    rb = ctx.get_param("render_batch")
    bb = ctx.get_param("bwd_batch")
    lens = (pipe.tile_start[1:].to(torch.int64) - pipe.tile_start[:-1].to(torch.int64)).view_as(tile_max)
    loaded_fwd = int(torch.minimum(lens, ((tile_max + rb) // rb) * rb).sum())
    loaded_bwd = int(((tile_max + bb - 1) // bb * bb).clamp(max=lens).sum())
    touched = int((grads["color"].abs().sum(0) > 0).sum())
    chunk = ctx.get_param("bin_chunk")
    # records the prefix path binned (the distinct ids of the lists)
    selected = int(torch.unique(pipe.ids[:n_inst]).numel()) if R > 0 else 0
    pairs = int(pipe.img_nlast.to(torch.int64).sum())  # (pixel, composited entry) pairs
    st = dict(n=a.n, instances=n_inst, pixels=P, tiles=views.tile_count, records=views.rec_count,
              nlim=views.rec_count, cm=views.tile_count * ((views.rec_count + chunk - 1) // chunk),
              loaded_fwd=loaded_fwd, loaded_bwd=loaded_bwd, touched=touched, selected=selected, pairs=pairs,
              fused_loss=True, copies=ctx.get_param("bwd_copies"))
    log(f"[bench] instances {n_inst}, touched Gaussians {touched}, entries loaded fwd {loaded_fwd}, "
        f"binning LDS limit {ctx.get_param('lds_limit')}")

    # timed region 1: graph replays (or eager steps with --no-graph)
    graph = None
    if not a.no_graph:
        s = torch.cuda.Stream()
        s.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(s):
            for _ in range(2):
                step()
        torch.cuda.current_stream().wait_stream(s)
        torch.cuda.synchronize()
        graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(graph):
            step()
        torch.cuda.synchronize()
        for _ in range(a.warmup):
            graph.replay()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t_wall = time.perf_counter()
    e0.record()
    for _ in range(a.steps):
        if graph is not None:
            graph.replay()
        else:
            step()
    e1.record()
    torch.cuda.synchronize()
    t_wall = time.perf_counter() - t_wall
    over, _, inc = pipe.check()
    assert not over and inc == 0, "timed steps were not exact"
    ms = e0.elapsed_time(e1) / a.steps
    log(f"[bench] {'graph' if graph is not None else 'eager'}: {ms:.4f} ms/step ({1000.0 / ms:.1f} iters/s)")
    # distribution of single steps (events around each), beside the mean above
    single = []
    for _ in range(a.steps):
        f0, f1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        f0.record()
        if graph is not None:
            graph.replay()
        else:
            step()
        f1.record()
        f1.synchronize()
        single.append(f0.elapsed_time(f1))
    p10, p50, p90 = (float(np.percentile(single, q)) for q in (10, 50, 90))

    # timed region 2: eager steps with per-kernel HIP events
    ctx.kernel_times()
    ctx.set_param("timing", 1)
    e2, e3 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e2.record()
    for _ in range(a.steps):
        step()
    e3.record()
    torch.cuda.synchronize()
    kt = ctx.kernel_times()
    ctx.set_param("timing", 0)
    eager_ms = e2.elapsed_time(e3) / a.steps
    per_step = {k: v[1] / a.steps for k, v in kt.items()}
    avg_launch_us = {k: 1000.0 * v[1] / v[0] for k, v in kt.items()}
    dom = max(per_step, key=per_step.get)
    dom_bytes = kernel_bytes(dom, st)
    dom_us = avg_launch_us[dom]
    base = dom.split("<")[0]
    if base in FLOPS_PER_PAIR:
        # compositing is bound by vector FP32 arithmetic, not by HBM
        flops = FLOPS_PER_PAIR[base] * pairs
        roof = {"bound": "alu", "kernel": dom, "achieved": round(flops / (dom_us * 1e-6) / 1e12, 3),
                "peak": FP32_VECTOR_PEAK_TFS, "unit": "TFLOP/s"}
        roof["frac"] = round(roof["achieved"] / FP32_VECTOR_PEAK_TFS, 4)
        roof["algorithmic_flops"] = flops
        roof["hbm_algorithmic_bytes"] = dom_bytes
    else:
        achieved = dom_bytes / (dom_us * 1e-6) / 1e9 if dom_bytes else None
        roof = {"bound": "hbm", "kernel": dom, "achieved": round(achieved, 1) if achieved else None,
                "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4) if achieved else None,
                "algorithmic_bytes": dom_bytes}
    roof["traffic"] = pmc_traffic(dom)
    roof["avg_launch_us"] = round(dom_us, 2)
    log("[bench] per-step kernel time (us): " + ", ".join(f"{k}={1000 * v:.1f}" for k, v in
                                                          sorted(per_step.items(), key=lambda x: -x[1])))
    # whole-iteration byte model
    total_bytes = 0
    for k, (n_l, _) in kt.items():
        b = kernel_bytes(k, st)
        if b:
            total_bytes += b * n_l / a.steps
    iter_frac = total_bytes / (ms * 1e-3) / (HBM_PEAK_GBS * 1e9)
    copy_gbs = copy_bandwidth_gbs(torch)
    cold_ms = cold_cache_ms(torch, graph, step, a.steps) if graph is not None else None
    atomics = atomic_roofline(ctx, gs, torch, st, avg_launch_us)

    # per-frame MP update at the same scale (reported beside, not in the step)
    mp_ms, mp_graph_ms = mp_update_ms(ctx, gs, synth, torch, a, g, cam, pipe, tc, td)

    out = {
        "metric": METRIC,
        "value": round(1000.0 / ms, 2),
        "unit": "iters/s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": round(ms, 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"{a.n} Gaussians, one {a.width}x{a.height} view, render+loss+backward to all "
                               f"Gaussian parameters and the pose", "n_gaussians": a.n, "width": a.width,
                   "height": a.height, "instances": n_inst, "prefix_rank": R, "knobs": knobs,
                   "composited_pairs": pairs, "parallelism": "single-gpu",
                   "timed": "hip graph replay" if graph is not None else "eager"},
        "roofline": roof,
        "roofline_iteration": {"bound": "hbm", "achieved": round(total_bytes / (ms * 1e-3) / 1e9, 1),
                               "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(iter_frac, 4),
                               "algorithmic_bytes": int(total_bytes)},
        "eager_ms_per_step": round(eager_ms, 4),
        "kernel_us_per_step": {k: round(1000 * v, 2) for k, v in sorted(per_step.items(), key=lambda x: -x[1])},
        "step_ms_p10_p50_p90": [round(p10, 4), round(p50, 4), round(p90, 4)],
        "cold_cache_ms_per_step": round(cold_ms, 5) if cold_ms else None,
        "atomic_roofline": atomics,
        "clocks": CLOCKS,
        "copy_gbs": round(copy_gbs, 1),
        "iteration_copy_frac": round(total_bytes / (ms * 1e-3) / (copy_gbs * 1e9), 4),
        "mp_update_ms": round(mp_ms, 4),
        "mp_update_graph_ms": round(mp_graph_ms, 4),
        "wall_s_timed": round(t_wall, 3),
    }
    if not a.no_extras:
        del pipe, grads
        torch.cuda.empty_cache()
        out["window_batch"] = window_batch(ctx, a, g, g_t)
        out["uneven_batch"] = uneven_batch(ctx)
        out["learned_mp"] = learned_mp(ctx, a, g, cam, tc, td)
        out["tracking"] = tracking_run(ctx)
        out["epipolar"] = epipolar_run(ctx)
        out["ablation"] = ablation_run(ctx)
    CLOCKS["end"] = rocm_smi_clocks()
    if not a.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(g, cam, tc.cpu().numpy().reshape(3, -1), td.cpu().numpy())
    print(json.dumps(out), flush=True)


def _graph_time(torch, step, reps=20):
    """ms per replay of a HIP graph of step()."""
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        step()
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        step()
    for _ in range(3):
        graph.replay()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        graph.replay()
    e1.record()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / reps


def _full_count(ctx, views, gst, n):
    """List entries of full lists (grows the probe capacity to the reported count)."""
    from paper_2602_21644_amd import gs
    cap = max(1 << 20, 16 * n)
    while True:
        probe = gs.Pipeline(ctx, views, capacity=cap, max_rank=0)
        probe.forward(gst)
        over, n_inst, _ = probe.check()
        del probe
        if not over:
            return n_inst
        cap = int(n_inst * 1.1) + (1 << 16)


def _render_targets(ctx, views, g_dev, full=False):
    """Observed frames of a view batch: colour and depth (0 where A < 0.5),
    rendered with exact prefix lists (or full lists)."""
    import torch
    from paper_2602_21644_amd import gs, optim
    n = int(g_dev["opacity_logit"].shape[0])
    gst = gs.gaussians_struct(g_dev)
    if full:
        R, n_inst = 0, _full_count(ctx, views, gst, n)
    else:
        R, n_inst = optim.choose_rank(ctx, views, gst, n)
    tp = gs.Pipeline(ctx, views, capacity=int(1.25 * n_inst) + (1 << 16), max_rank=R)
    tp.forward(gst)
    over, _, inc = tp.check()
    assert not over and inc == 0
    A = 1.0 - tp.img_T
    tc = tp.img_color.clone()
    td = torch.where(A >= 0.5, tp.img_depth, torch.zeros_like(A)).contiguous()
    return tc, td


def _batch_step(ctx, views, g_dev, tc, td, full=False):
    """Exact prefix rank (or full lists), pipeline and step() of render + loss
    + backward."""
    import torch
    from paper_2602_21644_amd import gs, optim
    n = int(g_dev["opacity_logit"].shape[0])
    gst = gs.gaussians_struct(g_dev)
    if full:
        R, n_inst = 0, _full_count(ctx, views, gst, n)
    else:
        R, n_inst = optim.choose_rank(ctx, views, gst, n)
    pipe = gs.Pipeline(ctx, views, capacity=int(1.25 * n_inst) + (1 << 16), max_rank=R)
    grads = gs.alloc_grads(n)
    pose = torch.zeros(6 * views.V, device="cuda")
    grs = gs.grads_struct(grads, pose)

    def step():
        pipe.forward_loss(gst, tc, td)
        pipe.backward(gst, grs)

    # the graph replays write these: they live as long as the step
    step.outputs = (grads, pose)
    return pipe, step, R, n_inst


def tracking_run(ctx, n=200_000, W=640, H=480, iters=100):
    """Pose-only tracking (the tracking configuration: 200k Gaussians, one
    640x480 view, 100 iterations of render, loss, pose gradient, Adam on the
    twist and retraction, replayed from one captured hip graph) from a pose
    0.5 deg and 1 cm off the one the target was rendered at."""
    import torch
    from paper_2602_21644_amd import gs, optim, synth
    g, cam, tcam, g_t, sl = synth.moving_box_scene(2, n, W, H)
    gd = gs.to_device(g)
    tv = gs.ViewBatch([cam], n)
    tp = gs.Pipeline(ctx, tv, capacity=n * 128)
    tp.forward(gs.gaussians_struct(gd))
    over, _, _ = tp.check()
    assert not over
    tc = tp.img_color.clone()
    td = torch.where(1.0 - tp.img_T >= 0.5, tp.img_depth, torch.zeros_like(tp.img_depth)).contiguous()
    del tp
    T0 = synth.perturbed_pose(synth.rng_for(20), deg=0.5, trans=0.01, base=cam["T_cw"])
    trk = optim.Tracker(ctx, gd, synth.camera(W, H, T0))
    trk.run(tc, td, iters=2, T_init=T0)  # captures the graph
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    T, loss, exact = trk.run(tc, td, iters=iters, T_init=T0)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / iters
    Tt = np.asarray(cam["T_cw"], np.float64)
    Rr = np.asarray(T, np.float64)[:, :3] @ Tt[:, :3].T
    ang = float(np.degrees(np.arccos(np.clip((np.trace(Rr) - 1) / 2, -1.0, 1.0))))
    # camera centres c = -R^T t
    c_est = -np.asarray(T, np.float64)[:, :3].T @ np.asarray(T, np.float64)[:, 3]
    c_true = -Tt[:, :3].T @ Tt[:, 3]
    dist = float(np.linalg.norm(c_est - c_true))
    log(f"[bench] tracking: {ms:.4f} ms per iteration, final error {ang:.4f} deg {dist * 1e3:.3f} mm")
    return {"n_gaussians": n, "width": W, "height": H, "iterations": iters, "prefix_rank": trk.rank,
            "ms_per_iteration": round(ms, 4), "iters_per_s": round(1000.0 / ms, 1),
            "start_error": [0.5, 10.0], "final_error_deg_mm": [round(ang, 4), round(dist * 1e3, 3)],
            "exact": bool(exact)}


def ablation_run(ctx):
    """The synthetic analogue of the temporal-MP, MP-fusion and scheduling
    ablations: 40 frames of a 100k-Gaussian moving-box sequence at 320x240
    through tracking, epipolar verification, the scheduler and the MP update,
    once per variant (structure of those tables, not their numbers)."""
    from paper_2602_21644_amd import sequence
    rows = sequence.ablation(ctx, seed=31, n=100_000, W=320, H=240, frames=40)
    for r in rows:
        log(f"[bench] ablation {r['variant']}: refreshes {r['refreshes']}, flips {r['flip_ratio_pct']}%, "
            f"MP error {r['mp_abs_error']}, label error {r['label_error_pct']}%, ATE {r['ate_cm']} cm")
    return {"sequence": "100000 Gaussians, 320x240, 40 frames, 3 moving boxes (8% of the Gaussians)",
            "rows": rows}


def epipolar_run(ctx, n=1_000_000, W=640, H=480, n_cand=50000):
    """Epipolar verification and static recovery (Eq. (18)-(19)) of 50k
    candidate Gaussians of a 1M-Gaussian map, 4-28 synthetic matches each,
    between two keyframes 5 frames apart: median of 20 calls (HIP events),
    and the select kernel's duration against its algorithmic HBM bytes."""
    import torch
    from paper_2602_21644_amd import gs, synth
    c = synth.epipolar_case(7, n, W, H, n_cand, per=(4, 28))
    views = gs.ViewBatch([c["cam1"], c["cam2"]], n)
    dev = lambda x: torch.from_numpy(np.ascontiguousarray(x)).cuda()
    p1, p2, ids, seg = dev(c["p1"]), dev(c["p2"]), dev(c["ids"]), dev(c["seg"])
    m, K = int(c["p1"].shape[1]), int(c["ids"].size)
    mp0 = dev(c["mp"])
    mp = mp0.clone()
    d = torch.empty(m, device="cuda")
    dbar = torch.empty(K, device="cuda")
    state = torch.empty(K, dtype=torch.uint8, device="cuda")

    def call():
        gs.gs_epipolar_verify(ctx, views.s, 0, 1, p1, p2, ids, seg, mp, d, dbar, state)

    times = []
    for i in range(22):
        mp.copy_(mp0)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        call()
        e1.record()
        e1.synchronize()
        if i >= 2:
            times.append(e0.elapsed_time(e1))
    ctx.kernel_times()
    ctx.set_param("timing", 1)
    for _ in range(10):
        call()
    torch.cuda.synchronize()
    kt = ctx.kernel_times()
    ctx.set_param("timing", 0)
    mp.copy_(mp0)
    call()
    torch.cuda.synchronize()
    sel_us = 1000.0 * kt["epi_select_kernel"][1] / kt["epi_select_kernel"][0]
    nbytes = m * 20 + K * 21  # p1, p2 read and d written per match; id, range, mp, dbar, state per candidate
    ms = float(np.median(times))
    restored = int((state == gs.GS_EPI_RESTORED).sum())
    log(f"[bench] epipolar: {K} candidates, {m} matches, {ms:.4f} ms per call, select kernel {sel_us:.1f} us, "
        f"{restored} restored")
    return {"n_gaussians": n, "candidates": K, "matches": m, "ms_per_call": round(ms, 4),
            "matches_per_s": round(m / (ms * 1e-3), 1), "select_kernel_us": round(sel_us, 2),
            "select_hbm_gbs": round(nbytes / (sel_us * 1e-6) / 1e9, 1),
            "select_hbm_frac": round(nbytes / (sel_us * 1e-6) / 1e9 / HBM_PEAK_GBS, 4), "restored": restored}


def window_batch(ctx, a, g, g_t):
    """8 keyframes (every 5th frame of the camera walk) of the 1M scene
    rendered and back-propagated in one call sequence, timed as a graph."""
    import torch
    from paper_2602_21644_amd import gs, synth
    cams = synth.window_cameras(a.seed + 1, 8, a.width, a.height, spacing=5)
    views = gs.ViewBatch(cams, a.n)
    tc, td = _render_targets(ctx, views, gs.to_device(g_t))
    torch.cuda.empty_cache()
    gd = gs.to_device(g)
    pipe, step, R, n_inst = _batch_step(ctx, views, gd, tc, td)
    ms = _graph_time(torch, step)
    over, _, inc = pipe.check()
    assert not over and inc == 0
    log(f"[bench] 8-view window: {ms:.3f} ms per batched iteration")
    return {"views": 8, "n_gaussians": a.n, "width": a.width, "height": a.height, "prefix_rank": R,
            "instances": n_inst, "ms_per_step": round(ms, 4), "frame_iters_per_s": round(8000.0 / ms, 1)}


def uneven_batch(ctx):
    """4 scenes (50k at 320x240, 150k at 640x480, 300k at 960x540, 600k at
    1280x720; 1-5 moving boxes each) x 8 consecutive frames = 32 views
    rendered and back-propagated in one captured graph."""
    import torch
    from paper_2602_21644_amd import gs, synth
    specs = [(50_000, 320, 240), (150_000, 640, 480), (300_000, 960, 540), (600_000, 1280, 720)]
    rng = np.random.default_rng(400)
    scenes, targets, cams, vs = [], [], [], []
    for i, (n, W, H) in enumerate(specs):
        # the scene extends 15% beyond the first view on every side: the
        # following frames look past its edges
        g, cam, tcam, g_t, sl = synth.moving_box_scene(400 + i, n, W, H, n_boxes=int(rng.integers(1, 6)),
                                                       margin=0.15)
        scenes.append(g)
        targets.append(g_t)
        cams += synth.window_cameras(410 + i, 8, W, H, spacing=1)
        vs += [i] * 8
    begin = np.concatenate([[0], np.cumsum([s[0] for s in specs])]).tolist()
    n_all = int(begin[-1])
    views = gs.ViewBatch(cams, n_all, view_scene=vs, scene_begin=begin)
    tc, td = _render_targets(ctx, views, gs.to_device(synth.concat_gaussians(targets)))
    torch.cuda.empty_cache()
    gd = gs.to_device(synth.concat_gaussians(scenes))
    pipe, step, R, n_inst = _batch_step(ctx, views, gd, tc, td)
    ms = _graph_time(torch, step)
    over, _, inc = pipe.check()
    assert not over and inc == 0
    log(f"[bench] uneven 32-frame batch: {ms:.3f} ms per graph replay")
    return {"frames": 32, "scenes": [f"{n}@{W}x{H}" for n, W, H in specs], "prefix_rank": R, "instances": n_inst,
            "ms_per_step": round(ms, 4), "frames_per_s": round(32000.0 / ms, 1)}


def learned_mp(ctx, a, g, cam, tc, td):
    """The learned-MP protocol at the headline size (1M Gaussians, 640x480):
    the surrogate trained on the plain cue's M_p of 2,000 frames (sequences
    1000-1019, 100 frames each, 1-5 moving boxes in front of a static layer),
    then sequences 5000-5004 (100 frames each) tracked and MP-updated at the
    tracked pose with the plain cue and with the surrogate under its fallback
    rule. MP abs error, label error, pose error and the MP source's time per
    frame for both forms."""
    import time as _t
    from paper_2602_21644_amd import mp_learn
    t0 = _t.perf_counter()
    sur, used, first, last = mp_learn.train_c5(ctx, n=a.n, width=a.width, height=a.height)
    t_train = _t.perf_counter() - t0
    res = mp_learn.evaluate_c5(ctx, sur, n=a.n, width=a.width, height=a.height)
    log(f"[bench] learned MP: trained on {used} frames in {t_train:.1f} s (BCE {first:.4f} -> {last:.4f}); "
        f"plain {res['plain']}; learned {res['learned']}")
    return {"protocol": "train 1000-1019 x 100 frames, test 5000-5004 x 100 frames, 1M Gaussians at 640x480, "
                        "tracking 10 iterations per frame from the previous estimate",
            "train_frames": used, "train_s": round(t_train, 1), "bce_first_last": [round(first, 4), round(last, 4)],
            **{f"{k}_{form}": v for form in ("plain", "learned") for k, v in res[form].items()}}


def kernel_source_hash(kernel):
    """sha256 of the HIP source that defines `kernel` (None when unknown)."""
    import hashlib
    src = {"render_bwd_kernel": "k_render.hip", "render_fwd_kernel": "k_render.hip",
           "project_kernel": "k_project.hip"}.get(kernel.split("<")[0])
    if not src:
        return None
    path = os.path.join(ROOT, "paper_2602_21644_amd", "csrc", src)
    with open(path, "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()


def pmc_traffic(kernel):
    """HBM bytes per launch from the recorded counters, None when the kernel
    changed since they were taken."""
    rec = PMC_TRAFFIC.get(kernel)
    if not rec or rec["sha256"] != kernel_source_hash(kernel):
        return None
    return int(1024 * (rec["fetch_kib"] * PMC_SCALE["fetch"] + rec["write_kib"] * PMC_SCALE["write"]))


def rocm_smi_clocks():
    """Current clocks from rocm-smi (None when the tool is not there)."""
    import subprocess
    try:
        r = subprocess.run(["rocm-smi", "--showclocks", "--json"], capture_output=True, text=True, timeout=20)
        d = json.loads(r.stdout)
    except Exception as exc:  # no rocm-smi, or no JSON
        return {"error": type(exc).__name__}
    out = {}
    for card, vals in d.items():
        if isinstance(vals, dict):
            out[card] = {k: v for k, v in vals.items() if "clock" in k.lower() or "freq" in k.lower()}
    return out


CLOCKS = {}


def cold_cache_ms(torch, graph, step, steps, flush_bytes=512 << 20):
    """Median ms of single graph replays, each after a 512 MiB device write
    that evicts the working set from the L2s and the Infinity Cache (the
    write itself is outside the timed events)."""
    junk = torch.empty(flush_bytes // 4, dtype=torch.float32, device="cuda")
    ts = []
    for i in range(min(steps, 50)):
        junk.fill_(float(i))
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        graph.replay()
        e1.record()
        e1.synchronize()
        ts.append(e0.elapsed_time(e1))
    del junk
    return float(np.median(ts))


def atomic_roofline(ctx, gs, torch, st, avg_launch_us):
    """The backward's float atomics against gs_measure_atomics on the same
    pattern: the touched records, ten components each, one atomic per staged
    entry and component (an upper bound on the kernel's count), in the tuned
    number of per-XCD copies."""
    n_rec = max(int(st["touched"]), 1)
    n_ops = int(st["loaded_bwd"]) * 10
    copies = int(st.get("copies", 1))
    acc = torch.zeros(copies * n_rec * 10, device="cuda")
    gs.gs_measure_atomics(ctx, acc, n_rec, n_ops, copies)
    torch.cuda.synchronize()
    ts = []
    for _ in range(20):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        gs.gs_measure_atomics(ctx, acc, n_rec, n_ops, copies)
        e1.record()
        e1.synchronize()
        ts.append(e0.elapsed_time(e1))
    ms = float(np.median(ts))
    rate = n_ops / (ms * 1e-3)
    bwd = [v for k, v in avg_launch_us.items() if k.startswith("render_bwd_kernel")]
    return {"records": n_rec, "atomics": n_ops, "copies": copies, "ms": round(ms, 4), "atomics_per_s": round(rate, 1),
            "backward_us": round(bwd[0], 2) if bwd else None,
            "atomics_share_of_backward": round(1000.0 * ms / bwd[0], 4) if bwd else None}


def oracle_timing():
    """The FP64 oracle's forward + loss + backward of one iteration, median of
    3 runs (1 run single-threaded at 1M Gaussians), on all host threads and on
    one: C1 (2,000 Gaussians, 64x48), C2 (200k, 640x480, pose-only tracking
    case), the metric workload (1M, 640x480) and one 640x480 view of the
    8-keyframe window over the same 1M scene."""
    import platform
    import oracle
    from paper_2602_21644_amd import synth

    def one(g, cam, tc, td):
        t0 = time.perf_counter()
        pr = oracle.project(g, cam)
        im = oracle.render(pr, g, cam)
        L = oracle.loss(im, tc, td)
        g2d = oracle.render_backward(pr, g, cam, L["dC"], L["dD"], L["dM"], L["dT"])
        oracle.project_backward(g, cam, g2d)
        return time.perf_counter() - t0

    def target(g_t, tcam):
        im = oracle.render(oracle.project(g_t, tcam), g_t, tcam)
        return im["C"].astype(np.float32), np.where(1 - im["T"] >= 0.5, im["D"], 0.0).astype(np.float32)

    cases = {}
    g, cam, tcam = synth.tiny_scene(seed=1)
    cases["C1"] = (g, cam) + target(g, tcam)
    g, cam, tcam, g_t, _ = synth.moving_box_scene(2, 200_000, 640, 480)
    cases["C2"] = (g, cam) + target(g_t, tcam)
    g, cam, tcam, g_t, _ = synth.moving_box_scene(11, 1_000_000, 640, 480)
    cases["metric"] = (g, cam) + target(g_t, tcam)
    wc = synth.window_cameras(12, 8, 640, 480, spacing=5)
    cases["C3_view"] = (g, wc[3]) + target(g_t, wc[3])
    full = oracle.num_threads()
    cpu = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    cpu = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    out = {"cpu_model": cpu, "nproc": os.cpu_count(), "omp_threads": full, "machine": platform.machine(),
           "rows": {}}
    for name, (gg, cc, tc, td) in cases.items():
        row = {}
        for threads in (full, 1):
            oracle.set_threads(threads)
            runs = 1 if threads == 1 and synth.n_gaussians(gg) >= 1_000_000 else 3
            row[f"s_{threads}t"] = round(float(np.median([one(gg, cc, tc, td) for _ in range(runs)])), 4)
            row[f"runs_{threads}t"] = runs
        oracle.set_threads(full)
        row["n_gaussians"] = synth.n_gaussians(gg)
        row["pixels"] = cc["width"] * cc["height"]
        out["rows"][name] = row
        log(f"[oracle] {name}: {row}")
    return out


def copy_bandwidth_gbs(torch, nbytes=256 << 20, reps=10):
    """Device-to-device copy bandwidth (read + write bytes per second) of a
    256 MiB buffer, median of `reps` copies: the stream rate the byte model is
    also held against."""
    src = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    dst.copy_(src)
    torch.cuda.synchronize()
    ts = []
    for _ in range(reps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        dst.copy_(src)
        e1.record()
        e1.synchronize()
        ts.append(e0.elapsed_time(e1))
    del src, dst
    return 2 * nbytes / (float(np.median(ts)) * 1e-3) / 1e9


def mp_update_ms(ctx, gs, synth, torch, a, g, cam, pipe, tc, td):
    """Times gs_mp_update on the rendered frame (3 instance masks from the
    boxes' screen rectangles): median of 20 eager calls, and median of 20
    replays of the call captured in a hip graph."""
    n = a.n
    views = gs.ViewBatch([cam], n)
    M = views.rec_count
    P = a.width * a.height
    # projected means are needed: project once more with the planar outputs
    m2d = torch.empty(2 * M, device="cuda")
    proj = gs.Proj()
    proj.m = M
    proj.rec, proj.rect, proj.depth_key, proj.mean2d = pipe.proj.rec, pipe.proj.rect, pipe.proj.depth_key, gs.ptr(m2d)
    gs.gs_project(ctx, views.s, gs.gaussians_struct(gs.to_device(g)), proj)
    inst = torch.zeros(P, dtype=torch.int32, device="cuda")
    inst.view(a.height, a.width)[100:220, 200:320] = 1
    inst.view(a.height, a.width)[300:400, 400:520] = 2
    inst.view(a.height, a.width)[50:150, 450:600] = 3
    prior = torch.tensor([0.05, 0.9, 0.9, 0.9], device="cuda")
    conf = torch.tensor([0.1, 0.9, 0.9, 0.9], device="cuda")
    frame = gs.MPFrame(gs.ptr(inst), 3, gs.ptr(prior), gs.ptr(conf), 1, None)
    pp = gs.MPParams(*[gs.MP_DEFAULTS[k] for k in gs.MP_PARAM_NAMES], 0, 0)
    mp = torch.rand(n, device="cuda")
    Ut = torch.zeros(n, device="cuda")
    al = torch.zeros(n, device="cuda")
    dyn = torch.zeros(n, dtype=torch.uint8, device="cuda")
    pr = torch.zeros(n, dtype=torch.uint8, device="cuda")
    stats = torch.zeros(8, device="cuda")
    out = gs.MPOut(gs.ptr(Ut), gs.ptr(al), gs.ptr(dyn), gs.ptr(pr), None, None, gs.ptr(stats))
    ws = torch.zeros(gs.gs_workspace_size(ctx, views.s, gs.GS_OP_MP_UPDATE), dtype=torch.uint8, device="cuda")
    tgt = gs.Target(gs.ptr(tc), gs.ptr(td))
    times = []
    for i in range(22):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        gs.gs_mp_update(ctx, views.s, proj, pipe.img, tgt, frame, pp, mp, out, ws)
        e1.record()
        torch.cuda.synchronize()
        if i >= 2:
            times.append(e0.elapsed_time(e1))
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        gs.gs_mp_update(ctx, views.s, proj, pipe.img, tgt, frame, pp, mp, out, ws)
    torch.cuda.current_stream().wait_stream(side)
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        gs.gs_mp_update(ctx, views.s, proj, pipe.img, tgt, frame, pp, mp, out, ws)
    gtimes = []
    for i in range(22):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        graph.replay()
        e1.record()
        torch.cuda.synchronize()
        if i >= 2:
            gtimes.append(e0.elapsed_time(e1))
    return float(np.median(times)), float(np.median(gtimes))


def cpu_baseline(g, cam, tc, td, budget_s=10.0):
    """The FP64 oracle on the host: whole iterations of the step (projection,
    render of every pixel, loss, render adjoint, projection adjoint) repeated
    until about `budget_s` seconds of work, at least one."""
    import oracle
    n_it = 0
    t0 = time.perf_counter()
    while True:
        pr = oracle.project(g, cam)
        im = oracle.render(pr, g, cam)
        L = oracle.loss(im, tc, td)
        g2d = oracle.render_backward(pr, g, cam, L["dC"], L["dD"], L["dM"], L["dT"])
        oracle.project_backward(g, cam, g2d)
        n_it += 1
        el = time.perf_counter() - t0
        if el >= budget_s:
            break
    return {"value": round(n_it / el, 5), "unit": "iters/s", "cores": oracle.num_threads(), "kind": "oracle",
            "sample": f"{n_it} whole iterations of the step (every pixel, every Gaussian) in {el:.1f} s"}


if __name__ == "__main__":
    main()
