#!/usr/bin/env python3
"""Throughput of the differentiable Gaussian rasteriser on one MI355X.

Workload (the tracking configuration): a synthetic 4x4x3 m room with 200k
Gaussians, 8 camera poses along a smooth trajectory, 640x480, f = 525.
One step = forward + combined L1 loss + backward to every Gaussian
parameter and to the poses, for all 8 views.  Targets are renders at the
true poses; the renderer is evaluated at poses 2 deg / 2 cm away.  The tile
shape is the one the library's autotuner picks for this input.

Reported (one JSON line):
  value         views/s of the batched path (all views in one launch
                sequence), full gradients, inputs resident in HBM
  plain         the same views one launch sequence each, the pair capacity
                checked once after the timed loop (like the batched path);
                plain_synced checks it after every view (one host
                synchronisation per view)
  pose_only     batched, gradients to the poses only (tracking mode)
  graph         batched, replayed from a captured HIP graph
  autograd      batched through the torch autograd function render_loss
                (forward + backward, no host synchronisation)
  stages_ms     per-stage averages from HIP events on the library's stream
  roofline      the dominant kernel (the backward blend) against the FP32
                VALU peak, from counted work and the per-pair operation
                counts of the roofline model (transcendentals at quarter rate)
  cpu_baseline  the FP64 oracle on the host, at one thread and at every core
  pose_fd       FP32 central-difference check of the pose gradients on 64
                Gaussians of the large anisotropic scene
  uneven_batch  the 1M-Gaussian room with 32 poses at four resolutions, and
                the 3M-Gaussian multi-room scene with 16 views at 1200x680:
                autotuned tile, one captured fwd+bwd per replay
  next_rows     the steps around the path: the 40-iteration tracking loop
                of one view as one graph replay, the mapping loop (10
                iterations per graph replay), the mapping Adam step (HBM
                roofline), new Gaussians from a 640x480 RGB-D frame, and the
                batched step with isotropic Gaussians
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "fwd+bwd views/sec at 640×480, 200k Gaussians (batched vs plain); pose-grad FD err"

# MI355X: 256 CUs x 4 SIMD x 16 lanes x 2.4 GHz = FP32 VALU lane-operation slots per second
# (one non-packed FP32 instruction per lane per slot; 157.3 TFLOP/s counts packed FMA as 4 FLOP)
VALU_PEAK_LANE_OPS = 256 * 4 * 16 * 2.4e9
HBM_PEAK_GBS = 8000.0
COPY_BYTES = 256 << 20   # the calibration copy reads and writes this many bytes
# Roofline model: algorithmic FP32 lane-operation slots per (pixel, Gaussian)
# pair of the blend; a transcendental instruction (exp2, reciprocal) runs at
# quarter rate and counts 4 slots.
TRANS_SLOTS = 4
C_ALPHA = 9 + TRANS_SLOTS    # offset, quadratic form, opacity product, clamp, 1/255 test; one exp2
C_BLEND = 8                  # transmittance update, stop test, weight, five channel sums
C_GRAD = 40 + TRANS_SLOTS    # dL/dalpha, behind-sum update, ten partials; one reciprocal
# the per-pair counts the kernels were written against (reported as a second figure)
IMPL_C_ALPHA, IMPL_C_BLEND, IMPL_C_GRAD = 17, 10, 45
TRAFFIC_PROFILE = os.path.join("profiles", "blend_bwd_traffic.json")


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--n", type=int, default=200_000)
    ap.add_argument("--views", type=int, default=8)
    ap.add_argument("--tile", default="auto", help="WxH, or auto (the library's autotuner)")
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle CPU baseline")
    ap.add_argument("--no-plain", action="store_true")
    ap.add_argument("--no-graph", action="store_true")
    ap.add_argument("--cpu-views", type=int, default=8, help="views in the oracle's all-core sample")
    ap.add_argument("--no-next", action="store_true", help="skip the tracking / mapping / densify / isotropic legs")
    ap.add_argument("--no-uneven", action="store_true", help="skip the 32-view and 3M-Gaussian legs")
    ap.add_argument("--no-fd", action="store_true", help="skip the pose finite-difference check")
    ap.add_argument("--profile-steps", type=int, default=0,
                    help="only run this many batched steps (for a profiler) and print nothing else")
    ap.add_argument("--profile-workload", default="tracking", choices=["tracking", "frame", "uneven", "large"],
                    help="with --profile-steps: the 8-view tracking-room step, one 640x480 view's 40-iteration "
                         "tracking loop (run profile-steps times, eagerly), the 32-view uneven batch or the 3M scene")
    ap.add_argument("--deterministic", action="store_true",
                    help="with --profile-steps: the fixed-order backward (GSR_DETERMINISTIC)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="with --profile-steps: also copy 256 MiB device to device, the reference for the "
                         "HBM byte counters")
    return ap.parse_args()


def _t32(a, dev):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a, np.float32)).to(dev)


def _params(raster, G, dev):
    return raster.GaussianParams(_t32(G.means, dev), _t32(G.quats, dev), _t32(G.log_scales, dev),
                                 _t32(G.opacity_logits, dev), _t32(G.rgb, dev))


def timed(fn, steps, warmup):
    """Average ms per call of fn over `steps` calls after `warmup`, from HIP
    events on the current stream."""
    import torch
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    a = torch.cuda.Event(enable_timing=True)
    b = torch.cuda.Event(enable_timing=True)
    a.record()
    for _ in range(steps):
        fn()
    b.record()
    torch.cuda.synchronize()
    return a.elapsed_time(b) / steps


def roofline(work: dict, bwd_ms: float, traffic=None, traffic_source=None) -> dict:
    """The backward blend against the FP32 VALU peak.  Strict: E' (c_alpha +
    c_grad) over the contributions only; tile list: E c_alpha + E' c_grad
    over every evaluated (pixel, entry) pair.  The reduction over a wave's
    pixels (R reduced (wave, entry) pairs) is not counted as algorithmic work."""
    E, Ec, R = work["eval_bwd"], work["contrib_bwd"], work["reduce_bwd"]
    strict = Ec * (C_ALPHA + C_GRAD)
    lst = E * C_ALPHA + Ec * C_GRAD
    s = bwd_ms * 1e-3
    peak = VALU_PEAK_LANE_OPS
    impl_strict = Ec * (IMPL_C_ALPHA + IMPL_C_GRAD)
    impl_list = impl_strict + (E - Ec) * IMPL_C_ALPHA
    return {"bound": "alu", "kernel": "k_blend_bwd", "achieved": strict / s / 1e12, "peak": peak / 1e12,
            "unit": "T lane-op/s", "frac": strict / s / peak, "frac_list": lst / s / peak,
            "traffic": traffic, "traffic_source": traffic_source,
            "avg_launch_ms": bwd_ms, "duration_source": "HIP events around the kernel's launch on the library's "
                                                        "stream, averaged over the timed region",
            "ops_per_launch": strict, "list_ops_per_launch": lst, "work": {"E": E, "E_contrib": Ec, "R": R},
            "model": {"c_alpha": C_ALPHA, "c_blend": C_BLEND, "c_grad": C_GRAD, "transcendental_slots": TRANS_SLOTS,
                      "frac": "E_contrib (c_alpha + c_grad) / t / peak",
                      "frac_list": "(E c_alpha + E_contrib c_grad) / t / peak"},
            "impl_model": {"c_alpha": IMPL_C_ALPHA, "c_blend": IMPL_C_BLEND, "c_grad": IMPL_C_GRAD,
                           "frac": impl_strict / s / peak, "frac_list": impl_list / s / peak}}


def main():
    args = parse()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path "
              "(run with --gpus 1)", file=sys.stderr)
        sys.exit(2)
    import torch
    from paper_2408_05635_amd import raster, scenes

    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    if args.profile_steps and args.profile_workload in ("uneven", "large"):
        profile_uneven(args, raster, scenes, dev)
        return
    w = scenes.config2(n_views=args.views, n=args.n)
    g = _params(raster, w.gaussians, dev)
    q, t = _t32(w.views.quat, dev), _t32(w.views.trans, dev)
    qt, tt = _t32(w.target_views.quat, dev), _t32(w.target_views.trans, dev)
    cams = w.views.cams
    V = len(cams)
    P = sum(c.width * c.height for c in cams)
    rast = raster.Rasterizer(0)
    opts = raster.RenderOptions(tile=(16, 16), **w.weights)

    # targets: renders at the true poses (inputs of the workload)
    trgb, tdep, tsil, _ = rast.forward(g, qt, tt, cams, opts)
    targets = dict(rgb=trgb, depth=tdep, sil=tsil)
    tuned = None
    if args.tile == "auto":
        tile, ms_tune = rast.autotune(g, q, t, cams, targets, opts, reps=5)
        tuned = {"tile": list(tile), "ms_per_call": ms_tune}
        print(f"[bench] autotuned tile {tile[0]}x{tile[1]} ({ms_tune:.3f} ms per call)", file=sys.stderr, flush=True)
    else:
        tile = tuple(int(x) for x in args.tile.split("x"))
    tw, th = tile
    opts = raster.RenderOptions(tile=(tw, th), deterministic=bool(args.profile_steps and args.deterministic),
                                **w.weights)
    if args.profile_steps and args.profile_workload == "frame":
        profile_frame(args, rast, raster, w, g, q, t, targets, opts)
        return
    out = rast.render_loss_grad(g, q, t, cams, targets, opts, check=True)   # sizes the pair capacity
    torch.cuda.synchronize()
    M, K, ovf = rast.last_counters
    assert not ovf

    def batched_step(o=opts, dst=out):
        rast.render_loss_grad(g, q, t, cams, targets, o, check=False, out=dst)

    if args.profile_steps:
        for _ in range(args.profile_steps):
            batched_step()
        torch.cuda.synchronize()
        if args.copy_calibration:
            src = torch.empty(COPY_BYTES // 4, dtype=torch.float32, device=dev).fill_(1.0)
            dst = torch.empty_like(src)
            torch.cuda.synchronize()
            dst.copy_(src)
            torch.cuda.synchronize()
        print(json.dumps({"profile_steps": args.profile_steps, "pairs": K, "visible": M, "tile": [tw, th]}),
              flush=True)
        return

    # batched, full gradients; per-stage HIP events recorded over the same region
    for _ in range(args.warmup):
        batched_step()
    torch.cuda.synchronize()
    rast.read_timing()
    rast.set_timing(True)
    ms_batched = timed(batched_step, args.steps, 0)
    rast.set_timing(False)
    stages = rast.read_timing()
    assert not rast.check_overflow(), "pair capacity overflowed during the timed region"
    print(f"[bench] batched {ms_batched:.3f} ms/step ({V * 1000.0 / ms_batched:.1f} views/s)", file=sys.stderr,
          flush=True)
    stage_ms = {k: (v[0] / v[1] if v[1] else 0.0) for k, v in stages.items()}

    # pose-only (tracking) mode
    o_pose = raster.RenderOptions(**{**opts.__dict__, "gauss_grads": False})
    out_pose = rast.alloc_outputs(g, V, P, o_pose)
    rast.render_loss_grad(g, q, t, cams, targets, o_pose, check=True, out=out_pose)
    ms_pose = timed(lambda: batched_step(o_pose, out_pose), args.steps, args.warmup)
    assert not rast.check_overflow()
    print(f"[bench] pose-only {ms_pose:.3f} ms/step", file=sys.stderr, flush=True)

    # plain: one view per launch sequence
    plain = plain_synced = None
    if not args.no_plain:
        rast1 = raster.Rasterizer(0)   # its own workspace, sized for one view
        Pv = P // V
        singles = []
        for v in range(V):
            tg_v = dict(rgb=trgb[3 * Pv * v:3 * Pv * (v + 1)], depth=tdep[Pv * v:Pv * (v + 1)],
                        sil=tsil[Pv * v:Pv * (v + 1)])
            ov = rast1.alloc_outputs(g, 1, Pv, opts)
            qv, tv = q[v:v + 1].contiguous(), t[v:v + 1].contiguous()
            rast1.render_loss_grad(g, qv, tv, [cams[v]], tg_v, opts, check=True, out=ov)   # sizes the capacity
            singles.append((qv, tv, [cams[v]], tg_v, ov))

        def plain_step(check):
            for (qv, tv, cv, tgv, ov) in singles:
                rast1.render_loss_grad(g, qv, tv, cv, tgv, opts, check=check, out=ov)

        ms_plain = timed(lambda: plain_step(False), args.steps, args.warmup)
        assert not rast1.check_overflow()
        ms_plain_sync = timed(lambda: plain_step(True), args.steps, args.warmup)
        plain = dict(value=V * 1000.0 / ms_plain, ms_per_step=ms_plain,
                     protocol="one launch sequence per view; pair capacity checked once after the timed loop")
        plain_synced = dict(value=V * 1000.0 / ms_plain_sync, ms_per_step=ms_plain_sync,
                            protocol="one launch sequence per view, each followed by its pair-count readback")
        print(f"[bench] plain {ms_plain:.3f} ms/step, with a readback per view {ms_plain_sync:.3f}",
              file=sys.stderr, flush=True)

    # batched, replayed from a HIP graph captured by the library (gsr_graph_capture)
    graph = None
    if not args.no_graph:
        s = torch.cuda.Stream()
        s.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(s):
            gid, gout = rast.capture_graph(g, q, t, cams, targets, opts)
            ms_graph = timed(lambda: rast.launch_graph(gid), args.steps, args.warmup)
            s.synchronize()
            assert not rast.check_overflow()
            same = all(torch.equal(gout[k], out[k]) for k in ("rgb", "depth", "sil", "loss"))
            gdiff = max(float(((gout[k].double() - out[k].double()).abs().max() /
                               out[k].double().abs().max()).item()) for k in ("g_means", "dq_t"))
            rast.destroy_graph(gid)
        torch.cuda.synchronize()
        graph = dict(value=V * 1000.0 / ms_graph, ms_per_step=ms_graph, images_and_loss_bitwise_equal_to_eager=bool(same),
                     gradients_max_rel_diff_to_eager=gdiff)
        print(f"[bench] graph {ms_graph:.3f} ms/step", file=sys.stderr, flush=True)

    # the same step with GSR_DETERMINISTIC: a row per (tile, entry) summed per
    # record in a fixed order, instead of the default's float atomics
    o_det = raster.RenderOptions(**{**opts.__dict__, "deterministic": True})
    out_det = rast.alloc_outputs(g, V, P, o_det)
    rast.render_loss_grad(g, q, t, cams, targets, o_det, check=True, out=out_det)
    for _ in range(args.warmup):
        batched_step(o_det, out_det)
    torch.cuda.synchronize()
    rast.read_timing()
    rast.set_timing(True)
    ms_det = timed(lambda: batched_step(o_det, out_det), args.steps, 0)
    rast.set_timing(False)
    st_det = rast.read_timing()
    assert not rast.check_overflow()
    deterministic = dict(value=V * 1000.0 / ms_det, ms_per_step=ms_det,
                         stages_ms={k: (v[0] / v[1] if v[1] else 0.0) for k, v in st_det.items()},
                         gradients_max_rel_diff_to_default=max(
                             float(((out_det[k].double() - out[k].double()).abs().max() /
                                    out_det[k].double().abs().max()).item())
                             for k in ("g_means", "g_quats", "g_log_scales", "g_opacity_logits", "g_rgb", "dq_t", "dt")))
    print(f"[bench] deterministic {ms_det:.3f} ms/step", file=sys.stderr, flush=True)

    # the same step through the autograd function (forward + loss.backward())
    autograd = autograd_bench(rast, raster, w, g, q, t, cams, targets, opts, args)

    # counted work of one batched step (a separate, untimed call)
    o_cnt = raster.RenderOptions(**{**opts.__dict__, "count_work": True})
    rast.render_loss_grad(g, q, t, cams, targets, o_cnt, check=False, out=out)
    work = rast.read_work()
    traffic, traffic_src = measured_traffic("blend_bwd", (tw, th))
    roof = roofline(work, stage_ms["blend_bwd"], traffic, traffic_src)
    roof["tile"] = [tw, th]
    fwd_ms = stage_ms["blend_fwd"]
    roof["blend_fwd"] = {"frac_list": (work["eval_fwd"] * C_ALPHA + work["contrib_fwd"] * C_BLEND) /
                                      (fwd_ms * 1e-3) / VALU_PEAK_LANE_OPS,
                         "frac": work["contrib_fwd"] * (C_ALPHA + C_BLEND) / (fwd_ms * 1e-3) / VALU_PEAK_LANE_OPS,
                         "avg_launch_ms": fwd_ms}

    uneven = None if args.no_uneven else uneven_bench(rast, raster, scenes, dev, args)

    # pose-gradient check: FP32 central differences on 64 Gaussians of the large scene seen by view 0
    pose_fd = None
    if not args.no_fd:
        pose_fd = pose_fd_check(rast, raster, scenes.config5(), dev)

    next_rows = None if args.no_next else next_rows_bench(rast, raster, scenes, w, g, q, t, targets, opts, args)

    # CPU baseline: the oracle on a bounded sample of the same workload
    cpu = None
    if not args.no_cpu:
        cpu = cpu_baseline(w, args.cpu_views)

    value = V * 1000.0 / ms_batched
    res = {
        "metric": METRIC, "value": value, "unit": "views/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms_batched, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": f"tracking room: {args.n} Gaussians, {V} poses at 640x480, fwd+loss+bwd to all "
                               f"Gaussian parameters and poses, batched in one launch sequence, autotuned tile",
                   "n_gaussians": args.n, "views": V, "width": 640, "height": 480, "tile": [tw, th],
                   "autotune": tuned, "visible_records": M, "pairs": K},
        "plain": plain,
        "plain_synced": plain_synced,
        "pose_only": dict(value=V * 1000.0 / ms_pose, ms_per_step=ms_pose),
        "deterministic": deterministic,
        "graph": graph,
        "autograd": autograd,
        "batched_over_plain": (value / plain["value"]) if plain else None,
        "stages_ms": stage_ms,
        "work": work,
        "roofline": roof,
        "cpu_baseline": cpu,
        "pose_fd": pose_fd,
        "uneven_batch": uneven,
        "next_rows": next_rows,
    }
    print(json.dumps(res), flush=True)


def autograd_bench(rast, raster, w, g, q, t, cams, targets, opts, args):
    """render_loss (torch.autograd.Function) forward and loss.backward() for the
    batched step, with the capacity check off (verified after the loop)."""
    import torch
    leaves = [x.clone().requires_grad_(True) for x in g.tensors()]
    ga = raster.GaussianParams(*leaves)
    qa, ta = q.clone().requires_grad_(True), t.clone().requires_grad_(True)
    params = leaves + [qa, ta]

    last = {}

    def step():
        for p in params:
            p.grad = None
        loss = raster.render_loss(rast, ga, qa, ta, cams, targets, opts, check=False)
        loss.backward()
        last["loss"] = loss

    ms = timed(step, args.steps, args.warmup)
    assert not rast.check_overflow()
    V = len(cams)
    print(f"[bench] autograd {ms:.3f} ms/step", file=sys.stderr, flush=True)
    return dict(value=V * 1000.0 / ms, ms_per_step=ms, loss_dtype=str(last["loss"].dtype).replace("torch.", ""),
                path="raster.render_loss (autograd.Function) forward + backward, check=False")


def _uneven_leg(rast, raster, w, dev, label, reps, warmup):
    """Autotuned tile, one fused call captured in a graph, timed replays; work
    counters and per-stage times from eager calls at the same tile."""
    import torch
    g = _params(raster, w.gaussians, dev)
    q, t = _t32(w.views.quat, dev), _t32(w.views.trans, dev)
    qt, tt = _t32(w.target_views.quat, dev), _t32(w.target_views.trans, dev)
    cams = w.views.cams
    V = len(cams)
    P = sum(c.width * c.height for c in cams)
    base = raster.RenderOptions(tile=(16, 16), **w.weights)
    trgb, tdep, tsil, _ = rast.forward(g, qt, tt, cams, base)
    targets = dict(rgb=trgb, depth=tdep, sil=tsil)
    if w.weights.get("w_prior", 0.0) > 0.0 and w.prior_noise is not None:
        targets["prior"] = (tdep * (1.0 + _t32(w.prior_noise[:P], dev))).contiguous()
    tile, ms_tune = rast.autotune(g, q, t, cams, targets, base, reps=3)
    opts = raster.RenderOptions(tile=tile, **w.weights)
    out = rast.render_loss_grad(g, q, t, cams, targets, opts, check=True)
    M, K, _ = rast.last_counters
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        gid, gout = rast.capture_graph(g, q, t, cams, targets, opts)
        ms = timed(lambda: rast.launch_graph(gid), reps, warmup)
        s.synchronize()
        ovf = rast.check_overflow()
        rast.destroy_graph(gid)
    torch.cuda.synchronize()
    rast.read_timing()
    rast.set_timing(True)
    timed(lambda: rast.render_loss_grad(g, q, t, cams, targets, opts, check=False, out=out), reps, 0)
    rast.set_timing(False)
    st = rast.read_timing()
    stage_ms = {k: (v[0] / v[1] if v[1] else 0.0) for k, v in st.items()}
    o_cnt = raster.RenderOptions(**{**opts.__dict__, "count_work": True})
    rast.render_loss_grad(g, q, t, cams, targets, o_cnt, check=False, out=out)
    work = rast.read_work()
    roof = roofline(work, stage_ms["blend_bwd"])
    res = dict(workload=label, views=V, pixels=P, n_gaussians=w.gaussians.n,
               resolutions=sorted({f"{c.width}x{c.height}" for c in cams}), tile=list(tile),
               autotune_ms_per_call=ms_tune, value=V * 1000.0 / ms, unit="views/s", ms_per_step=ms,
               megapixels_per_s=P / ms / 1e3, visible_records=M, pairs=K, overflow=bool(ovf),
               stages_ms=stage_ms, roofline={k: roof[k] for k in ("frac", "frac_list", "achieved", "avg_launch_ms", "work")})
    print(f"[bench] {label}: tile {tile}, {ms:.3f} ms per step ({V * 1000.0 / ms:.0f} views/s)", file=sys.stderr,
          flush=True)
    del g, out, targets
    torch.cuda.empty_cache()
    return res


def uneven_bench(rast, raster, scenes, dev, args):
    reps = max(5, args.steps // 2)
    res = {}
    res["config4"] = _uneven_leg(raster.Rasterizer(0), raster, scenes.config4(), dev,
                                 "uneven room: 1M Gaussians, 32 poses at 320x240..1200x680, fwd+loss+bwd, "
                                 "one graph replay", reps, 2)
    res["config5"] = _uneven_leg(raster.Rasterizer(0), raster, scenes.config5(), dev,
                                 "large multi-room: 3M anisotropic Gaussians, 16 views at 1200x680, depth prior, "
                                 "fwd+loss+bwd, one graph replay", max(3, reps // 2), 1)
    return res


def profile_frame(args, rast, raster, w, g, q, t, targets, opts):
    """--profile-steps for the tracking frame: one 640x480 view, 40 pose-only
    iterations with the decoupled step, eagerly (every launch visible to a
    kernel trace), profile-steps times from the same start pose."""
    import torch
    P1 = 640 * 480
    tg1 = {k: v[:(3 * P1 if k == "rgb" else P1)].contiguous() for k, v in targets.items()}
    hp = raster.PoseAdam(lr_rot=1e-3, lr_pos=1e-3)
    rt = raster.Rasterizer(0)   # its own workspace, sized for one view, as a tracking front end holds it
    for _ in range(args.profile_steps):
        q1, t1 = q[:1].clone(), t[:1].clone()
        rt.track(g, q1, t1, [w.views.cams[0]], tg1, opts, hp, 40)
    torch.cuda.synchronize()
    print(json.dumps({"profile_steps": args.profile_steps, "workload": "frame", "iterations": 40}), flush=True)


def profile_uneven(args, raster, scenes, dev):
    """--profile-steps for the uneven (32-view) or large (3M) workload: eager
    fused calls at the autotuned tile."""
    import torch
    w = scenes.config4() if args.profile_workload == "uneven" else scenes.config5()
    rast = raster.Rasterizer(0)
    g = _params(raster, w.gaussians, dev)
    q, t = _t32(w.views.quat, dev), _t32(w.views.trans, dev)
    qt, tt = _t32(w.target_views.quat, dev), _t32(w.target_views.trans, dev)
    cams = w.views.cams
    base = raster.RenderOptions(tile=(16, 16), **w.weights)
    trgb, tdep, tsil, _ = rast.forward(g, qt, tt, cams, base)
    targets = dict(rgb=trgb, depth=tdep, sil=tsil)
    tile, _ = rast.autotune(g, q, t, cams, targets, base, reps=2)
    opts = raster.RenderOptions(tile=tile, **w.weights)
    out = rast.render_loss_grad(g, q, t, cams, targets, opts, check=True)
    for _ in range(args.profile_steps):
        rast.render_loss_grad(g, q, t, cams, targets, opts, check=False, out=out)
    torch.cuda.synchronize()
    print(json.dumps({"profile_steps": args.profile_steps, "workload": args.profile_workload, "tile": list(tile),
                      "pairs": rast.last_counters[1]}), flush=True)


def next_rows_bench(rast, raster, scenes, w, g, q, t, targets, opts, args):
    """The rows after the path, each timed with HIP events on the current stream."""
    import torch
    dev = q.device
    res = {}
    P1 = 640 * 480
    # tracking: one view, 40 pose-only iterations captured in one graph; a
    # replay continues from the pose and state it finds
    cam0 = [w.views.cams[0]]
    q1, t1 = q[:1].clone(), t[:1].clone()
    tg1 = {k: v[:(3 * P1 if k == "rgb" else P1)].contiguous() for k, v in targets.items()}
    qt0 = w.target_views.quat[0].astype(np.float64)
    ct0 = -_rot(qt0).T @ w.target_views.trans[0].astype(np.float64)

    def pose_err(qq, tt):
        qa = qq[0].double().cpu().numpy()
        ta = tt[0].double().cpu().numpy()
        ang = 2 * np.degrees(np.arccos(min(1.0, abs(float(np.dot(qa / np.linalg.norm(qa), qt0 / np.linalg.norm(qt0)))))))
        return ang, float(np.linalg.norm(-_rot(qa).T @ ta - ct0))

    e0 = pose_err(q1, t1)
    hp = raster.PoseAdam(lr_rot=1e-3, lr_pos=1e-3)
    rt = raster.Rasterizer(0)   # its own workspace, sized for one view, as a tracking front end holds it
    # the tile autotuned for this shape: one view, pose gradients only
    tile1, _ = rt.autotune(g, q1, t1, cam0, tg1, raster.RenderOptions(**{**opts.__dict__, "gauss_grads": False}),
                           reps=3)
    opts1 = raster.RenderOptions(**{**opts.__dict__, "tile": tile1})
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        tr = rt.track(g, q1, t1, cam0, tg1, opts1, hp, 40, capture=True)
        rt.launch_graph(tr["graph"])
        s.synchronize()
        e1 = pose_err(q1, t1)
        lh = tr["loss_hist"][:, 0].cpu().numpy()
        reps = max(3, args.steps // 4)
        ms_frame = timed(lambda: rt.launch_graph(tr["graph"]), reps, 1)
        s.synchronize()
        ovf = rt.check_overflow()
        rt.destroy_graph(tr["graph"])
    torch.cuda.synchronize()
    res["tracking"] = dict(workload="one 640x480 view of the 200k room, pose-only fwd+loss+bwd + decoupled Adam step, "
                                    "40 iterations as one graph replay, own context (pair capacity and autotuned tile for one view)",
                           tile=list(tile1), pair_capacity=rt.pair_capacity, iterations=40, ms_per_frame=ms_frame,
                           iterations_per_s=40 * 1000.0 / ms_frame, overflow=bool(ovf),
                           rotation_err_deg=[e0[0], e1[0]], centre_err_cm=[100 * e0[1], 100 * e1[1]],
                           loss_first_last=[float(lh[0]), float(lh[-1])])
    print(f"[bench] tracking {ms_frame:.3f} ms per 40-iteration frame", file=sys.stderr, flush=True)
    # the same loop for all 8 poses at once (independent per view: a camera rig or pose hypotheses)
    q8, t8 = q.clone(), t.clone()
    with torch.cuda.stream(s):
        tr8 = rast.track(g, q8, t8, w.views.cams, targets, opts, hp, 40, capture=True)
        rast.launch_graph(tr8["graph"])
        s.synchronize()
        ms_frame8 = timed(lambda: rast.launch_graph(tr8["graph"]), max(3, args.steps // 4), 1)
        s.synchronize()
        ovf8 = rast.check_overflow()
        rast.destroy_graph(tr8["graph"])
    torch.cuda.synchronize()
    V8 = len(w.views.cams)
    res["tracking_batched"] = dict(views=V8, iterations=40, ms_per_frame=ms_frame8,
                                   view_iterations_per_s=V8 * 40 * 1000.0 / ms_frame8, overflow=bool(ovf8))
    print(f"[bench] tracking {V8} views: {ms_frame8:.3f} ms per 40-iteration frame", file=sys.stderr, flush=True)

    # mapping loop: the mapping configuration's perturbed 500k map, 8 keyframes, 10 iterations
    # (render + loss + Gaussian gradients + Adam step) per graph replay
    wm = scenes.config3()
    gm = _params(raster, wm.gaussians, dev)
    gt = _params(raster, wm.truth, dev)
    qm, tm = _t32(wm.views.quat, dev), _t32(wm.views.trans, dev)
    om = raster.RenderOptions(**{**wm.weights, "w_prior": 0.0}, tile=opts.tile)
    trgb, tdep, tsil, _ = rast.forward(gt, qm, tm, wm.views.cams, om)
    tgm = dict(rgb=trgb.clone(), depth=tdep.clone(), sil=tsil.clone())
    with torch.cuda.stream(s):
        mp = rast.map_iterate(gm, qm, tm, wm.views.cams, tgm, om, raster.MapAdam(), 10, capture=True)
        rast.launch_graph(mp["graph"])
        s.synchronize()
        l0 = mp["loss_hist"].sum(1).cpu().numpy()
        reps = max(3, args.steps // 4)
        ms_map = timed(lambda: rast.launch_graph(mp["graph"]), reps, 1)
        s.synchronize()
        l1 = mp["loss_hist"].sum(1).cpu().numpy()
        ovf = rast.check_overflow()
        rast.destroy_graph(mp["graph"])
    torch.cuda.synchronize()
    res["mapping"] = dict(workload=f"mapping room: {wm.gaussians.n} Gaussians (perturbed map), {wm.views.n} keyframes "
                                   "at 640x480, fwd+loss+bwd to all Gaussian parameters + Adam step, 10 iterations "
                                   "per graph replay",
                          ms_per_iteration=ms_map / 10, iterations_per_s=10 * 1000.0 / ms_map, overflow=bool(ovf),
                          loss_first_replay=[float(l0[0]), float(l0[-1])],
                          loss_after=float(l1[-1]), replays=1 + 1 + reps)
    print(f"[bench] mapping {ms_map / 10:.3f} ms per iteration", file=sys.stderr, flush=True)
    del gm, gt, tgm

    # mapping Adam step at the mapping (500k) and large (3M) map sizes
    res["map_step"] = []
    for n in (500_000, 3_000_000):
        gen = torch.Generator(device=dev)
        gen.manual_seed(61)
        mk = lambda *sh: torch.randn(*sh, generator=gen, device=dev)  # noqa: E731
        gm = raster.GaussianParams(mk(n, 3), mk(n, 4), mk(n, 3), mk(n), mk(n, 3))
        grads = {"g_" + k: mk(*getattr(gm, k).shape) * 1e-3 for k in ("means", "quats", "log_scales",
                                                                      "opacity_logits", "rgb")}
        st = rast.map_opt_init(gm)
        ms = timed(lambda: rast.map_opt_step(gm, grads, st), max(5, args.steps), 2)
        floats = 14 * n
        algo = floats * 4 * 7   # x read+write, g read, m and v read+write
        gbs = algo / (ms * 1e-3) / 1e9
        res["map_step"].append(dict(n_gaussians=n, ms=ms, algorithmic_bytes=algo, achieved_gbs=gbs,
                                    roofline=dict(bound="hbm", achieved=gbs, peak=HBM_PEAK_GBS, unit="GB/s",
                                                  frac=gbs / HBM_PEAK_GBS)))
        print(f"[bench] map step n={n}: {ms:.3f} ms ({gbs:.0f} GB/s)", file=sys.stderr, flush=True)
        del gm, grads, st

    # new Gaussians from a 640x480 RGB-D frame (silhouette-guided)
    cam = w.views.cams[0]
    gen = torch.Generator(device=dev)
    gen.manual_seed(62)
    depth = torch.rand(P1, generator=gen, device=dev) * 4.0
    sil = torch.rand(P1, generator=gen, device=dev)
    rgb = torch.rand(3 * P1, generator=gen, device=dev)
    cap = P1
    outg = raster.GaussianParams(torch.empty(cap, 3, device=dev), torch.empty(cap, 4, device=dev),
                                 torch.empty(cap, 3, device=dev), torch.empty(cap, device=dev),
                                 torch.empty(cap, 3, device=dev))
    n_new = torch.zeros(1, dtype=torch.int64, device=dev)
    ms_d = timed(lambda: rast.densify(cam, q[0], t[0], rgb, depth, sil, outg, 0, 0.5, n_new=n_new),
                 max(5, args.steps), 2)
    res["densify"] = dict(width=640, height=480, ms=ms_d, new_gaussians=int(n_new.item()),
                          pixels_per_s=P1 * 1000.0 / ms_d)
    print(f"[bench] densify {ms_d:.3f} ms", file=sys.stderr, flush=True)

    # the batched step with isotropic Gaussians (one log-scale each, no rotation)
    giso = raster.GaussianParams(g.means, g.quats, g.log_scales.mean(1, keepdim=True).contiguous(),
                                 g.opacity_logits, g.rgb)
    V = len(w.views.cams)
    P = V * P1
    oiso = rast.alloc_outputs(giso, V, P, opts)
    rast.render_loss_grad(giso, q, t, w.views.cams, targets, opts, check=True, out=oiso)
    ms_iso = timed(lambda: rast.render_loss_grad(giso, q, t, w.views.cams, targets, opts, check=False, out=oiso),
                   args.steps, args.warmup)
    ovf = rast.check_overflow()
    res["isotropic"] = dict(value=V * 1000.0 / ms_iso, unit="views/s", ms_per_step=ms_iso, overflow=bool(ovf))
    print(f"[bench] isotropic {ms_iso:.3f} ms/step", file=sys.stderr, flush=True)
    return res


def kernel_source_hash() -> str:
    import glob
    import hashlib
    h = hashlib.sha256()
    for f in sorted(glob.glob(os.path.join(ROOT, "paper_2408_05635_amd", "csrc", "*"))):
        with open(f, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def measured_traffic(kernel: str, tile):
    """HBM bytes per launch of `kernel` from the committed rocprofv3
    FETCH_SIZE / WRITE_SIZE summary (copy-calibrated), with its source; None
    if the kernel sources or the tile changed since the counters were taken
    (the counters cannot be read from inside this process)."""
    path = os.path.join(ROOT, TRAFFIC_PROFILE)
    if not os.path.exists(path):
        return None, None
    with open(path) as fh:
        t = json.load(fh)
    if t.get("kernel") != "k_" + kernel or t.get("source_sha256") != kernel_source_hash() or \
            list(t.get("tile", [16, 16])) != list(tile):
        return None, "stale: " + TRAFFIC_PROFILE
    return t["read_bytes"] + t["write_bytes"], "stored: " + TRAFFIC_PROFILE + \
        " (rocprofv3 FETCH_SIZE and WRITE_SIZE passes over this 8-view step at this tile with the current kernel" \
        " sources, scaled by a device copy's counts; " + t.get("profile", "") + ")"


def decision_stable_pose_fd(rast, raster, g, q0, t0, cams, tg, opts, h):
    """FP32 central differences of the loss with respect to the pose, over the
    pixels whose decisions (contributing records, clamps, cut-off) and L1
    residual signs are the same at every probed pose: elsewhere the image
    jumps (a Gaussian crossing the 1/255 threshold) or the loss has a kink,
    and the difference quotient does not converge to the gradient there.  The
    analytic gradient is taken with the same pixel weights.  Returns the
    analytic and FD gradients (q then t) and the number of stable pixels."""
    import torch
    o = raster.RenderOptions(**{**opts.__dict__, "gauss_grads": False, "pixel_hash": True})
    P = tg["depth"].numel()

    def run(qq, tt, weight=None):
        t = dict(tg)
        if weight is not None:
            t["weight"] = weight
        out = rast.render_loss_grad(g, qq, tt, cams, t, o)
        return out, rast.pixel_state(g, qq, tt, cams, o)["hash"]

    def signature(out, hsh):   # decisions and the signs of the L1 residuals
        parts = [hsh.to(torch.int64), torch.sign(out["depth"] - tg["depth"]).to(torch.int64),
                 torch.sign(out["sil"] - tg["sil"]).to(torch.int64)]
        if "prior" in tg:
            parts.append(torch.sign(out["depth"] - tg["prior"]).to(torch.int64))
        rgb = torch.sign(out["rgb"] - tg["rgb"]).to(torch.int64)
        return parts + [rgb[c * P:(c + 1) * P] for c in range(3)]

    base, h0 = run(q0, t0)
    sig0 = signature(base, h0)
    stable = torch.ones_like(h0, dtype=torch.bool)
    probes = []
    for j in range(7):
        for sgn in (1.0, -1.0):
            qq, tt = q0.clone(), t0.clone()
            if j < 4:
                qq[0, j] += sgn * h
            else:
                tt[0, j - 4] += sgn * h
            probes.append((qq, tt))
            out, hh = run(qq, tt)
            for a, b in zip(signature(out, hh), sig0):
                stable &= a == b
    wgt = stable.to(torch.float32)
    an, _ = run(q0, t0, wgt)
    analytic = np.concatenate([an["dq_t"].double().cpu().numpy().ravel(), an["dt"].double().cpu().numpy().ravel()])
    fd = np.zeros(7)
    for j in range(7):
        lp = run(*probes[2 * j], wgt)[0]["loss_total"].item()
        lm = run(*probes[2 * j + 1], wgt)[0]["loss_total"].item()
        fd[j] = (lp - lm) / (2 * h)
    return analytic, fd, int(stable.sum().item())


def pose_fd_check(rast, raster, w, dev):
    """64 Gaussians of the large anisotropic scene whose means project inside
    view 0 at a useful depth (sub-seed 51), rendered alone at 1200x680 with
    the scene's loss (silhouette and depth prior); targets at the true pose."""
    G = w.gaussians
    qv = w.views.quat[0].astype(np.float64)
    R = _rot(qv)
    Xc = G.means.astype(np.float64) @ R.T + w.views.trans[0].astype(np.float64)
    cam = w.views.cams[0]
    u = cam.fx * Xc[:, 0] / Xc[:, 2] + cam.cx
    v = cam.fy * Xc[:, 1] / Xc[:, 2] + cam.cy
    ok = np.nonzero((Xc[:, 2] > 0.5) & (u > 40) & (u < cam.width - 40) & (v > 40) & (v < cam.height - 40))[0]
    sel = np.sort(np.random.default_rng(51).choice(ok, size=min(64, ok.size), replace=False))
    sub = G.subset(sel)
    g = _params(raster, sub, dev)
    cams = [cam]
    opts = raster.RenderOptions(tile=(16, 16), **w.weights)
    qt, tt = _t32(w.target_views.quat[:1], dev), _t32(w.target_views.trans[:1], dev)
    trgb, tdep, tsil, _ = rast.forward(g, qt, tt, cams, opts)
    tg = dict(rgb=trgb, depth=tdep, sil=tsil)
    if w.weights.get("w_prior", 0.0) > 0.0:
        P = cam.width * cam.height
        tg["prior"] = (tdep * (1.0 + _t32(w.prior_noise[:P], dev))).contiguous()
    q0, t0 = _t32(w.views.quat[:1], dev), _t32(w.views.trans[:1], dev)
    res = {"workload": "64 Gaussians of the 3M multi-room scene seen by view 0, 1200x680, full loss with "
                       "silhouette and depth prior", "gaussians": int(sel.size),
           "method": "decision-stable central differences, FP32 renders, FP64 loss sum"}
    for h in (1e-3, 1e-4):
        an, fd, n_stable = decision_stable_pose_fd(rast, raster, g, q0, t0, cams, tg, opts, h)
        res[f"h={h:g}"] = {"rel_err_dq": float(np.abs(fd[:4] - an[:4]).max() / max(np.abs(an[:4]).max(), 1e-30)),
                           "rel_err_dt": float(np.abs(fd[4:] - an[4:]).max() / max(np.abs(an[4:]).max(), 1e-30)),
                           "stable_pixels": n_stable}
    print(f"[bench] pose FD {res}", file=sys.stderr, flush=True)
    return res


def _rot(q):
    w, x, y, z = q / np.linalg.norm(q)
    return np.array([[1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y)],
                     [2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x)],
                     [2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)]])


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    import platform
    return platform.processor() or "unknown"


def _oracle_rate(w, n_views, threads, min_seconds):
    import oracle
    sub = w.views.select(range(n_views))
    tsub = w.target_views.select(range(n_views))
    tr = oracle.run(w.gaussians, tsub, threads=threads)
    tg = oracle.Targets(tr.rgb, tr.depth, tr.sil)
    reps, dt = 0, 0.0
    while dt < min_seconds:
        t0 = time.perf_counter()
        oracle.run(w.gaussians, sub, oracle.Options(**w.weights), tg, want_grads=True, threads=threads)
        dt += time.perf_counter() - t0
        reps += 1
    return reps * n_views / dt, reps, dt


def cpu_baseline(w, n_views, min_seconds=10.0, min_seconds_1=6.0):
    """The FP64 oracle (as it stands) on the host: fwd + loss + bwd of the
    tracking views, at every core this process may use (n_views views) and at
    one thread (one view), each repeated until at least the given seconds of
    CPU work are timed."""
    cores = len(os.sched_getaffinity(0))
    cores = min(cores, int(os.environ.get("OMP_NUM_THREADS", cores)))
    v_all, reps, dt = _oracle_rate(w, n_views, cores, min_seconds)
    v_one, reps1, dt1 = _oracle_rate(w, 1, 1, min_seconds_1)
    print(f"[bench] oracle {v_all:.2f} views/s on {cores} threads, {v_one:.3f} on one", file=sys.stderr, flush=True)
    return {"value": v_all, "unit": "views/s", "cores": cores, "kind": "oracle",
            "sample": f"{n_views} of the {w.views.n} tracking views, full 640x480, fwd+loss+bwd, FP64, "
                      f"{reps} repetitions", "seconds": dt, "cpu_model": cpu_model(), "nproc": os.cpu_count(),
            "single_thread": {"value": v_one, "unit": "views/s", "cores": 1,
                              "sample": f"view 0, full 640x480, fwd+loss+bwd, FP64, {reps1} repetitions",
                              "seconds": dt1}}


if __name__ == "__main__":
    main()
