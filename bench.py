#!/usr/bin/env python3
"""Throughput of the differentiable Gaussian rasteriser on one MI355X.

Workload (the tracking configuration): a synthetic 4x4x3 m room with 200k
Gaussians, 8 camera poses along a smooth trajectory, 640x480, f = 525.
One step = forward + combined L1 loss + backward to every Gaussian
parameter and to the poses, for all 8 views.  Targets are renders at the
true poses; the renderer is evaluated at poses 2 deg / 2 cm away.

Reported (one JSON line):
  value         views/s of the batched path (all views in one launch
                sequence), full gradients, inputs resident in HBM
  plain         the same views one at a time (one launch sequence and one
                pair-count check per view)
  pose_only     batched, gradients to the poses only (tracking mode)
  graph         batched, replayed from a captured HIP graph
  stages_ms     per-stage averages from HIP events on the library's stream
  roofline      the dominant kernel (the backward blend) against the FP32
                VALU peak, from counted work
  cpu_baseline  the FP64 oracle on the host cores, on a bounded sample
  pose_fd       FP32 central-difference check of the pose gradients
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
# algorithmic FP32 lane-op slots per (pixel, Gaussian) pair of the blend,
# transcendental ops at quarter rate (4 slots): see the roofline section of the design notes
C_ALPHA = 17     # dx, dy (split mean), factor products, exp2, opacity, clamp, 1/255 test
C_BLEND = 10     # transmittance update, stop test, 4 channel FMAs + silhouette, position
C_GRAD = 45      # transmittance recovery (rcp), dL/dalpha, behind-accumulators, 10 partials


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--n", type=int, default=200_000)
    ap.add_argument("--views", type=int, default=8)
    ap.add_argument("--tile", default="16x16")
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle CPU baseline")
    ap.add_argument("--no-plain", action="store_true")
    ap.add_argument("--no-graph", action="store_true")
    ap.add_argument("--cpu-views", type=int, default=8, help="views in the oracle's timed sample")
    ap.add_argument("--no-next", action="store_true", help="skip the tracking / mapping / densify / isotropic legs")
    ap.add_argument("--profile-steps", type=int, default=0,
                    help="only run this many batched steps (for a profiler) and print nothing else")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="with --profile-steps: also copy 256 MiB device to device, the reference for the "
                         "HBM byte counters")
    return ap.parse_args()


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
    tw, th = (int(x) for x in args.tile.split("x"))
    w = scenes.config2(n_views=args.views, n=args.n)
    t32 = lambda a: torch.from_numpy(np.ascontiguousarray(a, np.float32)).to(dev)  # noqa: E731
    G = w.gaussians
    g = raster.GaussianParams(t32(G.means), t32(G.quats), t32(G.log_scales), t32(G.opacity_logits), t32(G.rgb))
    q, t = t32(w.views.quat), t32(w.views.trans)
    qt, tt = t32(w.target_views.quat), t32(w.target_views.trans)
    cams = w.views.cams
    V = len(cams)
    P = sum(c.width * c.height for c in cams)
    opts = raster.RenderOptions(tile=(tw, th), **w.weights)
    rast = raster.Rasterizer(0)

    # targets: renders at the true poses (inputs of the workload)
    trgb, tdep, tsil, _ = rast.forward(g, qt, tt, cams, opts)
    targets = dict(rgb=trgb, depth=tdep, sil=tsil)
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
        print(json.dumps({"profile_steps": args.profile_steps, "pairs": K, "visible": M}), flush=True)
        return

    def timed(fn, steps, warmup):
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

    # batched, full gradients; per-stage HIP events recorded over the same region
    for _ in range(args.warmup):
        batched_step()
    torch.cuda.synchronize()
    rast.read_timing()
    rast.set_timing(True)
    ms_batched = timed(batched_step, args.steps, 0)
    rast.set_timing(False)
    stages = rast.read_timing()
    _, _, ovf2 = rast.read_counters(rast.shared_workspace())
    assert not ovf2, "pair capacity overflowed during the timed region"
    print(f"[bench] batched {ms_batched:.3f} ms/step ({V * 1000.0 / ms_batched:.1f} views/s)", file=sys.stderr,
          flush=True)
    stage_ms = {k: (v[0] / v[1] if v[1] else 0.0) for k, v in stages.items()}

    # pose-only (tracking) mode
    o_pose = raster.RenderOptions(**{**opts.__dict__, "gauss_grads": False})
    out_pose = rast.alloc_outputs(g, V, P, o_pose)
    rast.render_loss_grad(g, q, t, cams, targets, o_pose, check=True, out=out_pose)
    ms_pose = timed(lambda: batched_step(o_pose, out_pose), args.steps, args.warmup)
    print(f"[bench] pose-only {ms_pose:.3f} ms/step", file=sys.stderr, flush=True)

    # plain: one view per launch sequence, each with its pair-count check
    plain = None
    if not args.no_plain:
        rast1 = raster.Rasterizer(0)   # its own workspace, sized for one view
        singles = []
        for v in range(V):
            tg_v = dict(rgb=trgb[3 * P // V * v:3 * P // V * (v + 1)], depth=tdep[P // V * v:P // V * (v + 1)],
                        sil=tsil[P // V * v:P // V * (v + 1)])
            singles.append((q[v:v + 1].contiguous(), t[v:v + 1].contiguous(), [cams[v]], tg_v,
                            rast1.alloc_outputs(g, 1, P // V, opts)))

        def plain_step():
            for (qv, tv, cv, tgv, ov) in singles:
                rast1.render_loss_grad(g, qv, tv, cv, tgv, opts, check=True, out=ov)

        ms_plain = timed(plain_step, args.steps, args.warmup)
        plain = dict(value=V * 1000.0 / ms_plain, ms_per_step=ms_plain)
        print(f"[bench] plain {ms_plain:.3f} ms/step", file=sys.stderr, flush=True)

    # batched, replayed from a HIP graph captured by the library (gsr_graph_capture)
    graph = None
    if not args.no_graph:
        s = torch.cuda.Stream()
        s.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(s):
            gid, gout = rast.capture_graph(g, q, t, cams, targets, opts)
            ms_graph = timed(lambda: rast.launch_graph(gid), args.steps, args.warmup)
            s.synchronize()
            _, _, ovf3 = rast.read_counters(rast.shared_workspace())
            assert not ovf3
            same = all(torch.equal(gout[k], out[k]) for k in ("rgb", "loss", "g_means", "dq_t"))
            rast.destroy_graph(gid)
        torch.cuda.synchronize()
        graph = dict(value=V * 1000.0 / ms_graph, ms_per_step=ms_graph, bitwise_equal_to_eager=bool(same))
        print(f"[bench] graph {ms_graph:.3f} ms/step", file=sys.stderr, flush=True)

    # counted work of one batched step (a separate, untimed call)
    o_cnt = raster.RenderOptions(**{**opts.__dict__, "count_work": True})
    rast.render_loss_grad(g, q, t, cams, targets, o_cnt, check=False, out=out)
    work = rast.read_work()
    ops_fwd = work["contrib_fwd"] * (C_ALPHA + C_BLEND)
    ops_bwd = work["contrib_bwd"] * (C_ALPHA + C_GRAD)
    ops_bwd_list = ops_bwd + (work["eval_bwd"] - work["contrib_bwd"]) * C_ALPHA
    dom = "blend_bwd" if stage_ms["blend_bwd"] >= stage_ms["blend_fwd"] else "blend_fwd"
    dom_ops = ops_bwd if dom == "blend_bwd" else ops_fwd
    dom_ms = stage_ms[dom]
    achieved = dom_ops / (dom_ms * 1e-3) / 1e12
    peak = VALU_PEAK_LANE_OPS / 1e12
    roofline = {"bound": "alu", "kernel": dom, "achieved": achieved, "peak": peak, "unit": "T lane-op/s",
                "frac": achieved / peak, "traffic": measured_traffic(dom),
                "frac_list": ((ops_bwd_list if dom == "blend_bwd" else ops_fwd) / (dom_ms * 1e-3) / 1e12) / peak,
                "ops_per_launch": dom_ops, "avg_launch_ms": dom_ms}

    # pose-gradient check: FP32 central differences on 64 Gaussians seen by view 0
    pose_fd = pose_fd_check(rast, raster, w, dev, opts)

    next_rows = None if args.no_next else next_rows_bench(rast, raster, scenes, w, g, q, t, targets, opts, timed,
                                                          args)

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
                               f"Gaussian parameters and poses, batched in one launch sequence",
                   "n_gaussians": args.n, "views": V, "width": 640, "height": 480, "tile": [tw, th],
                   "visible_records": M, "pairs": K},
        "plain": plain,
        "pose_only": dict(value=V * 1000.0 / ms_pose, ms_per_step=ms_pose),
        "graph": graph,
        "batched_over_plain": (value / plain["value"]) if plain else None,
        "stages_ms": stage_ms,
        "work": work,
        "roofline": roofline,
        "cpu_baseline": cpu,
        "pose_fd": pose_fd,
        "next_rows": next_rows,
    }
    print(json.dumps(res), flush=True)


def next_rows_bench(rast, raster, scenes, w, g, q, t, targets, opts, timed, args):
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
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        tr = rast.track(g, q1, t1, cam0, tg1, opts, hp, 40, capture=True)
        rast.launch_graph(tr["graph"])
        s.synchronize()
        e1 = pose_err(q1, t1)
        lh = tr["loss_hist"][:, 0].cpu().numpy()
        reps = max(3, args.steps // 4)
        ms_frame = timed(lambda: rast.launch_graph(tr["graph"]), reps, 1)
        s.synchronize()
        _, _, ovf = rast.read_counters(rast.shared_workspace())
        rast.destroy_graph(tr["graph"])
    torch.cuda.synchronize()
    res["tracking"] = dict(workload="one 640x480 view of the 200k room, pose-only fwd+loss+bwd + decoupled Adam step, "
                                    "40 iterations as one graph replay", iterations=40, ms_per_frame=ms_frame,
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
        _, _, ovf8 = rast.read_counters(rast.shared_workspace())
        rast.destroy_graph(tr8["graph"])
    torch.cuda.synchronize()
    V8 = len(w.views.cams)
    res["tracking_batched"] = dict(views=V8, iterations=40, ms_per_frame=ms_frame8,
                                   view_iterations_per_s=V8 * 40 * 1000.0 / ms_frame8, overflow=bool(ovf8))
    print(f"[bench] tracking {V8} views: {ms_frame8:.3f} ms per 40-iteration frame", file=sys.stderr, flush=True)

    # mapping loop: the mapping configuration's perturbed 500k map, 8 keyframes, 10 iterations
    # (render + loss + Gaussian gradients + Adam step) per graph replay
    wm = scenes.config3()
    t32 = lambda a: torch.from_numpy(np.ascontiguousarray(a, np.float32)).to(dev)  # noqa: E731
    Gm, Gt = wm.gaussians, wm.truth
    gm = raster.GaussianParams(t32(Gm.means), t32(Gm.quats), t32(Gm.log_scales), t32(Gm.opacity_logits), t32(Gm.rgb))
    gt = raster.GaussianParams(t32(Gt.means), t32(Gt.quats), t32(Gt.log_scales), t32(Gt.opacity_logits), t32(Gt.rgb))
    qm, tm = t32(wm.views.quat), t32(wm.views.trans)
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
        _, _, ovf = rast.read_counters(rast.shared_workspace())
        rast.destroy_graph(mp["graph"])
    torch.cuda.synchronize()
    res["mapping"] = dict(workload=f"mapping room: {Gm.n} Gaussians (perturbed map), {wm.views.n} keyframes at 640x480, "
                                   "fwd+loss+bwd to all Gaussian parameters + Adam step, 10 iterations per graph replay",
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
    _, _, ovf = rast.read_counters(rast.shared_workspace())
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


def measured_traffic(kernel: str):
    """HBM bytes per launch of `kernel` from the committed rocprofv3 FETCH_SIZE /
    WRITE_SIZE summary (copy-calibrated), or None if the kernel sources changed
    since the counters were taken."""
    path = os.path.join(ROOT, "profiles", "blend_bwd_traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        t = json.load(fh)
    if t.get("kernel") != "k_" + kernel or t.get("source_sha256") != kernel_source_hash():
        return None
    return t["read_bytes"] + t["write_bytes"]


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
    dev = q0.device

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
        lp = run(*probes[2 * j], wgt)[0]["loss"].sum().item()
        lm = run(*probes[2 * j + 1], wgt)[0]["loss"].sum().item()
        fd[j] = (lp - lm) / (2 * h)
    return analytic, fd, int(stable.sum().item())


def pose_fd_check(rast, raster, w, dev, opts):
    import torch
    G = w.gaussians
    # Gaussians whose means project inside view 0 at a useful depth, 64 of them (seeded)
    qv = w.views.quat[0].astype(np.float64)
    R = _rot(qv)
    Xc = G.means.astype(np.float64) @ R.T + w.views.trans[0].astype(np.float64)
    cam = w.views.cams[0]
    u = cam.fx * Xc[:, 0] / Xc[:, 2] + cam.cx
    v = cam.fy * Xc[:, 1] / Xc[:, 2] + cam.cy
    ok = np.nonzero((Xc[:, 2] > 0.5) & (u > 40) & (u < cam.width - 40) & (v > 40) & (v < cam.height - 40))[0]
    sel = np.sort(np.random.default_rng(51).choice(ok, size=min(64, ok.size), replace=False))
    sub = G.subset(sel)
    t32 = lambda a: torch.from_numpy(np.ascontiguousarray(a, np.float32)).to(dev)  # noqa: E731
    g = raster.GaussianParams(t32(sub.means), t32(sub.quats), t32(sub.log_scales), t32(sub.opacity_logits),
                              t32(sub.rgb))
    cams = [cam]
    qt, tt = t32(w.target_views.quat[:1]), t32(w.target_views.trans[:1])
    trgb, tdep, tsil, _ = rast.forward(g, qt, tt, cams, opts)
    tg = dict(rgb=trgb, depth=tdep, sil=tsil)
    q0, t0 = t32(w.views.quat[:1]), t32(w.views.trans[:1])
    res = {"gaussians": int(sel.size), "method": "decision-stable central differences, FP32 renders, FP64 loss sum"}
    for h in (1e-3, 1e-4):
        an, fd, n_stable = decision_stable_pose_fd(rast, raster, g, q0, t0, cams, tg, opts, h)
        res[f"h={h:g}"] = {"rel_err_dq": float(np.abs(fd[:4] - an[:4]).max() / max(np.abs(an[:4]).max(), 1e-30)),
                           "rel_err_dt": float(np.abs(fd[4:] - an[4:]).max() / max(np.abs(an[4:]).max(), 1e-30)),
                           "stable_pixels": n_stable}
    return res


def _rot(q):
    w, x, y, z = q / np.linalg.norm(q)
    return np.array([[1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y)],
                     [2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x)],
                     [2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)]])


def cpu_baseline(w, n_views, min_seconds=10.0):
    """The FP64 oracle (as it stands) on the host cores: fwd + loss + bwd of
    n_views of the same scene and poses, repeated until at least min_seconds
    of CPU work have been timed."""
    import oracle
    cores = len(os.sched_getaffinity(0))
    cores = min(cores, int(os.environ.get("OMP_NUM_THREADS", cores)))
    sub = w.views.select(range(n_views))
    tsub = w.target_views.select(range(n_views))
    tr = oracle.run(w.gaussians, tsub, threads=cores)
    tg = oracle.Targets(tr.rgb, tr.depth, tr.sil)
    reps, dt = 0, 0.0
    while dt < min_seconds:
        t0 = time.perf_counter()
        oracle.run(w.gaussians, sub, oracle.Options(**w.weights), tg, want_grads=True, threads=cores)
        dt += time.perf_counter() - t0
        reps += 1
    return {"value": reps * n_views / dt, "unit": "views/s", "cores": cores, "kind": "oracle",
            "sample": f"{n_views} of the {w.views.n} tracking views, full 640x480, fwd+loss+bwd, FP64, "
                      f"{reps} repetitions", "seconds": dt}


if __name__ == "__main__":
    main()
