"""Benchmark of the wavelet rasterizer on one MI355X.

Headline workload: 3D static view synthesis -- 1,000,000 seeded wavelet
primitives (unit-cube cluster mixture), one 1920x1080 pinhole view on a seeded
orbit, front-to-back alpha blending (T < 1e-4 cutoff), forward + backward in
FP32.  A step is one full pass of the render path: projection, tile binning,
depth and tile sorts, tile ranges, forward blend, backward blend and the
projection backward, with the upstream gradient dL/dimage already resident.

Prints one JSON line (contract: metric, value, unit, ..., roofline,
cpu_baseline) with the secondary workloads beside it: the 512x512 fit step,
the 768x512 fitting loop, 64 batched uneven fits (hipGraph + autotuner), and
the server at three offered loads and at saturation.  --gpus N > 1 is
refused: this build runs on one GPU.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import subprocess
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "fwd+bwd frames/s @1080p,1M prims; served p50/p99 ms vs plain rasterizer"

# Algorithmic cost of one support pair (a pixel inside a primitive's support,
# up to the pixel's stopping pair), the unit the blend roofline counts: FP32
# ALU operations of the per-pixel rule and its gradient, and the
# transcendental instructions it needs (the transmittance recovery of the
# alpha backward is one reciprocal).
PAIR_COST = {("alpha", "fwd"): (16, ("exp2", "cos")),
             ("alpha", "bwd"): (40, ("exp2", "cos", "sin", "rcp")),
             ("add", "fwd"): (13, ("exp2", "cos")),
             ("add", "bwd"): (30, ("exp2", "cos", "sin"))}
# MI355X FP32 vector peak: 157.3 TFLOP/s published, a fused multiply-add
# counted as two flops, i.e. 78.6e12 FP32 lane-operations per second
# (256 CUs x 2.4 GHz x 128 FP32 lanes per CU and clock).  The issue-rate probe
# reaches about three quarters of it with plain (non-packed) FMAs, so it is the
# peak whether or not packed FP32 is used; a transcendental nominally takes 4
# issue slots of it (quarter rate).
VALU_PEAK = 157.3e12 / 2.0
NOMINAL_TRANS_SLOTS = 4.0
HBM_PEAK = 8.0e12


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--prims", type=int, default=1_000_000)
    ap.add_argument("--tile", type=str, default="16x16")
    ap.add_argument("--persistent", type=int, default=3,
                    help="blend launch form: 0 grid, 1 persistent tile queue, 2 queue with longest lists first, "
                         "3 grid with longest lists first")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--extras", type=str, default="plain2d,batched,fit,serve,deform",
                    help="comma list of secondary workloads (plain2d, batched, fit, serve, deform) or none")
    ap.add_argument("--serve-requests", type=int, default=2000)
    ap.add_argument("--serve-warmup", type=int, default=200)
    ap.add_argument("--fit-steps", type=int, default=1000)
    ap.add_argument("--copy-probe-mb", type=int, default=0,
                    help="copy this many MiB device to device once before the run (a kernel of known traffic that "
                         "calibrates hardware byte counters)")
    ap.add_argument("--cpu-worker", type=str, default="", help=argparse.SUPPRESS)
    return ap.parse_args()


TRAFFIC_FILE = os.path.join(ROOT, "profiles", "pmc_traffic_3d_1080p_1M_alpha.md")
# blend launch forms (wipes_params.persistent)
LAUNCH_NAMES = ("grid", "tile queue", "tile queue, longest first", "grid, longest first")


def measured_traffic(kernel):
    """HBM bytes per launch of `kernel` from the committed counter summary, or None when there
    is none or the kernel source changed since the counters were taken."""
    import hashlib
    import re
    try:
        text = open(TRAFFIC_FILE).read()
    except OSError:
        return None
    m = re.search(r"source_sha256 = ([0-9a-f]{64})", text)
    t = re.search(r"traffic_bytes_per_launch\[%s\] = ([0-9.eE+]+)" % kernel, text)
    if not m or not t:
        return None
    src = open(os.path.join(ROOT, "paper_2508_12615_amd", "csrc", "blend.hip"), "rb").read()
    if hashlib.sha256(src).hexdigest() != m.group(1):
        return None
    return float(t.group(1))


# --------------------------------------------------------------------- peaks

def measure_rates(ctx, log):
    """Issue rates of FMA and of each transcendental (wipes_probe_issue_rate) and the
    device-to-device copy bandwidth, on this GPU."""
    import torch
    from paper_2508_12615_amd import binding as B
    rates = {op: B.wipes_probe_issue_rate(ctx, op) for op in B.PROBE_OPS}
    # a transcendental's cost in issue slots of the FP32 peak: its time per lane-op times the peak
    slots = {op: VALU_PEAK / rates[op] for op in B.PROBE_OPS if op != "fma"}
    n = 1 << 28   # 1 GiB of float32
    src = torch.ones(n, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    bw = 0.0
    for _ in range(4):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        dst.copy_(src)
        b.record()
        b.synchronize()
        bw = max(bw, 2 * 4 * n / (a.elapsed_time(b) * 1e-3))
    del src, dst
    torch.cuda.empty_cache()
    log("rates: %s; copy %.0f GB/s" % ({k: "%.3g" % v for k, v in rates.items()}, bw / 1e9))
    return dict(lane_ops_per_s={k: v for k, v in rates.items()}, trans_slots=slots, copy_bytes_per_s=bw,
                fma_peak_frac=rates["fma"] / VALU_PEAK, copy_peak_frac=bw / HBM_PEAK)


def blend_roofline(mode, kind, pairs, ms, rates, kernel):
    """Roofline entry of a blend kernel: pairs x (ALU + transcendental slots) / time, a
    transcendental counted at its measured cost in issue slots of the FP32 peak."""
    alu, trans = PAIR_COST[(mode, kind)]
    slots = rates["trans_slots"]
    ops = alu + sum(slots[t] for t in trans)
    ops_nominal = alu + NOMINAL_TRANS_SLOTS * len(trans)
    ach = pairs * ops / (ms * 1e-3)
    fma = rates["lane_ops_per_s"]["fma"]
    return dict(bound="alu", achieved=ach / 1e12, peak=VALU_PEAK / 1e12, unit="T lane-op/s", frac=ach / VALU_PEAK,
                traffic=measured_traffic("blend_" + kind) if mode == "alpha" else None, kernel=kernel,
                support_pairs=int(pairs), ms=ms, ops_per_pair=ops, alu_per_pair=alu, transcendentals=list(trans),
                frac_nominal_slots=pairs * ops_nominal / (ms * 1e-3) / VALU_PEAK,
                frac_of_measured_fma_rate=ach / fma)


def graph_step(r, images, dL, K, ref_image, steps, warmup):
    """The same fwd + bwd step captured once as a hipGraph (wipes_graph_capture: project, bin/sort with
    the instance count kept on the device, forward and backward blend, projection backward) and
    replayed: no host synchronisation per step.  Capacity from the warm-up frame's instance count; the
    replays must not overflow it and must render the plain step's image bit for bit."""
    import torch
    from paper_2508_12615_amd import binding as B
    grads = [{k: torch.empty_like(v) for k, v in images[0]["prims"].items()}]
    batch, keep, _ = r.make_batch(images, grads)
    cap = int(K * 1.1) + 4096
    sb, bb = B.wipes_workspace_size(r.params, batch, cap, True)
    screen = torch.empty(sb, dtype=torch.uint8, device=r.device)
    bins = torch.empty(bb, dtype=torch.uint8, device=r.device)
    sbuf = B.wipes_buffer(screen.data_ptr(), sb, 0, 0, 0)
    bbuf = B.wipes_buffer(bins.data_ptr(), bb, cap, 1, 0)
    npx = ref_image.shape[0]
    image = torch.empty((npx, 3), dtype=torch.float32, device=r.device)
    T = torch.empty(npx, dtype=torch.float32, device=r.device)
    last = torch.empty(npx, dtype=torch.int32, device=r.device)
    g = B.wipes_graph_capture(r.ctx, r.params, batch, sbuf, bbuf, image.data_ptr(), T.data_ptr(), last.data_ptr(),
                              None, dL.data_ptr(), True)
    stream = torch.cuda.current_stream(r.device).cuda_stream
    try:
        for _ in range(warmup):
            B.wipes_graph_launch(g, stream)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            B.wipes_graph_launch(g, stream)
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) * 1e3 / steps
        st, k2 = B.wipes_check_overflow(r.ctx, r.params, batch, sbuf)
        if st != B.WIPES_OK or k2 != K:
            raise RuntimeError("graph replay: instance count %d against %d (capacity %d)" % (k2, K, cap))
        if not torch.equal(image, ref_image):
            raise RuntimeError("graph replay renders a different image")
    finally:
        B.wipes_graph_destroy(g)
    return ms


def stage_profile(r, step, steps):
    """Mean ms per launch of every stage over `steps` calls of step(), from HIP events the library
    records around each stage on its stream."""
    import torch
    from paper_2508_12615_amd import binding as B
    B.wipes_profile_enable(r.ctx, True)
    B.wipes_profile_read(r.ctx)
    for _ in range(steps):
        step()
    torch.cuda.synchronize()
    prof = B.wipes_profile_read(r.ctx)
    B.wipes_profile_enable(r.ctx, False)
    return {k: v[0] / max(v[1], 1) for k, v in prof.items() if v[1] > 0}


# ------------------------------------------------------------ secondary GPU

def bench_plain2d(rates, log):
    """512x512 2D fit step (1/f target, 10k primitives, RS covariances, additive): one plain
    forward + L2 gradient + backward per step, timed, with per-stage times and the blend
    rooflines."""
    import torch
    from paper_2508_12615_amd import binding as B
    from paper_2508_12615_amd import synth
    from paper_2508_12615_amd.raster import Rasterizer
    c = synth.config1()
    dev = torch.device("cuda", 0)
    prims = {k: torch.from_numpy(v).to(dev) for k, v in c["prims"].items()}
    target = torch.from_numpy(c["target"]).to(dev).reshape(-1, 3)
    r = Rasterizer(B.WIPES_2D_ADDITIVE, device=dev)
    images = [dict(camera=(512, 512), prims=prims)]

    def step():
        f = r.forward(images, with_backward=True)
        r.backward(images, f, 2.0 * (f.image - target) / (3 * 512 * 512))
        return f

    for _ in range(10):
        f = step()
    torch.cuda.synchronize()
    stats = r.stats(images, f)
    n = 200
    t0 = time.perf_counter()
    for _ in range(n):
        step()
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / n
    st = stage_profile(r, step, 50)
    log("plain2d: %.3f ms/step" % ms)
    return dict(workload="512x512 2D fit step, 10k primitives, additive, fwd+L2+bwd (plain calls)",
                ms_per_step=ms, steps_per_s=1e3 / ms, stages_us={k: round(v * 1e3, 2) for k, v in st.items()},
                roofline_blend={k: blend_roofline("add", k, stats["support_" + k], st["blend_" + k], rates,
                                                  "blend_" + k) for k in ("fwd", "bwd")},
                work=stats)


def bench_batched(rates, log):
    """64 uneven 2D fits (256-1024 px sides, 2k-50k primitives): the autotuner picks tile shape
    and launch form on the batch, then one fwd+L2+bwd step as one hipGraph replay vs 64 plain
    per-image steps; blend rooflines from the same kernels launched eagerly on the whole batch."""
    import torch
    from paper_2508_12615_amd import binding as B
    from paper_2508_12615_amd import synth
    from paper_2508_12615_amd.fit import BatchedFit
    from paper_2508_12615_amd.raster import Rasterizer, autotune
    dev = torch.device("cuda", 0)
    ims = []
    for im in synth.config4():
        ims.append(dict(width=im["width"], height=im["height"], target=torch.from_numpy(im["target"]).to(dev),
                        prims={k: torch.from_numpy(v).to(dev) for k, v in im["prims"].items()}))
    log("batched: inputs ready")
    # autotune on the batch (fwd + bwd), then the graph with the chosen configuration
    tuner = Rasterizer(B.WIPES_2D_ADDITIVE, device=dev)
    views0 = [dict(camera=(im["width"], im["height"]), prims=im["prims"]) for im in ims]
    times = autotune(tuner, views0, with_backward=True, reps=3)
    best = (tuner.params.tile_w, tuner.params.tile_h, tuner.params.persistent)
    log("batched: autotuner chose %s" % (best,))
    fit = BatchedFit(ims, tile=best[:2], persistent=best[2])
    for _ in range(3):
        fit.render_grads()
    torch.cuda.synchronize()
    fit.check_capacity()
    reps = 10
    t0 = time.perf_counter()
    for _ in range(reps):
        fit.render_grads()
    torch.cuda.synchronize()
    t_graph = (time.perf_counter() - t0) / reps
    fit.check_capacity()
    # the same kernels, launched eagerly on the whole batch, for per-stage times
    rb = Rasterizer(B.WIPES_2D_ADDITIVE, device=dev, tile_w=best[0], tile_h=best[1], persistent=best[2])
    views = fit._image_views()

    def step_b():
        f = rb.forward(views, with_backward=True)
        rb.backward(views, f, fit.dL)
        return f

    fb = step_b()
    torch.cuda.synchronize()
    stats = rb.stats(views, fb)
    st = stage_profile(rb, step_b, 5)
    rast = Rasterizer(B.WIPES_2D_ADDITIVE, device=dev)

    def plain_all():
        for b, v in enumerate(views):
            f = rast.forward([v], with_backward=True)
            W, H = fit.sizes[b]
            o = sum(w * h for (w, h) in fit.sizes[:b])
            dL = 2.0 * (f.image - fit.target[o:o + W * H]) / (3 * W * H)
            rast.backward([v], f, dL)
    plain_all()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(2):
        plain_all()
    torch.cuda.synchronize()
    t_plain = (time.perf_counter() - t0) / 2
    fit.close()
    npx = sum(w * h for (w, h) in fit.sizes)
    return dict(workload="64 uneven 2D fits (%d pixels, %d primitives) fwd+L2+bwd" % (npx, int(fit.offsets[-1])),
                graph_ms=t_graph * 1e3, plain_ms=t_plain * 1e3, images_per_s_graph=64 / t_graph,
                images_per_s_plain=64 / t_plain, speedup=t_plain / t_graph,
                autotuned=dict(tile="%dx%d" % best[:2], launch=LAUNCH_NAMES[best[2]], candidates_ms={"%dx%d/%d" % c: round(v, 3) for c, v in times.items()}),
                stages_ms={k: round(v, 4) for k, v in st.items()},
                roofline_blend={k: blend_roofline("add", k, stats["support_" + k], st["blend_" + k], rates,
                                                  "blend_" + k) for k in ("fwd", "bwd")},
                work=stats)


def bench_fit(steps, log):
    """768x512 1/f texture with stripe patches, 70k primitives, Adam on the L2 loss,
    as the plain autograd loop and as one hipGraph replay per step, from the same start."""
    import torch
    from paper_2508_12615_amd import binding as Bd
    from paper_2508_12615_amd import synth
    from paper_2508_12615_amd.fit import fit_graph, fit_plain, psnr
    from paper_2508_12615_amd.raster import Rasterizer, render
    dev = torch.device("cuda", 0)
    c = synth.config2()
    target = torch.from_numpy(c["target"]).to(dev)
    prims = {k: torch.from_numpy(v).to(dev) for k, v in c["prims"].items()}
    with torch.no_grad():
        p0 = psnr(render(Rasterizer(Bd.WIPES_2D_ADDITIVE, device=dev), (c["width"], c["height"]), **prims), target)
    fit_plain({k: v.clone() for k, v in prims.items()}, target, 5)
    fit_graph({k: v.clone() for k, v in prims.items()}, target, 5)
    plain = fit_plain({k: v.clone() for k, v in prims.items()}, target, steps, log_every=max(1, steps // 4))
    log("fit: plain done")
    graph = fit_graph({k: v.clone() for k, v in prims.items()}, target, steps, log_every=max(1, steps // 4))
    log("fit: graph done")
    return dict(workload="768x512 fit, 70k primitives, %d Adam steps" % steps, psnr_init_db=p0,
                plain=dict(steps_per_s=steps / plain["seconds"], ms_per_step=plain["seconds"] * 1e3 / steps,
                           psnr_db=plain["psnr"], loss=[(i, round(v, 6)) for i, v in plain["history"]]),
                graph=dict(steps_per_s=steps / graph["seconds"], ms_per_step=graph["seconds"] * 1e3 / steps,
                           psnr_db=graph["psnr"], loss=[(i, round(v, 6)) for i, v in graph["history"]],
                           recaptures=graph["recaptures"]))


# multiply-adds per primitive of the deformation network (Eq. 8): 76 -> 256, four 256 -> 256, 332 -> 256,
# two 256 -> 256, 256 -> 13; the backward does twice as many (input and weight gradients)
DEFORM_MACS = 76 * 256 + 6 * 256 * 256 + 332 * 256 + 256 * 13
MFMA_BF16_PEAK = 2.5e15


def bench_deform(log, n=1_000_000, reps=10):
    """Eq. 8 deformation network over the 3D scene's primitives at one time: forward alone (the
    per-frame cost of a dynamic scene) and forward keeping the layer inputs + backward (a training
    step's cost), in both precisions.  Roofline of the forward: the bf16 matrix-core work the
    precision executes (three products per FP32-class product for BF16X3) over the event-timed call,
    against the dense bf16 peak; the FP32-equivalent algorithmic rate beside it."""
    import torch
    from paper_2508_12615_amd import binding as B
    from paper_2508_12615_amd import synth
    from paper_2508_12615_amd.deform import Deformation
    dev = torch.device("cuda", 0)
    shapes = [(256, 76)] + [(256, 256)] * 4 + [(256, 332)] + [(256, 256)] * 2 + [(13, 256)]
    params = torch.from_numpy(synth.deform_params(shapes, 2024)).to(dev)
    mean = torch.from_numpy(synth.scene_3d(n, 2025)["mean"]).to(dev)
    dout = torch.randn((n, 13), device=dev)
    res = {}
    for prec, name, products in ((B.WIPES_DEFORM_BF16X3, "bf16x3", 3), (B.WIPES_DEFORM_BF16, "bf16", 1)):
        net = Deformation(device=dev, precision=prec)
        ws = net.new_workspace(n)
        for keep in (False, True):
            def step():
                net.forward(params, mean, 0.625, keep_for_backward=keep, workspace=ws)
                if keep:
                    net.backward(params, mean, 0.625, dout, workspace=ws)
            step()
            torch.cuda.synchronize()
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record()
            for _ in range(reps):
                step()
            b.record()
            b.synchronize()
            ms = a.elapsed_time(b) / reps
            flops = 2.0 * DEFORM_MACS * n * (3 if keep else 1)
            key = "%s_%s" % (name, "fwd_bwd" if keep else "fwd")
            res[key] = dict(ms=ms, prims_per_s=n / (ms * 1e-3), alg_tflops=flops / (ms * 1e-3) / 1e12,
                            mfma_frac=products * flops / (ms * 1e-3) / MFMA_BF16_PEAK)
            log("deform %s: %.3f ms, %.1f TFLOP/s algorithmic, %.3f of the bf16 MFMA peak"
                % (key, ms, res[key]["alg_tflops"], res[key]["mfma_frac"]))
        net.close()
        del ws
    # a dynamic-scene frame (Sec. 4.3, 6D): the network at time t, the offsets applied, the 1080p view
    # rendered; and the training step through all three (render and network backward)
    from paper_2508_12615_amd.deform import apply_offsets
    from paper_2508_12615_amd.raster import Rasterizer
    c = synth.config3(n)
    prims = {k: torch.from_numpy(v).to(dev) for k, v in c["prims"].items()}
    net = Deformation(device=dev)
    r = Rasterizer(B.WIPES_3D_ALPHA, device=dev)
    W, H = c["camera"]["width"], c["camera"]["height"]
    dL = torch.randn((W * H, 3), device=dev) / (3 * W * H)

    def frame(train):
        if train:
            p = params.detach().requires_grad_(True)
            off = net(p, prims["mean"], 0.625)
            dyn = apply_offsets(net, prims, off)
            f = r.forward([dict(camera=c["camera"], prims=dyn)], with_backward=True)
            grads = r.backward([dict(camera=c["camera"], prims=dyn)], f, dL)[0]
            torch.autograd.backward([dyn[k] for k in ("mean", "freq", "quat", "scale")],
                                    [grads[k] for k in ("mean", "freq", "quat", "scale")])
            return p.grad
        off = net.forward(params, prims["mean"], 0.625)
        dyn = apply_offsets(net, prims, off)
        return r.forward([dict(camera=c["camera"], prims=dyn)]).image

    for train in (False, True):
        frame(train)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            frame(train)
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) * 1e3 / reps
        key = "dynamic_frame_train" if train else "dynamic_frame"
        res[key] = dict(ms=ms, frames_per_s=1e3 / ms)
        log("deform %s: %.3f ms (%.1f frames/s)" % (key, ms, 1e3 / ms))
    net.close()
    del prims, r
    torch.cuda.empty_cache()
    f = res["bf16x3_fwd"]
    ach = 3 * 2.0 * DEFORM_MACS * n / (f["ms"] * 1e-3)
    roof = dict(bound="mfma", achieved=ach / 1e12, peak=MFMA_BF16_PEAK / 1e12, unit="TFLOP/s",
                frac=ach / MFMA_BF16_PEAK, traffic=None, kernel="k_deform_fwd (BF16X3)",
                fp32_equivalent_tflops=f["alg_tflops"], fp32_vector_peak_tflops=157.3)
    return dict(workload="Eq. 8 deformation network, %d primitives, one time; dynamic frame = network + "
                         "applied offsets + 1920x1080 alpha render of the same scene (train: + render and "
                         "network backward)" % n,
                macs_per_primitive=DEFORM_MACS, roofline=roof, **res)


def bench_serving(n_req, n_warm, log, rates, budget=3 << 29):
    """8 resident scenes (0.1-2M primitives, linear motion), Poisson requests at 540p-1080p
    with seeded poses and times.  The plain rasterizer's capacity (one request at a time,
    synchronous) sets the arrival rate; at each offered load rho the library's continuously
    batching server (HBM arena capped at `budget` bytes, so admission binds on memory) and
    the plain rasterizer serve the same arrivals; a saturated run submits everything at once."""
    import torch
    from paper_2508_12615_amd import binding as B
    from paper_2508_12615_amd import synth
    from paper_2508_12615_amd.raster import Rasterizer
    from paper_2508_12615_amd.serve import Server, run_plain, run_served
    dev = torch.device("cuda", 0)
    scenes = [{k: torch.from_numpy(v).to(dev) for k, v in synth.serve_scene(s).items()} for s in range(8)]
    log("serving: scenes ready")
    probe = synth.serve_requests(64, 1000.0, seed_arrivals=5101, seed_poses=5201)
    rast = Rasterizer(B.WIPES_3D_ALPHA, device=dev)
    outs = [torch.empty((r["camera"]["height"], r["camera"]["width"], 3), device=dev) for r in probe]
    for r in probe:
        r["t_arrive"] = 0.0
    run_plain(rast, scenes, probe[:8], outs[:8])                     # warm-up
    lat, span = run_plain(rast, scenes, probe, outs)
    service_ms = span * 1e3 / len(probe)
    # work per request (forward support pairs, wipes_render_stats) over 16 of the probe requests
    pairs = []
    for r in probe[:16]:
        views = [dict(camera=r["camera"], prims=scenes[r["scene"]])]
        pairs.append(rast.stats(views, rast.forward(views))["support_fwd"])
    pairs_per_request = float(np.mean(pairs))
    srv = Server(max_slots=16, max_batch=8, persistent=3, hbm_budget_bytes=budget)
    ids = [srv.load_scene(sc) for sc in scenes]
    pct = lambda v, q: float(np.percentile(v, q))  # noqa: E731
    runs = []
    for rho in (0.5, 0.8, 0.95, None):
        rate = (rho or 1.0) / (service_ms * 1e-3)
        reqs = synth.serve_requests(n_warm + n_req, rate, seed_arrivals=5100 + int(100 * (rho or 1.0)))
        if rho is None:
            for r in reqs:
                r["t_arrive"] = 0.0
        outs = [torch.empty((r["camera"]["height"], r["camera"]["width"], 3), device=dev) for r in reqs]
        # warm-up requests first (not measured), then the measured ones on a fresh clock
        run_plain(rast, scenes, [dict(r, t_arrive=0.0) for r in reqs[:16]], outs[:16])
        lat_p, span_p = run_plain(rast, scenes, reqs[n_warm:], outs[n_warm:])
        run_served(srv, ids, [dict(r, t_arrive=r["t_arrive"]) for r in reqs[:n_warm]], outs[:n_warm])
        srv.reset_stats()
        t_shift = reqs[n_warm]["t_arrive"]
        lat_s, span_s = run_served(srv, ids, [dict(r, t_arrive=r["t_arrive"] - t_shift) for r in reqs[n_warm:]],
                                   outs[n_warm:])
        st = srv.stats()
        runs.append(dict(rho=rho if rho is not None else "saturated", offered_per_s=rate if rho else None,
                         served=dict(p50_ms=pct(lat_s, 50), p99_ms=pct(lat_s, 99), frames_per_s=n_req / span_s,
                                     mean_batch=st["mean_batch"], deferred=int(st["deferred"]),
                                     arena_peak_mb=st["arena_peak_bytes"] / 2**20),
                         plain=dict(p50_ms=pct(lat_p, 50), p99_ms=pct(lat_p, 99), frames_per_s=n_req / span_p)))
        log("serving rho=%s: served p50/p99 %.2f/%.2f ms (%.0f fps, batch %.2f, deferred %d), plain %.2f/%.2f ms "
            "(%.0f fps)" % (rho, runs[-1]["served"]["p50_ms"], runs[-1]["served"]["p99_ms"],
                            runs[-1]["served"]["frames_per_s"], st["mean_batch"], st["deferred"],
                            runs[-1]["plain"]["p50_ms"], runs[-1]["plain"]["p99_ms"], runs[-1]["plain"]["frames_per_s"]))
    srv.close()
    sat = runs[-1]
    # the saturated service against the blend forward's VALU roofline: the requests' support pairs at
    # the per-pair cost, over the whole service time per request (projection, sort and admission
    # included, so a lower bound on the blend kernel's own fraction)
    roof = blend_roofline("alpha", "fwd", pairs_per_request, 1e3 / sat["served"]["frames_per_s"], rates,
                          "served frames (whole service time)")
    roof["support_pairs_per_request"] = pairs_per_request
    roof["traffic"] = None   # the committed counters are the headline frame's, not the served batches
    return dict(workload="8 resident scenes of 0.1-2M wavelet primitives with linear motion, Poisson requests at "
                         "960x540-1920x1080; %d warm-up + %d measured requests per load; arena %d MiB" % (
                             n_warm, n_req, budget >> 20),
                plain_service_ms=service_ms, loads=runs, roofline=roof,
                saturated_served_over_plain=sat["served"]["frames_per_s"] / sat["plain"]["frames_per_s"])


# ---------------------------------------------------------------- CPU oracle

def _cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_worker(kind):
    """One timed sample of the FP64 oracle (run in a child process so OMP_NUM_THREADS applies);
    prints a JSON object with the seconds of each part."""
    sys.path.insert(0, os.path.join(ROOT, "oracle"))
    sys.path.insert(0, os.path.join(ROOT, "tests"))
    import oracle as O
    from helpers import oracle_camera, oracle_params
    from paper_2508_12615_amd import synth
    out = {}
    if kind in ("c3_full", "c3_window"):
        c = synth.config3()
        cam = dict(c["camera"])
        if kind == "c3_window":   # a centred 480x270 window of the frame: 1/16 of its pixels
            cam.update(width=480, height=270, cx=cam["cx"] - 720.0, cy=cam["cy"] - 405.0)
        P = oracle_params(O.MODE_ALPHA3D, O.COV_QUAT_SCALE)
        ocam = oracle_camera(cam)
        W, H = cam["width"], cam["height"]
        g = np.random.default_rng(1).normal(0, 1.0 / (3 * W * H), (H, W, 3))
        t0 = time.perf_counter()
        scr = O.project(P, c["prims"], ocam)
        keys = O.depth_keys(c["prims"], ocam)
        t1 = time.perf_counter()
        img, T, last, tie = O.render_o2(P, W, H, scr, keys)
        t2 = time.perf_counter()
        O.render_bwd_o2(P, W, H, scr, T, last, g, keys)
        t3 = time.perf_counter()
        out = dict(project=t1 - t0, fwd=t2 - t1, bwd=t3 - t2)
    elif kind == "c1":
        c = synth.config1()
        P = oracle_params(O.MODE_ADD2D, O.COV_RS)
        rows = np.arange(0, 512, 16)   # every 16th row: 1/16 of the pixels, brute force over all primitives
        pix = (rows[:, None] * 512 + np.arange(512)[None, :]).reshape(-1)
        t0 = time.perf_counter()
        scr = O.project(P, c["prims"])
        t1 = time.perf_counter()
        img = O.render_o1(P, 512, 512, scr, pix=pix)[0]
        t2 = time.perf_counter()
        O.render_bwd_o1(P, 512, 512, scr, img - c["target"].reshape(-1, 3)[pix], pix=pix)
        t3 = time.perf_counter()
        out = dict(project=t1 - t0, fwd=t2 - t1, bwd=t3 - t2, pixel_fraction=1.0 / 16)
    elif kind == "c2":
        c = synth.config2()
        P = oracle_params(O.MODE_ADD2D, O.COV_RS)
        t0 = time.perf_counter()
        scr = O.project(P, c["prims"])
        img = O.render_o2(P, 768, 512, scr)[0]
        ds = O.render_bwd_o2(P, 768, 512, scr, np.ones(768 * 512), -np.ones(768 * 512, np.int32),
                             2.0 * (img - c["target"]) / (3 * 768 * 512))
        O.project_bwd(P, c["prims"], scr, ds)
        out = dict(step=time.perf_counter() - t0)
    elif kind == "c4":
        P = oracle_params(O.MODE_ADD2D, O.COV_RS)
        ims = synth.config4()
        sel = ims[::8]   # 8 of the 64 images
        t0 = time.perf_counter()
        for im in sel:
            W, H = im["width"], im["height"]
            scr = O.project(P, im["prims"])
            img = O.render_o2(P, W, H, scr)[0]
            ds = O.render_bwd_o2(P, W, H, scr, np.ones(W * H), -np.ones(W * H, np.int32),
                                 2.0 * (img - im["target"]) / (3 * W * H))
            O.project_bwd(P, im["prims"], scr, ds)
        out = dict(seconds=time.perf_counter() - t0, pixels=sum(im["width"] * im["height"] for im in sel),
                   pixels_all=sum(im["width"] * im["height"] for im in ims))
    elif kind == "c5":
        P = oracle_params(O.MODE_ALPHA3D, O.COV_QUAT_SCALE)
        reqs = synth.serve_requests(4, 1000.0)
        host = {}
        t = 0.0
        for r in reqs:
            if r["scene"] not in host:
                host[r["scene"]] = synth.serve_scene(r["scene"])
            prims = host[r["scene"]]
            ocam = oracle_camera(r["camera"])
            t0 = time.perf_counter()
            scr = O.project(P, prims, ocam)
            O.render_o2(P, r["camera"]["width"], r["camera"]["height"], scr, O.depth_keys(prims, ocam))
            t += time.perf_counter() - t0
        out = dict(seconds=t, requests=len(reqs))
    elif kind == "deform":
        import deform as D   # oracle/deform.py
        rows = 20_000
        params = synth.deform_params(D.layer_shapes(), 2024)
        x = synth.scene_3d(rows, 2025)["mean"]
        dout = np.random.default_rng(7).normal(0.0, 1.0, (rows, D.N_OUT))
        D.backward(params, x, 0.625, dout)   # thread pool start and first-touch pages outside the timing
        t0 = time.perf_counter()
        D.forward(params, x, 0.625)
        t1 = time.perf_counter()
        D.backward(params, x, 0.625, dout)
        t2 = time.perf_counter()
        out = dict(fwd=t1 - t0, fwd_bwd=t2 - t1, rows=rows)
    print(json.dumps(out), flush=True)


def cpu_baseline(log):
    """The FP64 oracle as it stands, timed on this host: median of 3 samples per configuration,
    on all host threads and on one thread (the headline only), CPU model stated."""
    nthreads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))

    def run(kind, threads):
        env = dict(os.environ, OMP_NUM_THREADS=str(threads))
        r = subprocess.run([sys.executable, os.path.abspath(__file__), "--cpu-worker", kind], env=env,
                           capture_output=True, text=True, timeout=900)
        if r.returncode != 0:
            raise RuntimeError("cpu worker %s failed: %s" % (kind, r.stderr[-2000:]))
        return json.loads(r.stdout.strip().splitlines()[-1])

    def med(kind, threads, f):
        vals = [f(run(kind, threads)) for _ in range(3)]
        return float(np.median(vals)), vals

    full, full_all = med("c3_full", nthreads, lambda d: d["project"] + d["fwd"] + d["bwd"])
    log("cpu: c3 full frame %.2f s on %d threads" % (full, nthreads))
    # one thread: the projection of all primitives plus 16 x the window's forward and backward
    one, one_all = med("c3_window", 1, lambda d: d["project"] + 16.0 * (d["fwd"] + d["bwd"]))
    log("cpu: c3 one thread %.1f s (extrapolated)" % one)
    c1, _ = med("c1", nthreads, lambda d: d["project"] + (d["fwd"] + d["bwd"]) / d["pixel_fraction"])
    c2, _ = med("c2", nthreads, lambda d: d["step"])
    c4, _ = med("c4", nthreads, lambda d: d["seconds"] * d["pixels_all"] / d["pixels"])
    c5, _ = med("c5", nthreads, lambda d: d["seconds"] / d["requests"])
    log("cpu: c1 %.2f s, c2 %.2f s/step, c4 %.1f s, c5 %.2f s/request" % (c1, c2, c4, c5))
    dfw, _ = med("deform", nthreads, lambda d: d["fwd"] / d["rows"])
    dfb, _ = med("deform", nthreads, lambda d: d["fwd_bwd"] / d["rows"])
    log("cpu: deform %.3g s/row forward, %.3g s/row forward + backward" % (dfw, dfb))
    return dict(value=1.0 / full, unit="frames/s", cores=nthreads, kind="oracle",
                sample="full 1920x1080 frame, 1M primitives: FP64 projection, forward and backward "
                       "(support-scatter organisation of the oracle), median of 3 (%s s)" % ", ".join(
                           "%.2f" % v for v in full_all),
                cpu_model=_cpu_model(), median_of=3,
                one_thread=dict(value=1.0 / one, unit="frames/s", cores=1,
                                sample="projection of all 1M primitives + 16 x a centred 480x270 window's forward "
                                       "and backward (1/16 of the pixels, the frame's densest part: an upper bound on "
                                       "the time), median of 3 (%s s)" % ", ".join(
                                           "%.1f" % v for v in one_all)),
                configs=dict(
                    plain2d=dict(value=1.0 / c1, unit="fwd+bwd steps/s", sample="512x512, 10k primitives: brute "
                                 "force over every 16th row, extrapolated to the image"),
                    fit=dict(value=1.0 / c2, unit="Adam steps/s", sample="one fwd+L2+bwd step of the 768x512, "
                             "70k-primitive fit (without the optimiser update)"),
                    batched=dict(value=64.0 / c4, unit="images/s", sample="8 of the 64 images fwd+L2+bwd, "
                                 "extrapolated by pixel count"),
                    serving=dict(value=1.0 / c5, unit="frames/s", sample="forward of 4 served requests"),
                    deform=dict(value=1.0 / dfw, unit="primitives/s (forward)", fwd_bwd=1.0 / dfb,
                                sample="the FP64 network on 20k of the scene's primitives (numpy matrix products), "
                                       "forward, and forward + backward")))


# ---------------------------------------------------------------------- main

def main():
    a = parse()
    if a.cpu_worker:
        cpu_worker(a.cpu_worker)
        return
    if a.gpus != 1:
        print("bench.py runs on one GPU only (this build has no multi-GPU path); got --gpus %d" % a.gpus,
              file=sys.stderr)
        sys.exit(2)
    import torch
    from paper_2508_12615_amd import binding as B
    from paper_2508_12615_amd import synth
    from paper_2508_12615_amd.raster import Rasterizer
    log = lambda m: print(m, file=sys.stderr, flush=True)  # noqa: E731

    dev = torch.device("cuda", 0)
    if a.copy_probe_mb > 0:
        src = torch.ones(a.copy_probe_mb << 18, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    c = synth.config3(a.prims)
    cam = c["camera"]
    W, H = cam["width"], cam["height"]
    prims = {k: torch.from_numpy(v).to(dev) for k, v in c["prims"].items()}
    tw, th = (int(x) for x in a.tile.split("x"))
    r = Rasterizer(B.WIPES_3D_ALPHA, device=dev, tile_w=tw, tile_h=th, persistent=a.persistent)
    rates = measure_rates(r.ctx, log)
    images = [dict(camera=cam, prims=prims)]
    dL = torch.from_numpy(np.random.default_rng(1).normal(0, 1.0 / (3 * W * H), (W * H, 3)).astype(np.float32)).to(dev)

    def step():
        f = r.forward(images, with_backward=True)
        r.backward(images, f, dL)
        return f

    for _ in range(a.warmup):
        f = step()
    torch.cuda.synchronize()
    stats = r.stats(images, f)
    K = f.K
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(a.steps):
        step()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ms_step = (t1 - t0) * 1e3 / a.steps
    ms_graph = graph_step(r, images, dL, K, f.image, a.steps, a.warmup)
    log("gpu: %.3f ms/step plain, %.3f ms/step as one graph replay" % (ms_step, ms_graph))
    # per-stage times from a second, separately run set of steps: the stage
    # events themselves cost a few microseconds of idle GPU each, so they stay
    # out of the timed steps above
    stages = stage_profile(r, step, a.steps)
    dom = max(stages, key=stages.get)
    roof_blend = {k: blend_roofline("alpha", k, stats["support_" + k], stages["blend_" + k], rates, "blend_" + k)
                  for k in ("fwd", "bwd")}
    if dom in ("blend_fwd", "blend_bwd"):
        roof = roof_blend[dom.split("_")[1]]
    else:
        roof = dict(bound="hbm", achieved=None, peak=HBM_PEAK / 1e9, unit="GB/s", frac=None, traffic=None,
                    kernel=dom)
    # the whole step against the sum of the stages' rooflines (blends: VALU; the rest: HBM at the
    # algorithmic bytes per primitive and per instance)
    n = a.prims
    hbm_bytes = n * (148 + 150) + K * (12 + 2 * 24 + 8) + n * 4 * 24
    t_roof = sum(v["support_pairs"] * v["ops_per_pair"] / VALU_PEAK for v in roof_blend.values()) + hbm_bytes / HBM_PEAK
    out = dict(metric=METRIC, value=1e3 / ms_step, unit="frames/s", n_gpus=1, steps=a.steps, warmup=a.warmup,
               ms_per_step=ms_step, higher_is_better=True, scaling="weak", vs_baseline=None, dtype="f32",
               data="synthetic",
               config=dict(workload="3D static view synthesis: %d wavelet primitives, %dx%d, alpha blending, "
                                    "fwd+bwd" % (a.prims, W, H), tile="%dx%d" % (tw, th),
                           launch=LAUNCH_NAMES[a.persistent], instances=K),
               roofline=roof,
               step_roofline=dict(t_roof_ms=t_roof * 1e3, frac=t_roof * 1e3 / ms_step),
               stages_ms={k: round(v, 4) for k, v in stages.items()},
               roofline_blend=roof_blend, measured_peaks=rates, work=stats,
               graph_replay=dict(ms_per_step=ms_graph, frames_per_s=1e3 / ms_graph,
                                 note="the same step captured once as a hipGraph and replayed (no host "
                                      "synchronisation per step); same image bit for bit"))
    log("gpu: %.3f ms/step, stages %s" % (ms_step, out["stages_ms"]))
    del prims, r
    torch.cuda.empty_cache()
    extras = [] if a.extras == "none" else a.extras.split(",")
    if "plain2d" in extras:
        out["plain2d"] = bench_plain2d(rates, log)
    if "batched" in extras:
        out["batched"] = bench_batched(rates, log)
    if "fit" in extras:
        out["fit_loop"] = bench_fit(a.fit_steps, log)
    if "serve" in extras:
        out["serving"] = bench_serving(a.serve_requests, a.serve_warmup, log, rates)
    if "deform" in extras:
        out["deform"] = bench_deform(log)
    if not a.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(log)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
