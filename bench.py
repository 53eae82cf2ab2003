"""Benchmark of the wavelet rasterizer on one MI355X.

Headline workload: 3D static view synthesis -- 1,000,000 seeded wavelet
primitives (unit-cube cluster mixture), one 1920x1080 pinhole view on a seeded
orbit, front-to-back alpha blending (T < 1e-4 cutoff), forward + backward in
FP32.  A step is one full pass of the render path: projection, tile binning,
depth and tile sorts, tile ranges, forward blend, backward blend and the
projection backward, with the upstream gradient dL/dimage already resident.

Prints one JSON line (contract: metric, value, unit, ..., roofline,
cpu_baseline).  --gpus N > 1 is refused: this build runs on one GPU.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "fwd+bwd frames/s @1080p,1M prims; served p50/p99 ms vs plain rasterizer"

# Algorithmic FP32 VALU operations per support pair, from the per-pixel rule
# ("Roofline accounting"); transcendentals counted separately.
ALU_PER_PAIR = {("alpha", "fwd"): 22, ("alpha", "bwd"): 43, ("add", "fwd"): 16, ("add", "bwd"): 35}
TRANS_PER_PAIR = {("alpha", "fwd"): 2, ("alpha", "bwd"): 4, ("add", "fwd"): 2, ("add", "bwd"): 3}
# MI355X: 256 CUs x 4 SIMD x 16 lanes x 2.4 GHz = 39.3e12 FP32 lane-ops/s (packed FP32 is not used);
# a transcendental occupies TRANS_SLOTS issue slots (quarter rate on CDNA).
VALU_PEAK = 256 * 4 * 16 * 2.4e9
TRANS_SLOTS = 4.0
HBM_PEAK = 8.0e12


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--prims", type=int, default=1_000_000)
    ap.add_argument("--tile", type=str, default="16x16")
    ap.add_argument("--persistent", type=int, default=2,
                    help="blend launch form: 0 grid, 1 persistent tile queue, 2 queue with longest lists first")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--extras", type=str, default="serve,batched,fit",
                    help="comma list of secondary workloads to add to the JSON line (serve, batched, fit) or none")
    ap.add_argument("--serve-requests", type=int, default=240)
    ap.add_argument("--fit-steps", type=int, default=1000)
    ap.add_argument("--copy-probe-mb", type=int, default=0,
                    help="copy this many MiB device to device once before the run (a kernel of known traffic that "
                         "calibrates hardware byte counters)")
    return ap.parse_args()


TRAFFIC_FILE = os.path.join(ROOT, "profiles", "pmc_traffic_3d_1080p_1M_alpha.md")


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


def bench_serving(n_req, log, persistent=1, load=0.8):
    """Config 5: 8 resident scenes (0.1-2M primitives, linear motion), Poisson requests at
    540p-1080p; the library's continuously batching server vs the plain rasterizer serving one
    request at a time, at the same offered load (80 % of the plain rasterizer's capacity)."""
    import torch
    from paper_2508_12615_amd import binding as B
    from paper_2508_12615_amd import synth
    from paper_2508_12615_amd.raster import Rasterizer
    from paper_2508_12615_amd.serve import Server, run_plain, run_served
    dev = torch.device("cuda", 0)
    scenes = [{k: torch.from_numpy(v).to(dev) for k, v in synth.serve_scene(s).items()} for s in range(8)]
    log("serving: scenes ready")
    probe = synth.serve_requests(48, 1000.0, seed_arrivals=5101, seed_poses=5201)
    rast = Rasterizer(B.WIPES_3D_ALPHA, device=dev)
    outs = [torch.empty((r["camera"]["height"], r["camera"]["width"], 3), device=dev) for r in probe]
    for r in probe:
        r["t_arrive"] = 0.0
    run_plain(rast, scenes, probe[:8], outs[:8])                     # warm-up
    lat, span = run_plain(rast, scenes, probe, outs)
    service_ms = span * 1e3 / len(probe)
    rate = load / (service_ms * 1e-3)
    reqs = synth.serve_requests(n_req, rate)
    outs = [torch.empty((r["camera"]["height"], r["camera"]["width"], 3), device=dev) for r in reqs]
    lat_p, span_p = run_plain(rast, scenes, reqs, outs)
    log("serving: plain done")
    srv = Server(max_slots=16, max_batch=8, persistent=persistent, hbm_budget_bytes=4 << 30)
    ids = [srv.load_scene(sc) for sc in scenes]
    warm = [torch.empty((r["camera"]["height"], r["camera"]["width"], 3), device=dev) for r in probe[:16]]
    run_served(srv, ids, [dict(r, t_arrive=0.0) for r in probe[:16]], warm)   # warm-up
    srv.reset_stats()
    lat_s, span_s = run_served(srv, ids, reqs, outs)
    st = srv.stats()
    srv.close()
    log("serving: served done")
    pct = lambda v, q: float(np.percentile(v, q))  # noqa: E731
    return dict(workload="8 resident scenes of 0.1-2M wavelet primitives with linear motion, %d Poisson requests at "
                         "%.0f/s (%.0f%% of plain capacity), 960x540-1920x1080" % (n_req, rate, 100 * load),
                plain_service_ms=service_ms,
                served=dict(p50_ms=pct(lat_s, 50), p99_ms=pct(lat_s, 99), frames_per_s=n_req / span_s,
                            mean_batch=st["mean_batch"], deferred=st["deferred"],
                            arena_peak_mb=st["arena_peak_bytes"] / 2**20),
                plain=dict(p50_ms=pct(lat_p, 50), p99_ms=pct(lat_p, 99), frames_per_s=n_req / span_p))


def bench_batched(log):
    """Config 4: 64 uneven 2D fits (256-1024 px sides, 2k-50k primitives), one fwd+L2+bwd step
    as one hipGraph replay vs 64 plain per-image steps."""
    import torch
    from paper_2508_12615_amd import binding as B
    from paper_2508_12615_amd import synth
    from paper_2508_12615_amd.fit import BatchedFit
    from paper_2508_12615_amd.raster import Rasterizer
    dev = torch.device("cuda", 0)
    ims = []
    for im in synth.config4():
        ims.append(dict(width=im["width"], height=im["height"], target=torch.from_numpy(im["target"]).to(dev),
                        prims={k: torch.from_numpy(v).to(dev) for k, v in im["prims"].items()}))
    log("batched: inputs ready")
    fit = BatchedFit(ims, persistent=2)
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
    rast = Rasterizer(B.WIPES_2D_ADDITIVE, device=dev)
    views = fit._image_views()
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
                images_per_s_plain=64 / t_plain, speedup=t_plain / t_graph)


def bench_fit(steps, log):
    """Config 2: 768x512 1/f texture with stripe patches, 70k primitives, Adam on the L2 loss,
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


def cpu_baseline(prims, cam):
    """The FP64 oracle on the full frame: projection of every primitive, then the
    per-pixel rule forward and backward in its support-scatter organisation
    (O2: primitives in compositing order update the pixels of their support
    boxes), on all host threads."""
    sys.path.insert(0, os.path.join(ROOT, "oracle"))
    sys.path.insert(0, os.path.join(ROOT, "tests"))
    import oracle as O
    from helpers import oracle_camera, oracle_params
    P = oracle_params(O.MODE_ALPHA3D, O.COV_QUAT_SCALE)
    ocam = oracle_camera(cam)
    W, H = cam["width"], cam["height"]
    g = np.random.default_rng(1).normal(0, 1.0 / (3 * W * H), (H, W, 3))
    t0 = time.perf_counter()
    scr = O.project(P, prims, ocam)
    keys = O.depth_keys(prims, ocam)
    t1 = time.perf_counter()
    img, T, last, tie = O.render_o2(P, W, H, scr, keys)
    t2 = time.perf_counter()
    O.render_bwd_o2(P, W, H, scr, T, last, g, keys)
    t3 = time.perf_counter()
    return dict(value=1.0 / (t3 - t0), unit="frames/s", cores=int(os.environ.get("OMP_NUM_THREADS", os.cpu_count())),
                kind="oracle",
                sample="full frame, %d primitives, %dx%d: FP64 projection %.2f s, forward %.2f s, backward %.2f s "
                       "(support-scatter organisation of the oracle)" % (prims["opacity"].shape[0], W, H,
                                                                         t1 - t0, t2 - t1, t3 - t2))


def main():
    a = parse()
    if a.gpus != 1:
        print("bench.py runs on one GPU only (this build has no multi-GPU path); got --gpus %d" % a.gpus,
              file=sys.stderr)
        sys.exit(2)
    import torch
    from paper_2508_12615_amd import binding as B
    from paper_2508_12615_amd import synth
    from paper_2508_12615_amd.raster import Rasterizer

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
    # per-stage times from a second, separately run set of steps: the stage
    # events themselves cost a few microseconds of idle GPU each, so they stay
    # out of the timed steps above
    B.wipes_profile_enable(r.ctx, True)
    B.wipes_profile_read(r.ctx)                       # drop anything recorded so far
    for _ in range(a.steps):
        step()
    torch.cuda.synchronize()
    prof = B.wipes_profile_read(r.ctx)
    B.wipes_profile_enable(r.ctx, False)
    stages = {k: v[0] / max(v[1], 1) for k, v in prof.items() if v[1] > 0}
    dom = max(stages, key=stages.get)

    def alu_roof(kind, ms):
        pairs = stats["support_fwd" if kind == "fwd" else "support_bwd"]
        slots = ALU_PER_PAIR[("alpha", kind)] + TRANS_SLOTS * TRANS_PER_PAIR[("alpha", kind)]
        ach = pairs * slots / (ms * 1e-3)
        return dict(bound="alu", achieved=ach / 1e12, peak=VALU_PEAK / 1e12, unit="T lane-op/s",
                    frac=ach / VALU_PEAK, traffic=measured_traffic("blend_" + kind), kernel="blend_" + kind,
                    support_pairs=pairs, ops_per_pair=slots)

    if dom in ("blend_fwd", "blend_bwd"):
        roof = alu_roof(dom.split("_")[1], stages[dom])
    else:
        roof = dict(bound="hbm", achieved=None, peak=HBM_PEAK / 1e9, unit="GB/s", frac=None, traffic=None,
                    kernel=dom)
    out = dict(metric=METRIC, value=1e3 / ms_step, unit="frames/s", n_gpus=1, steps=a.steps, warmup=a.warmup,
               ms_per_step=ms_step, higher_is_better=True, scaling="weak", vs_baseline=None, dtype="f32",
               data="synthetic",
               config=dict(workload="3D static view synthesis: %d wavelet primitives, %dx%d, alpha blending, "
                                    "fwd+bwd" % (a.prims, W, H), tile="%dx%d" % (tw, th),
                           launch=("grid", "tile queue", "tile queue, longest first")[a.persistent], instances=K),
               roofline=roof,
               stages_ms={k: round(v, 4) for k, v in stages.items()},
               roofline_blend={k: alu_roof(k, stages["blend_" + k]) for k in ("fwd", "bwd")
                               if "blend_" + k in stages},
               work=stats)
    log = lambda m: print(m, file=sys.stderr, flush=True)  # noqa: E731
    log("gpu: %.3f ms/step, stages %s" % (ms_step, out["stages_ms"]))
    del prims, r
    torch.cuda.empty_cache()
    extras = [] if a.extras == "none" else a.extras.split(",")
    if "batched" in extras:
        out["batched"] = bench_batched(log)
    if "fit" in extras:
        out["fit_loop"] = bench_fit(a.fit_steps, log)
    if "serve" in extras:
        out["serving"] = bench_serving(a.serve_requests, log)
    if not a.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(c["prims"], cam)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
