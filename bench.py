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
ALU_PER_PAIR = {("alpha", "fwd"): 22, ("alpha", "bwd"): 52, ("add", "fwd"): 16, ("add", "bwd"): 44}
TRANS_PER_PAIR = {("alpha", "fwd"): 2, ("alpha", "bwd"): 4, ("add", "fwd"): 2, ("add", "bwd"): 3}
# MI355X: 256 CUs x 4 SIMD x 16 lanes x 2.4 GHz = 39.3e12 FP32 lane-ops/s (packed FP32 is not used);
# a transcendental occupies TRANS_SLOTS issue slots (quarter rate on CDNA).
VALU_PEAK = 256 * 4 * 16 * 2.4e9
TRANS_SLOTS = 4.0
HBM_PEAK = 8.0e12


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--prims", type=int, default=1_000_000)
    ap.add_argument("--tile", type=str, default="16x16")
    ap.add_argument("--persistent", type=int, default=0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-crop", type=int, default=16, help="CPU baseline crop = 1/cpu-crop of the frame")
    return ap.parse_args()


def cpu_baseline(prims, cam, crop_div):
    """The FP64 oracle on a bounded sample: projection of all primitives, then the
    per-pixel rule forward + backward over a centred crop of 1/crop_div of the
    frame (primitives whose support box misses the crop cannot touch it and are
    dropped first), extrapolated to a full frame."""
    sys.path.insert(0, os.path.join(ROOT, "oracle"))
    sys.path.insert(0, os.path.join(ROOT, "tests"))
    import oracle as O
    from helpers import oracle_camera, oracle_params
    P = oracle_params(O.MODE_ALPHA3D, O.COV_QUAT_SCALE)
    ocam = oracle_camera(cam)
    W, H = cam["width"], cam["height"]
    s = math.sqrt(crop_div)
    cw, ch = int(round(W / s)), int(round(H / s))
    x0, y0 = (W - cw) // 2, (H - ch) // 2
    t0 = time.perf_counter()
    scr = O.project(P, prims, ocam)
    keys = O.depth_keys(prims, ocam)
    t_proj = time.perf_counter() - t0
    hit = (scr[:, 15] != 0) & (scr[:, 0] + scr[:, 12] + 0.02 >= x0) & (scr[:, 0] - scr[:, 12] - 0.02 <= x0 + cw) & \
          (scr[:, 1] + scr[:, 13] + 0.02 >= y0) & (scr[:, 1] - scr[:, 13] - 0.02 <= y0 + ch)
    idx = np.flatnonzero(hit)
    sub = np.ascontiguousarray(scr[idx])
    subkeys = np.ascontiguousarray(keys[idx])
    ys, xs = np.mgrid[y0:y0 + ch, x0:x0 + cw]
    pix = (ys * W + xs).reshape(-1).astype(np.int64)
    g = np.random.default_rng(0).normal(0, 1, (pix.size, 3))
    t1 = time.perf_counter()
    O.render_o1(P, W, H, sub, subkeys, pix=pix)
    O.render_bwd_o1(P, W, H, sub, g, subkeys, pix=pix)
    t_pix = time.perf_counter() - t1
    frame_s = t_proj + t_pix * (W * H) / pix.size
    return dict(value=1.0 / frame_s, unit="frames/s", cores=int(os.environ.get("OMP_NUM_THREADS", os.cpu_count())),
                kind="oracle",
                sample="FP64 oracle: projection of all %d primitives (%.2f s) + per-pixel forward+backward over a "
                       "centred %dx%d crop (1/%d of the frame, %d primitives reach it; %.2f s), extrapolated to the "
                       "full frame" % (prims["opacity"].shape[0], t_proj, cw, ch, crop_div, idx.size, t_pix))


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
    B.wipes_profile_enable(r.ctx, True)
    B.wipes_profile_read(r.ctx)                       # drop anything recorded so far
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(a.steps):
        step()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    prof = B.wipes_profile_read(r.ctx)
    B.wipes_profile_enable(r.ctx, False)
    ms_step = (t1 - t0) * 1e3 / a.steps
    stages = {k: v[0] / max(v[1], 1) for k, v in prof.items() if v[1] > 0}
    dom = max(stages, key=stages.get)

    def alu_roof(kind, ms):
        pairs = stats["support_fwd" if kind == "fwd" else "support_bwd"]
        slots = ALU_PER_PAIR[("alpha", kind)] + TRANS_SLOTS * TRANS_PER_PAIR[("alpha", kind)]
        ach = pairs * slots / (ms * 1e-3)
        return dict(bound="alu", achieved=ach / 1e12, peak=VALU_PEAK / 1e12, unit="T lane-op/s",
                    frac=ach / VALU_PEAK, traffic=None, kernel="blend_" + kind, support_pairs=pairs,
                    ops_per_pair=slots)

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
                           persistent=bool(a.persistent), instances=K),
               roofline=roof,
               stages_ms={k: round(v, 4) for k, v in stages.items()},
               roofline_blend={k: alu_roof(k, stages["blend_" + k]) for k in ("fwd", "bwd")
                               if "blend_" + k in stages},
               work=stats)
    print("gpu: %.3f ms/step, stages %s" % (ms_step, out["stages_ms"]), file=sys.stderr, flush=True)
    if not a.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(c["prims"], cam, a.cpu_crop)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
