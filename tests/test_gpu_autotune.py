"""The autotuner (wipes_autotune) on the GPU: it times every tile shape and
blend launch form on a batch and picks one.  The per-pixel rule does not
depend on the tile, and each pixel blends its primitives in the same depth
order whatever the tile shape, so every candidate -- the chosen one included
-- must render the default configuration's image bit for bit (and, in alpha
mode, the same final transmittance; the stopping position is an index into
the tile-ordered list, so only whether a pixel has one is compared).  Gradients sum
the same per-pixel terms in a different grouping per tile shape, so they
agree to FP32 rounding of those sums (1e-4 relative per tensor, the bar of the
other cross-tile-shape comparisons; the derivation and the measured values,
2.3e-5 at most here, are given with test_tile_shape_and_launch_form_do_not_change_results).
"""
import numpy as np
import pytest

from helpers import rel_err, small_scene_2d, small_scene_3d, to_torch

XSHAPE_GRAD_TOL = 1e-4   # FP32 reordering across tile shapes (see test_gpu_parity)

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_2508_12615_amd import binding as B  # noqa: E402
from paper_2508_12615_amd.raster import Rasterizer, autotune, autotune_candidates  # noqa: E402


def _say(msg):
    print(msg, flush=True)


def _render(r, views, dL):
    f = r.forward(views, with_backward=True)
    g = r.backward(views, f, dL)
    torch.cuda.synchronize()
    out = dict(image=f.image.cpu().numpy())
    if f.T_final is not None:
        out["T"] = f.T_final.cpu().numpy()
        out["last"] = f.last.cpu().numpy()
    out["grads"] = [{k: v.cpu().numpy() for k, v in gi.items()} for gi in g]
    return out


def _check_all_candidates(mode, views, dL, label):
    tuner = Rasterizer(mode)
    times = autotune(tuner, views, with_backward=True, reps=1)
    cands = autotune_candidates()
    assert set(times) == set(cands) and all(t > 0.0 for t in times.values())
    best = (tuner.params.tile_w, tuner.params.tile_h, tuner.params.persistent)
    assert best in cands and times[best] == min(times.values())
    _say("%s: autotuner chose %s (%.3f ms)" % (label, best, times[best]))
    ref = _render(Rasterizer(mode), views, dL)
    worst = 0.0
    for (tw, th, pe) in cands:
        got = _render(Rasterizer(mode, tile_w=tw, tile_h=th, persistent=pe), views, dL)
        for k in ("image", "T"):
            if k in ref:
                assert np.array_equal(got[k], ref[k]), (label, (tw, th, pe), k)
        if "last" in ref:   # a position in the tile-ordered list: only whether a pixel has one is layout-free
            assert np.array_equal(got["last"] < 0, ref["last"] < 0), (label, (tw, th, pe))
        for gi, ri in zip(got["grads"], ref["grads"]):
            for k in ri:
                e = rel_err(gi[k], ri[k])
                worst = max(worst, e)
                assert e < XSHAPE_GRAD_TOL, (label, (tw, th, pe), k)
    _say("%s: worst cross-candidate gradient rel err %.2e" % (label, worst))


def test_autotune_2d_batch():
    sizes = [(200, 150, 3000), (96, 96, 800), (256, 130, 5000)]
    views = []
    for i, (W, H, n) in enumerate(sizes):
        views.append(dict(camera=(W, H), prims=to_torch(small_scene_2d(n, W, H, 600 + i))))
    npx = sum(W * H for W, H, _ in sizes)
    dL = torch.from_numpy(np.random.default_rng(3).normal(0, 1, (npx, 3)).astype(np.float32)).cuda()
    _check_all_candidates(B.WIPES_2D_ADDITIVE, views, dL, "2D")


def test_autotune_3d():
    prims, cam = small_scene_3d(6000, 240, 160, 610, 611)
    views = [dict(camera=cam, prims=to_torch(prims))]
    dL = torch.from_numpy(np.random.default_rng(4).normal(0, 1, (240 * 160, 3)).astype(np.float32)).cuda()
    _check_all_candidates(B.WIPES_3D_ALPHA, views, dL, "3D")
