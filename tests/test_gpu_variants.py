"""Primitive variants on the HIP path against the FP64 oracle, through the C ABI:

* the carrier phase phi0 (the carrier cos(f'.(x - mu') + phi0); Eq. 6 has
  none, so phi0 = 0 is the paper's primitive), both blend modes;
* the phase-preserving (covector) frequency transform f' = rows 0-1 of
  (J3 W)^-T f, beside the literal f' = J W f of Sec. 4.1;
* spherical-harmonic colour of degree 0..3 at the view direction (Sec. 3.1),
  gradients to the coefficients and to the mean through the direction.

Bars as everywhere: 1e-4 max-abs on non-tie pixels, tie pixels within their
jump bound, gradients 1e-3 relative per tensor with the upstream gradient
zeroed on tie pixels.
"""
import numpy as np
import pytest

import oracle as O
from helpers import compare_image, oracle_camera, oracle_params, rel_err, sanitize_dLdC, small_scene_3d, to_torch

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_2508_12615_amd import binding as B  # noqa: E402
from paper_2508_12615_amd import synth  # noqa: E402
from paper_2508_12615_amd.raster import Rasterizer  # noqa: E402


def _say(msg):
    print(msg, flush=True)


def test_phase_2d_additive():
    W, H, n = 120, 96, 600
    prims = synth.prims_2d(n, W, H, 41, phase=True)
    tp = to_torch(prims)
    r = Rasterizer(B.WIPES_2D_ADDITIVE)
    f = r.forward([dict(camera=(W, H), prims=tp)], with_backward=True)
    P = oracle_params(O.MODE_ADD2D, O.COV_RS)
    scr = O.project(P, prims)
    ref, _, _, tie, jb = O.render_o1(P, W, H, scr, jump=True)
    worst, nt = compare_image(f.image.cpu().numpy(), ref, tie, jb)
    # the phase matters: the same primitives without it render differently
    scr0 = O.project(P, {k: v for k, v in prims.items() if k != "phase"})
    ref0 = O.render_o1(P, W, H, scr0)[0]
    assert np.abs(ref0 - ref).max() > 0.1
    g = sanitize_dLdC(np.random.default_rng(7).normal(0, 1, (H * W, 3)), tie).astype(np.float32)
    grads, ds = r.backward([dict(camera=(W, H), prims=tp)], f, torch.from_numpy(g).cuda(), want_dscreen=True)
    ds_ref = O.render_bwd_o1(P, W, H, scr, g.astype(np.float64))
    assert rel_err(ds.cpu().numpy()[:, 11], ds_ref[:, 11]) < 1e-3
    pg = O.project_bwd(P, prims, scr, ds_ref)
    for k in ("mean", "cov", "freq", "color", "opacity", "phase"):
        assert rel_err(grads[0][k].cpu().numpy(), pg[k]) < 1e-3, k
    _say("phase 2D: max-abs %.2e, %d ties" % (worst, nt))


def _check_3d(prims, cam, bg=(0.0, 0.0, 0.0), keys_grad=("mean", "quat", "scale", "freq", "color", "opacity"),
              seed=8, **variant):
    W, H = cam["width"], cam["height"]
    tp = to_torch(prims)
    if variant.get("sh_degree", -1) >= 0:
        del tp["color"]                   # the colour comes from the coefficients
    r = Rasterizer(B.WIPES_3D_ALPHA, bg=bg, **variant)
    f = r.forward([dict(camera=cam, prims=tp)], with_backward=True)
    P = oracle_params(O.MODE_ALPHA3D, O.COV_QUAT_SCALE, bg=bg, **variant)
    ocam = oracle_camera(cam)
    scr = O.project(P, prims, ocam)
    keys = O.depth_keys(prims, ocam)
    ref, T, nc, tie, jb = O.render_o1(P, W, H, scr, keys, jump=True)
    worst, nt = compare_image(f.image.cpu().numpy(), ref, tie, jb, T_gpu=f.T_final.cpu().numpy(), T_ref=T)
    g = sanitize_dLdC(np.random.default_rng(seed).normal(0, 1, (H * W, 3)), tie).astype(np.float32)
    grads = r.backward([dict(camera=cam, prims=tp)], f, torch.from_numpy(g).cuda())[0]
    ds = O.render_bwd_o1(P, W, H, scr, g.astype(np.float64), keys)
    pg = O.project_bwd(P, prims, scr, ds, ocam)
    errs = {k: rel_err(grads[k].cpu().numpy(), pg[k]) for k in keys_grad}
    assert all(e < 1e-3 for e in errs.values()), errs
    return ref, worst, nt, errs


def test_phase_3d_alpha():
    prims, cam = small_scene_3d(3000, 192, 144, 3301, 3302, velocity=True, time=0.3, phase=True)
    ref, worst, nt, errs = _check_3d(prims, cam, bg=(0.1, 0.2, 0.3),
                                     keys_grad=("mean", "quat", "scale", "freq", "color", "opacity", "phase",
                                                "velocity"))
    _say("phase 3D: max-abs %.2e, %d ties, %s" % (worst, nt, errs))


@pytest.mark.parametrize("phase", [False, True])
def test_covector_3d(phase):
    prims, cam = small_scene_3d(3000, 192, 144, 3401, 3402, phase=phase, covector=True)
    # the same on-screen carrier at this resolution: f' scales as f / focal under the covector map
    prims["freq"] = (prims["freq"] * (cam["height"] / 1080.0)).astype(np.float32)
    names = ("mean", "quat", "scale", "freq", "color", "opacity") + (("phase",) if phase else ())
    ref, worst, nt, errs = _check_3d(prims, cam, keys_grad=names, freq_xform=B.WIPES_FREQ_COVECTOR)
    _say("covector%s: max-abs %.2e, %d ties, %s" % (" + phase" if phase else "", worst, nt, errs))


def test_covector_differs_from_vector():
    """Off the optical axis the two transforms give different f', hence different images."""
    prims, cam = small_scene_3d(2000, 96, 64, 3501, 3502, covector=True)
    prims["freq"] = (prims["freq"] * (cam["height"] / 1080.0)).astype(np.float32)
    ocam = oracle_camera(cam)
    rv = Rasterizer(B.WIPES_3D_ALPHA)
    rc = Rasterizer(B.WIPES_3D_ALPHA, freq_xform=B.WIPES_FREQ_COVECTOR)
    tp = to_torch(prims)
    iv = rv.forward([dict(camera=cam, prims=tp)]).image.cpu().numpy()
    ic = rc.forward([dict(camera=cam, prims=tp)]).image.cpu().numpy()
    assert np.abs(iv - ic).max() > 0.05
    P = oracle_params(O.MODE_ALPHA3D, O.COV_QUAT_SCALE, freq_xform=O.FREQ_COVECTOR)
    ref, T, nc, tie, jb = O.render_o1(P, cam["width"], cam["height"], O.project(P, prims, ocam),
                                      O.depth_keys(prims, ocam), jump=True)
    compare_image(ic, ref, tie, jb)


@pytest.mark.parametrize("deg", [0, 1, 2, 3])
def test_sh_colour(deg):
    prims, cam = small_scene_3d(3000, 192, 144, 3600 + deg, 3610 + deg, velocity=True, time=0.6, sh_degree=deg)
    ref, worst, nt, errs = _check_3d(prims, cam, keys_grad=("mean", "quat", "scale", "freq", "opacity", "sh",
                                                            "velocity"), sh_degree=deg)
    _say("SH degree %d: max-abs %.2e, %d ties, %s" % (deg, worst, nt, errs))


def test_all_variants_together():
    prims, cam = small_scene_3d(4000, 224, 160, 3701, 3702, velocity=True, time=0.8, phase=True, sh_degree=3,
                                covector=True)
    prims["freq"] = (prims["freq"] * (cam["height"] / 1080.0)).astype(np.float32)
    ref, worst, nt, errs = _check_3d(prims, cam, bg=(0.3, 0.3, 0.3),
                                     keys_grad=("mean", "quat", "scale", "freq", "opacity", "phase", "sh",
                                                "velocity"),
                                     sh_degree=3, freq_xform=B.WIPES_FREQ_COVECTOR)
    _say("covector + phase + SH3 + motion: max-abs %.2e, %d ties, %s" % (worst, nt, errs))


def test_sh_degree0_equals_direct_rgb():
    """SH degree 0 with coefficients c / Y00 renders the same image as direct RGB c (to FP32
    rounding of the coefficient scaling)."""
    prims, cam = small_scene_3d(2000, 96, 64, 3801, 3802)
    y00 = 0.5 / np.sqrt(np.pi)
    sh = (prims["color"].astype(np.float64) / y00)[:, None, :].astype(np.float32)
    tp = to_torch(prims)
    r0 = Rasterizer(B.WIPES_3D_ALPHA)
    rs = Rasterizer(B.WIPES_3D_ALPHA, sh_degree=0)
    ps = dict(tp)
    del ps["color"]
    ps["sh"] = torch.from_numpy(sh).cuda()
    a = r0.forward([dict(camera=cam, prims=tp)]).image
    b = rs.forward([dict(camera=cam, prims=ps)]).image
    assert float((a - b).abs().max()) < 1e-5


def test_variant_arguments_validated():
    r = Rasterizer(B.WIPES_3D_ALPHA, sh_degree=2)
    prims, cam = small_scene_3d(100, 32, 32, 1, 2)
    with pytest.raises(B.WipesError):   # SH colour without coefficients
        r.forward([dict(camera=cam, prims=to_torch(prims))])
    with pytest.raises(B.WipesError):   # SH colour is 3D only
        Rasterizer(B.WIPES_2D_ADDITIVE, sh_degree=0).forward(
            [dict(camera=(32, 32), prims=to_torch(synth.prims_2d(10, 32, 32, 3)))])
