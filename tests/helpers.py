"""Shared helpers of the test suite: the same seeded inputs fed to the HIP
path and to the FP64 oracle, plus tie-aware comparisons."""
from __future__ import annotations

import math

import numpy as np

import oracle as O

F32 = lambda x: float(np.float32(x))  # noqa: E731


def oracle_params(mode, cov, **kw):
    """Oracle constants equal to the library defaults rounded to FP32 (the
    library holds them in FP32, so both sides test the same thresholds)."""
    three_d = mode == O.MODE_ALPHA3D
    p = O.Params(mode=mode, cov=cov, alpha_min=F32(1.0 / 255.0), alpha_max=F32(0.99), T_min=F32(1e-4),
                 q_add=F32(9.0), blur_eps=F32(0.3) if three_d else 0.0, near_plane=F32(0.01),
                 fov_guard=F32(1.3), bg=(0.0, 0.0, 0.0))
    for k, v in kw.items():
        setattr(p, k, tuple(F32(x) for x in v) if k == "bg" else F32(v) if isinstance(v, float) else v)
    return p


def oracle_camera(cam: dict) -> O.Camera:
    vm = np.asarray(cam["viewmat"], np.float32).astype(np.float64)
    return O.Camera(width=int(cam["width"]), height=int(cam["height"]), fx=F32(cam["fx"]), fy=F32(cam["fy"]),
                    cx=F32(cam["cx"]), cy=F32(cam["cy"]), viewmat=vm, time=F32(cam.get("time", 0.0)))


def to_torch(prims: dict, device="cuda"):
    import torch
    return {k: torch.from_numpy(np.ascontiguousarray(v, dtype=np.float32)).to(device) for k, v in prims.items()}


def compare_image(gpu, ref, tie, jump, tol=1e-4, max_tie_frac=1e-3, min_tie_allow=2, T_gpu=None, T_ref=None):
    """Tie protocol.  A pixel is a tie pixel when one of its decisions (support, skip, stop, clamp,
    cull) lies within the stated margin of its threshold; the oracle flags it and bounds how far the
    pixel can move if that decision goes the other way (jump[:, 0] for the colour, jump[:, 1] for the
    final transmittance).  Non-tie pixels: max-abs error over the channels <= tol.  Tie pixels: error
    <= jump + tol.  The number of tie pixels is at most max_tie_frac of the pixels (at least
    min_tie_allow are allowed).  With T_gpu/T_ref the final transmittance is held to the same rule.
    Returns (worst non-tie error, tie pixel count)."""
    gpu = np.asarray(gpu, np.float64).reshape(-1, 3)
    ref = np.asarray(ref, np.float64).reshape(-1, 3)
    tie = np.asarray(tie).reshape(-1)
    jump = np.asarray(jump, np.float64).reshape(-1, 2)
    err = np.abs(gpu - ref).max(axis=1)
    ok = tie == 0
    worst = float(err[ok].max()) if ok.any() else 0.0
    n_tie = int((~ok).sum())
    assert worst <= tol, "max-abs error %.3g > %.3g at pixel %d" % (worst, tol, int(np.argmax(np.where(ok, err, 0))))
    over = np.flatnonzero(~ok & (err > jump[:, 0] + tol))
    assert over.size == 0, "tie pixel %d: error %.3g above its jump bound %.3g + %.3g" % (
        over[0], err[over[0]], jump[over[0], 0], tol)
    assert n_tie <= max(min_tie_allow, max_tie_frac * tie.size), "too many tie pixels: %d of %d" % (n_tie, tie.size)
    if T_gpu is not None:
        eT = np.abs(np.asarray(T_gpu, np.float64).reshape(-1) - np.asarray(T_ref, np.float64).reshape(-1))
        assert float(eT[ok].max(initial=0.0)) <= tol, "T_final error %.3g" % float(eT[ok].max())
        assert np.all(eT[~ok] <= jump[~ok, 1] + tol), "T_final error above the jump bound on a tie pixel"
    return worst, n_tie


def rel_err(a, b):
    """max|a - b| / max|b| (per tensor)."""
    a = np.asarray(a, np.float64)
    b = np.asarray(b, np.float64)
    den = max(float(np.abs(b).max()), 1e-30)
    return float(np.abs(a - b).max()) / den


def small_scene_2d(n, W, H, seed, cov="rs"):
    from paper_2508_12615_amd import synth
    return synth.prims_2d(n, W, H, seed, cov=cov)


def small_scene_3d(n, W, H, seed_scene, seed_cam, velocity=False, time=0.0, **variants):
    """Config-3 recipe at reduced size: a unit-cube cluster scene and an orbit camera
    (variants: phase, sh_degree, covector as synth.scene_3d)."""
    from paper_2508_12615_amd import synth
    prims = synth.scene_3d(n, seed_scene, velocity=velocity, **variants)
    cam = synth.orbit_camera(seed_cam, W, H, time=time)
    # keep the 3D test scenes visually dense at low resolution: scale up the splats
    prims["scale"] = (prims["scale"] * 1080.0 / H * 0.5).astype(np.float32)
    return prims, cam


def sanitize_dLdC(dL, tie):
    """Zero the upstream gradient on tie pixels (their gradients are not unique)."""
    dL = np.array(dL, np.float64).reshape(-1, 3)
    dL[np.asarray(tie).reshape(-1) != 0] = 0.0
    return dL


def near_tile_boundary(v, t, eps=1e-5):
    x = np.asarray(v, np.float64) / t
    return np.abs(x - np.round(x)) < eps


__all__ = ["oracle_params", "oracle_camera", "to_torch", "compare_image", "rel_err", "small_scene_2d",
           "small_scene_3d", "sanitize_dLdC", "F32", "math"]
