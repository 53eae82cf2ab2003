"""Seeded synthetic inputs shaped like the paper's workloads.

This module only draws numbers: it holds none of the rasterizer's arithmetic
and is the one piece of code shared by the tests, the oracle harness and the
benchmark.  Every generator uses ``numpy.random.Generator(PCG64(seed))`` with
a fixed draw order, so a seed gives byte-identical arrays on any machine.

The paper's datasets (Kodak, DIV2K, Mip-NeRF360, Tanks & Temples,
DeepBlending, D-NeRF, NeRF-DS) are not available; these stand in with the
same shapes (Sec. 5.1: Kodak-sized 768x512 and DIV2K/2 408..1020 px sides;
Table 3: 0.9..2.8 M primitive scenes).
"""
from __future__ import annotations

import math

import numpy as np


def rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(int(seed)))


# --------------------------------------------------------------------------
# Targets
# --------------------------------------------------------------------------

def texture_1f(height: int, width: int, seed: int) -> np.ndarray:
    """RGB float32 [H, W, 3] texture with a 1/f amplitude spectrum.

    Per channel: complex white Gaussian noise on the rFFT grid, amplitude
    scaled by 1 / max(|k|, 1/N) with |k| in cycles per pixel, DC removed,
    inverse FFT, affine map to mean 0.5 / std 0.15, clipped to [0, 1].
    """
    g = rng(seed)
    ky = np.fft.fftfreq(height)[:, None]
    kx = np.fft.rfftfreq(width)[None, :]
    kmag = np.sqrt(kx * kx + ky * ky)
    amp = 1.0 / np.maximum(kmag, 1.0 / max(height, width))
    out = np.empty((height, width, 3), dtype=np.float32)
    for ch in range(3):
        spec = (g.standard_normal(kmag.shape) + 1j * g.standard_normal(kmag.shape)) * amp
        spec[0, 0] = 0.0
        img = np.fft.irfft2(spec, s=(height, width))
        img = (img - img.mean()) / (img.std() + 1e-12) * 0.15 + 0.5
        out[..., ch] = np.clip(img, 0.0, 1.0)
    return out


def add_stripe_patches(img: np.ndarray, n_patches: int, seed: int) -> np.ndarray:
    """Embed high-frequency stripe patches 0.5 + 0.5 cos(2 pi k.x) (all channels).

    Patch sides 64..160 px, |k| ~ U(0.25, 0.45) cycles/px at a uniform angle;
    the synthetic stand-in for the paper's moire toy images (Fig. 4).
    """
    g = rng(seed)
    H, W, _ = img.shape
    out = img.copy()
    for _ in range(n_patches):
        side = int(g.integers(64, 161))
        y0 = int(g.integers(0, max(1, H - side)))
        x0 = int(g.integers(0, max(1, W - side)))
        kmag = g.uniform(0.25, 0.45)
        ang = g.uniform(0.0, 2.0 * math.pi)
        yy, xx = np.mgrid[y0:min(H, y0 + side), x0:min(W, x0 + side)]
        val = 0.5 + 0.5 * np.cos(2.0 * math.pi * kmag * (math.cos(ang) * xx + math.sin(ang) * yy))
        out[y0:y0 + side, x0:x0 + side, :] = val[..., None].astype(np.float32)
    return out


# --------------------------------------------------------------------------
# 2D primitives (image fitting)
# --------------------------------------------------------------------------

def prims_2d(n: int, width: int, height: int, seed: int, cov: str = "rs", phase: bool = False) -> dict:
    """2D wavelet primitives in pixel units.

    Draw order: mean ~ U([0,W] x [0,H]); s1, s2 ~ logU(1, 16) px;
    theta ~ U(0, pi); |f| = 2 pi U(0, 0.5) rad/px; direction psi ~ U(0, 2 pi);
    phase0 ~ U(0, 2 pi) (always drawn; returned as "phase" only when asked
    for, since the paper's primitive has no phase term); colour ~ U(0, 1)^3;
    opacity = 1.  cov="rs" returns (s1, s2, theta); cov="cholesky" returns
    (l11, l21, l22) = (s1, t, s2) with t ~ N(0, 2^2) drawn last.
    """
    g = rng(seed)
    mean = np.stack([g.uniform(0, width, n), g.uniform(0, height, n)], 1)
    s = np.exp(g.uniform(math.log(1.0), math.log(16.0), (n, 2)))
    theta = g.uniform(0.0, math.pi, n)
    fmag = 2.0 * math.pi * g.uniform(0.0, 0.5, n)
    psi = g.uniform(0.0, 2.0 * math.pi, n)
    _phase0 = g.uniform(0.0, 2.0 * math.pi, n)
    color = g.uniform(0.0, 1.0, (n, 3))
    freq = np.stack([fmag * np.cos(psi), fmag * np.sin(psi)], 1)
    if cov == "rs":
        covp = np.stack([s[:, 0], s[:, 1], theta], 1)
    elif cov == "cholesky":
        t = g.normal(0.0, 2.0, n)
        covp = np.stack([s[:, 0], t, s[:, 1]], 1)
    else:
        raise ValueError(cov)
    out = dict(mean=mean.astype(np.float32), cov=covp.astype(np.float32), freq=freq.astype(np.float32),
               color=color.astype(np.float32), opacity=np.ones(n, np.float32))
    if phase:
        out["phase"] = _phase0.astype(np.float32)
    return out


# --------------------------------------------------------------------------
# 3D primitives and cameras (novel-view synthesis)
# --------------------------------------------------------------------------

FOCAL_1080 = 540.0 / math.tan(math.radians(25.0))   # ~1158.1 px at 1920x1080


def scene_3d(n: int, seed: int, velocity: bool = False, n_clusters: int = 64, phase: bool = False,
             sh_degree: int = -1, covector: bool = False) -> dict:
    """3D wavelet primitives inside the unit cube.

    Draw order: cluster centres U(0.1, 0.9)^3, cluster std U(0.02, 0.15);
    cluster labels uniform; means N(centre, std^2 I) with anything outside
    [0,1]^3 redrawn; scales logU(1e-3, 3e-2) per axis; quaternions N(0, I4)
    (unnormalised); opacity U(0.05, 0.99); colour U(0.05, 0.99)^3; frequency
    direction uniform on S^2 with |f| = 2 pi U(0, 0.5) * 2.5 / FOCAL_1080
    (world rad/unit; about 0..pi rad/px on screen at depth 2.5 under the
    literal transform); optional velocity N(0, 0.05^2 I3) per unit time.
    Then, each only when asked for and in this order: carrier phase
    U(0, 2 pi); spherical-harmonic coefficients [n, (deg+1)^2, 3] with the
    constant band U(0.2, 3.5) and the others N(0, 0.15^2).  covector=True
    scales |f| by (FOCAL_1080 / 2.5)^2 instead (the same 0..pi rad/px on
    screen at depth 2.5 under the phase-preserving transform).
    """
    g = rng(seed)
    centres = g.uniform(0.1, 0.9, (n_clusters, 3))
    stds = g.uniform(0.02, 0.15, n_clusters)
    lab = g.integers(0, n_clusters, n)
    mean = centres[lab] + g.standard_normal((n, 3)) * stds[lab, None]
    bad = np.any((mean < 0.0) | (mean > 1.0), axis=1)
    while bad.any():
        k = int(bad.sum())
        mean[bad] = centres[lab[bad]] + g.standard_normal((k, 3)) * stds[lab[bad], None]
        bad = np.any((mean < 0.0) | (mean > 1.0), axis=1)
    scale = np.exp(g.uniform(math.log(1e-3), math.log(3e-2), (n, 3)))
    quat = g.standard_normal((n, 4))
    opac = g.uniform(0.05, 0.99, n)
    color = g.uniform(0.05, 0.99, (n, 3))
    d = g.standard_normal((n, 3))
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    fmag = 2.0 * math.pi * g.uniform(0.0, 0.5, n) * 2.5 / FOCAL_1080
    if covector:
        fmag = fmag * (FOCAL_1080 / 2.5) ** 2
    freq = d * fmag[:, None]
    out = dict(mean=mean.astype(np.float32), quat=quat.astype(np.float32), scale=scale.astype(np.float32),
               freq=freq.astype(np.float32), color=color.astype(np.float32), opacity=opac.astype(np.float32))
    if velocity:
        out["velocity"] = (g.standard_normal((n, 3)) * 0.05).astype(np.float32)
    if phase:
        out["phase"] = g.uniform(0.0, 2.0 * math.pi, n).astype(np.float32)
    if sh_degree >= 0:
        K = (sh_degree + 1) ** 2
        sh = np.empty((n, K, 3))
        sh[:, 0, :] = g.uniform(0.2, 3.5, (n, 3))
        sh[:, 1:, :] = g.normal(0.0, 0.15, (n, K - 1, 3))
        out["sh"] = sh.astype(np.float32)
    return out


def deform_params(shapes, seed: int, head: float = 0.05) -> np.ndarray:
    """Random weights of a fully connected network, flat FP32: for each layer
    (out, in) in `shapes`, W [out, in] row-major then b [out], both
    U(-1/sqrt(in), 1/sqrt(in)) (the usual default initialisation of a linear
    layer), the last layer's scaled by `head` (small initial offsets)."""
    g = rng(seed)
    parts = []
    for l, (m, k) in enumerate(shapes):
        s = 1.0 / math.sqrt(k) * (head if l == len(shapes) - 1 else 1.0)
        parts.append(g.uniform(-s, s, m * k))
        parts.append(g.uniform(-s, s, m))
    return np.concatenate(parts).astype(np.float32)


def look_at(eye, target, up=(0.0, 0.0, 1.0)) -> np.ndarray:
    """World->camera 4x4 matrix with OpenCV axes (x right, y down, z forward)."""
    eye = np.asarray(eye, np.float64)
    z = np.asarray(target, np.float64) - eye
    z /= np.linalg.norm(z)
    x = np.cross(z, np.asarray(up, np.float64))
    x /= np.linalg.norm(x)
    y = np.cross(z, x)
    R = np.stack([x, y, z], 0)
    V = np.eye(4)
    V[:3, :3] = R
    V[:3, 3] = -R @ eye
    return V


def orbit_camera(seed: int, width: int = 1920, height: int = 1080, radius: float = 2.5, time: float = 0.0) -> dict:
    """Pinhole camera on a seeded orbit about (0.5, 0.5, 0.5).

    Draw order: azimuth U(0, 2 pi), elevation U(-30, 30) deg.  The focal length
    keeps the 1920x1080 field of view (50 deg vertical) at any resolution.
    """
    g = rng(seed)
    az = g.uniform(0.0, 2.0 * math.pi)
    el = math.radians(g.uniform(-30.0, 30.0))
    c = np.array([0.5, 0.5, 0.5])
    eye = c + radius * np.array([math.cos(el) * math.cos(az), math.cos(el) * math.sin(az), math.sin(el)])
    f = FOCAL_1080 * height / 1080.0
    return dict(width=width, height=height, fx=f, fy=f, cx=width / 2.0, cy=height / 2.0,
                viewmat=look_at(eye, c), time=float(time))


# --------------------------------------------------------------------------
# Workload configurations
# --------------------------------------------------------------------------

def config1():
    """2D fit, plain: 512x512 1/f target, 10k primitives (RS), additive."""
    return dict(target=texture_1f(512, 512, 1001), prims=prims_2d(10_000, 512, 512, 1002), width=512, height=512)


def config2():
    """2D fitting loop: 768x512 1/f texture + 8 stripe patches, 70k primitives."""
    tgt = add_stripe_patches(texture_1f(512, 768, 2001), 8, 2003)
    return dict(target=tgt, prims=prims_2d(70_000, 768, 512, 2002), width=768, height=512)


def config3(n: int = 1_000_000):
    """3D static: 1M primitives, 1920x1080 orbit camera, alpha blending."""
    return dict(prims=scene_3d(n, 3001), camera=orbit_camera(3002))


def config4_sizes(n_images: int = 64):
    """Image sizes and primitive counts of the batched-fit workload."""
    g = rng(4999)
    W = g.integers(256, 1025, n_images)
    H = g.integers(256, 1025, n_images)
    N = np.round(np.exp(g.uniform(math.log(2000), math.log(50000), n_images))).astype(np.int64)
    return [(int(W[i]), int(H[i]), int(N[i])) for i in range(n_images)]


def config4(n_images: int = 64):
    """64 uneven 2D fits: per image (W, H, N), target 4000+i, primitives 4100+i."""
    out = []
    for i, (W, H, N) in enumerate(config4_sizes(n_images)):
        out.append(dict(width=W, height=H, target=texture_1f(H, W, 4000 + i), prims=prims_2d(N, W, H, 4100 + i)))
    return out


SERVE_SCENE_SIZES = (100_000, 250_000, 500_000, 750_000, 1_000_000, 1_250_000, 1_500_000, 2_000_000)
SERVE_RESOLUTIONS = ((960, 540), (1280, 720), (1600, 900), (1920, 1080))


def serve_scene(s: int, n: int | None = None) -> dict:
    """Resident scene s of the serving workload (config-3 recipe plus velocities)."""
    return scene_3d(SERVE_SCENE_SIZES[s] if n is None else n, 5000 + s, velocity=True)


def serve_requests(n_requests: int, rate_hz: float, n_scenes: int = 8, seed_arrivals: int = 5100,
                   seed_poses: int = 5200):
    """Poisson arrivals: list of dict(t_arrive, scene, camera) with seeded poses and times."""
    ga = rng(seed_arrivals)
    gp = rng(seed_poses)
    t = np.cumsum(ga.exponential(1.0 / rate_hz, n_requests))
    reqs = []
    for k in range(n_requests):
        scene = int(gp.integers(0, n_scenes))
        W, H = SERVE_RESOLUTIONS[int(gp.integers(0, len(SERVE_RESOLUTIONS)))]
        pose_seed = int(gp.integers(0, 2**31 - 1))
        tau = float(gp.uniform(0.0, 1.0))
        reqs.append(dict(t_arrive=float(t[k]), scene=scene, camera=orbit_camera(pose_seed, W, H, time=tau)))
    return reqs


def screen_records(n: int, width: int, height: int, seed: int, dup_depth_frac: float = 0.2) -> dict:
    """Synthetic FP32 screen-space records for binning tests.

    Means U(-40, W+40) x U(-40, H+40); half-extents logU(0.05, 80) px, with
    2% marked culled (-1); depths U(0.5, 5) with a fraction copied from other
    records so that equal keys occur; some means placed exactly on tile and
    pixel-centre boundaries; then a conic (ca, cb, cc) and padded support
    threshold Qs whose support ellipse has exactly those half-extents.
    """
    g = rng(seed)
    mx = g.uniform(-40.0, width + 40.0, n)
    my = g.uniform(-40.0, height + 40.0, n)
    rx = np.exp(g.uniform(math.log(0.05), math.log(80.0), n))
    ry = np.exp(g.uniform(math.log(0.05), math.log(80.0), n))
    depth = g.uniform(0.5, 5.0, n)
    dup = g.uniform(0.0, 1.0, n) < dup_depth_frac
    depth[dup] = depth[g.integers(0, n, int(dup.sum()))]
    cull = g.uniform(0.0, 1.0, n) < 0.02
    rx[cull] = -1.0
    snap = g.uniform(0.0, 1.0, n) < 0.1
    mx[snap] = np.round(mx[snap] / 8.0) * 8.0 + 0.5 * g.integers(0, 2, int(snap.sum()))
    my[snap] = np.round(my[snap] / 8.0) * 8.0
    rx[snap & ~cull] = np.round(rx[snap & ~cull]) + 0.5
    # conic and padded support threshold consistent with the box: Q ~ U(8, 12),
    # correlation ~ U(-0.95, 0.95), variances rx^2 / Q and ry^2 / Q
    rho = g.uniform(-0.95, 0.95, n)
    Q = g.uniform(8.0, 12.0, n)
    sxx, syy = np.abs(rx) ** 2 / Q, np.abs(ry) ** 2 / Q
    sxy = rho * np.sqrt(sxx * syy)
    det = sxx * syy - sxy * sxy
    return dict(mx=mx.astype(np.float32), my=my.astype(np.float32), rx=rx.astype(np.float32),
                ry=ry.astype(np.float32), depth=depth.astype(np.float32), ca=(syy / det).astype(np.float32),
                cb=(-sxy / det).astype(np.float32), cc=(sxx / det).astype(np.float32),
                Qs=(Q * 1.001 + 1e-3).astype(np.float32))
