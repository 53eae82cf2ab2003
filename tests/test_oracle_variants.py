"""Pins of the oracle's primitive variants, each against something other than
the oracle itself: closed forms, scipy's spherical harmonics, quadrature,
reductions to the base primitive, and central finite differences of the FP64
forward.

  * covector frequency transform (the phase-preserving reading of Sec. 4.1
    after Eq. 7, where f goes through the same ray-space map as Sigma);
  * per-primitive carrier phase phi0 (Eq. 6 carries none; phi0 = 0 is the
    paper's primitive);
  * spherical-harmonic colour of degree <= 3 (Sec. 3.1: 3DGS keeps colour as
    spherical-harmonic coefficients).
"""
import math

import numpy as np
import pytest
from scipy.spatial.transform import Rotation
from scipy.special import sph_harm_y

import oracle as O
from test_oracle_pins import _check_fd, p2, p3


# ----------------------------------------------------------------------------
# Covector transform: gradients
# ----------------------------------------------------------------------------

def _alpha_scene(seed, n=6, guard=False):
    g = np.random.default_rng(seed)
    V = np.eye(4); V[:3, :3] = Rotation.from_rotvec([0.1, -0.2, 0.05]).as_matrix(); V[:3, 3] = [-0.5, -0.5, 2.0]
    cam = O.Camera(width=28, height=24, fx=30.0, fy=32.0, cx=14.0, cy=12.0, viewmat=V, time=0.4)
    prims = p3(g.uniform(0.3, 0.7, (n, 3)), g.uniform(0.3, 0.95, n), g.uniform(0.05, 0.99, (n, 3)),
               scale=g.uniform(0.03, 0.12, (n, 3)), freq=g.normal(0, 8, (n, 3)), quat=g.normal(0, 1, (n, 4)))
    prims["velocity"] = g.normal(0, 0.05, (n, 3))
    return prims, cam


def test_fd_gradients_covector():
    """Covector f' = first two entries of (J3 W)^-T f: every parameter gradient (including the
    frequency, whose gradient goes through (J3 W)^-1, and the mean, which reaches J3 through t and
    t/|t|) against central differences."""
    prims, cam = _alpha_scene(42)
    P = O.Params(mode=O.MODE_ALPHA3D, cov=O.COV_QUAT_SCALE, freq_xform=O.FREQ_COVECTOR, blur_eps=0.3,
                 bg=(0.2, 0.1, 0.4))
    _check_fd(P, prims, cam.width, cam.height, cam,
              ["mean", "quat", "scale", "freq", "color", "opacity", "velocity"], rel=2e-6)


def test_fd_gradients_covector_guard_band():
    """Covector transform on a primitive outside the guard band (clamped rows of J)."""
    cam = O.Camera(width=32, height=32, fx=20.0, fy=20.0, cx=16.0, cy=16.0, viewmat=np.eye(4))
    prims = p3([[1.9, 0.1, 1.0], [0.05, -0.05, 1.5]], [0.8, 0.7], [[0.9, 0.2, 0.1], [0.1, 0.5, 0.9]],
               scale=[[0.6, 0.2, 0.3], [0.05, 0.04, 0.06]], freq=[[1.0, -0.5, 0.3], [2.0, 1.0, -1.0]],
               quat=[[0.9, 0.1, 0.2, -0.1], [0.7, -0.3, 0.1, 0.2]])
    P = O.Params(mode=O.MODE_ALPHA3D, cov=O.COV_QUAT_SCALE, freq_xform=O.FREQ_COVECTOR, blur_eps=0.3)
    _check_fd(P, prims, 32, 32, cam, ["mean", "quat", "scale", "freq"], rel=2e-6, seed=3)


def test_covector_frequency_gradient_closed_form():
    """On the optical axis f' = (z nu_x / fx, z nu_y / fy) exactly, so dL/dnu = (z/fx g_x, z/fy g_y, 0)
    for a screen-space frequency gradient g (no other screen gradient)."""
    cam = O.Camera(width=64, height=48, fx=500.0, fy=420.0, cx=32.0, cy=24.0, viewmat=np.eye(4))
    z = 3.0
    prims = p3([[0, 0, z]], [0.8], [[1, 1, 1]], scale=[[0.02, 0.05, 0.03]], freq=[[1.5, -2.0, 0.7]])
    P = O.Params(mode=O.MODE_ALPHA3D, cov=O.COV_QUAT_SCALE, freq_xform=O.FREQ_COVECTOR)
    scr = O.project(P, prims, cam)
    ds = np.zeros((1, O.SG_N)); ds[0, O.SG["fx"]] = 0.7; ds[0, O.SG["fy"]] = -1.3
    pg = O.project_bwd(P, prims, scr, ds, cam)
    assert np.allclose(pg["freq"][0], [z / 500 * 0.7, z / 420 * -1.3, 0.0], rtol=1e-12, atol=1e-15)


# ----------------------------------------------------------------------------
# Carrier phase
# ----------------------------------------------------------------------------

@pytest.mark.parametrize("phi0", [0.0, 0.9, 2.5, -1.7])
def test_phase_pixel_sum_closed_form(phi0):
    """Sum over pixels of W' with phase: pi sqrt(det S) (1 + cos(phi0) exp(-f^T S f / 2)) -- the
    integral of (1 + cos(f.d + phi0)) G / 2, whose sine part vanishes by symmetry -- and its phase
    derivative -pi sqrt(det S) sin(phi0) exp(-f^T S f / 2), from the backward of the sum."""
    S = np.array([[16.0, 5.0], [5.0, 9.0]])
    L = np.linalg.cholesky(S)
    f = np.array([0.6, -0.45])
    prims = p2([[80.3, 79.6]], [[L[0, 0], L[1, 0], L[1, 1]]], [f])
    prims["phase"] = np.array([phi0])
    P = O.Params(mode=O.MODE_ADD2D, cov=O.COV_CHOLESKY, q_add=50.0)
    scr = O.project(P, prims)
    img, _, _, _ = O.render_o1(P, 160, 160, scr)
    env = math.exp(-0.5 * f @ S @ f)
    want = math.pi * math.sqrt(np.linalg.det(S)) * (1 + math.cos(phi0) * env)
    assert abs(img[:, 0].sum() - want) < 1e-6 * want
    g = np.zeros((160 * 160, 3)); g[:, 0] = 1.0
    ds = O.render_bwd_o1(P, 160, 160, scr, g)
    dwant = -math.pi * math.sqrt(np.linalg.det(S)) * math.sin(phi0) * env
    assert abs(ds[0, O.SG["phase"]] - dwant) < 1e-6 * math.pi * math.sqrt(np.linalg.det(S))
    pg = O.project_bwd(P, prims, scr, ds)
    assert pg["phase"][0] == ds[0, O.SG["phase"]]


def test_phase_pointwise_at_mean():
    """W'(mu') = (1 + cos phi0) / 2: one primitive whose mean sits on a pixel centre, with colour 1."""
    for phi0 in (0.0, 1.0, math.pi):
        prims = p2([[10.5, 7.5]], [[3.0, 0.0, 2.0]], [[0.4, 0.2]])
        prims["phase"] = np.array([phi0])
        P = O.Params(mode=O.MODE_ADD2D, cov=O.COV_CHOLESKY)
        img, _, _, _ = O.render_o1(P, 21, 15, O.project(P, prims), pix=[7 * 21 + 10])
        assert abs(img[0, 0] - 0.5 * (1 + math.cos(phi0))) < 1e-15


def test_phase_pointwise_formula():
    """Every pixel of one additive primitive with a phase equals o c e(p) (1 + cos(f.(p - mu) + phi0)) / 2
    inside q <= 9, written out in numpy from a hand-inverted covariance (catches a phase added to the
    wrong term, or scaled)."""
    W, H = 24, 20
    prims = p2([[11.2, 9.7]], [[4.0, 1.0, 3.0]], [[0.7, -0.4]], opac=[0.6], color=[[0.3, 0.8, 0.5]])
    prims["phase"] = np.array([0.77])
    P = O.Params(mode=O.MODE_ADD2D, cov=O.COV_CHOLESKY)
    scr = O.project(P, prims)
    img, _, _, _ = O.render_o1(P, W, H, scr)
    Sg = np.array([[16.0, 4.0], [4.0, 10.0]])
    A = np.linalg.inv(Sg)
    ys, xs = np.mgrid[0:H, 0:W]
    d = np.stack([xs + 0.5 - 11.2, ys + 0.5 - 9.7], -1)
    q = np.einsum("...i,ij,...j->...", d, A, d)
    w = 0.5 * (1 + np.cos(d @ np.array([0.7, -0.4]) + 0.77)) * np.exp(-0.5 * q)
    want = np.where(q <= 9.0, 0.6 * w, 0.0)
    assert np.max(np.abs(img[:, 1].reshape(H, W) - 0.8 * want)) < 1e-14


def test_fd_gradients_phase_additive():
    g = np.random.default_rng(7)
    n = 5
    prims = p2(np.stack([g.uniform(4, 26, n), g.uniform(4, 22, n)], 1),
               np.stack([g.uniform(2, 5, n), g.normal(0, 1, n), g.uniform(2, 5, n)], 1), g.normal(0, 1.0, (n, 2)),
               color=g.uniform(0, 1, (n, 3)), opac=g.uniform(0.4, 1, n))
    prims["phase"] = g.uniform(-math.pi, math.pi, n)
    P = O.Params(mode=O.MODE_ADD2D, cov=O.COV_CHOLESKY)
    _check_fd(P, prims, 30, 26, None, ["mean", "cov", "freq", "phase", "color", "opacity"], rel=1e-6)


def test_fd_gradients_phase_alpha():
    prims, cam = _alpha_scene(42)
    prims["phase"] = np.random.default_rng(9).uniform(-math.pi, math.pi, 6)   # a tie-free draw
    P = O.Params(mode=O.MODE_ALPHA3D, cov=O.COV_QUAT_SCALE, blur_eps=0.3, bg=(0.2, 0.1, 0.4))
    _check_fd(P, prims, cam.width, cam.height, cam, ["phase", "mean", "freq", "opacity"], rel=2e-6)


# ----------------------------------------------------------------------------
# Spherical-harmonic colour
# ----------------------------------------------------------------------------

def _real_sh_scipy(l, m, dirs):
    """Real SH with the Condon-Shortley phase from scipy's complex harmonics (CS phase included):
    sqrt(2) Re Y_l^m (m > 0), sqrt(2) Im Y_l^|m| (m < 0), Y_l^0 (m = 0)."""
    x, y, z = dirs[:, 0], dirs[:, 1], dirs[:, 2]
    theta = np.arccos(np.clip(z, -1, 1))
    phi = np.arctan2(y, x)
    Y = sph_harm_y(l, abs(m), theta, phi)
    if m > 0:
        return math.sqrt(2) * Y.real
    if m < 0:
        return math.sqrt(2) * Y.imag
    return Y.real


def test_sh_basis_matches_scipy():
    g = np.random.default_rng(3)
    dirs = g.normal(0, 1, (400, 3))
    dirs /= np.linalg.norm(dirs, axis=1, keepdims=True)
    Y, _ = O.sh_basis(3, dirs)
    for l in range(4):
        for m in range(-l, l + 1):
            k = l * l + l + m
            assert np.max(np.abs(Y[:, k] - _real_sh_scipy(l, m, dirs))) < 1e-13, (l, m)


def test_sh_basis_orthonormal():
    """Gauss-Legendre in cos(theta) x uniform azimuth integrates the degree <= 6 products exactly."""
    xg, wg = np.polynomial.legendre.leggauss(12)
    nphi = 24
    phi = (np.arange(nphi) + 0.5) * 2 * math.pi / nphi
    ct, ph = np.meshgrid(xg, phi, indexing="ij")
    st = np.sqrt(1 - ct ** 2)
    dirs = np.stack([st * np.cos(ph), st * np.sin(ph), ct], -1).reshape(-1, 3)
    w = (wg[:, None] * np.full(nphi, 2 * math.pi / nphi)[None, :]).reshape(-1)
    Y, _ = O.sh_basis(3, dirs)
    G = (Y * w[:, None]).T @ Y
    assert np.max(np.abs(G - np.eye(16))) < 1e-12


def test_sh_polynomial_gradients():
    g = np.random.default_rng(4)
    dirs = g.normal(0, 1, (50, 3))
    dirs /= np.linalg.norm(dirs, axis=1, keepdims=True)
    _, G = O.sh_basis(3, dirs)
    # the polynomials extend off the sphere; central differences of that extension
    for a in range(3):
        e = np.zeros(3); e[a] = 1e-6
        Yp, _ = O.sh_basis(3, dirs + e)
        Ym, _ = O.sh_basis(3, dirs - e)
        assert np.max(np.abs((Yp - Ym) / 2e-6 - G[:, :, a])) < 1e-8


def test_sh_degree0_is_direct_rgb():
    """Degree 0 with sh0 = c / Y_00 renders exactly the direct-RGB image (no view dependence)."""
    prims, cam = _alpha_scene(11, n=20)
    Y00 = 0.5 / math.sqrt(math.pi)
    prims_sh = dict(prims)
    prims_sh["sh"] = (np.asarray(prims["color"]) / Y00)[:, None, :]
    P = O.Params(mode=O.MODE_ALPHA3D, cov=O.COV_QUAT_SCALE, blur_eps=0.3)
    Psh = O.Params(mode=O.MODE_ALPHA3D, cov=O.COV_QUAT_SCALE, blur_eps=0.3, sh_degree=0)
    i0, _, _, _ = O.render_o1(P, cam.width, cam.height, O.project(P, prims, cam), O.depth_keys(prims, cam))
    i1, _, _, _ = O.render_o1(Psh, cam.width, cam.height, O.project(Psh, prims_sh, cam), O.depth_keys(prims, cam))
    assert np.max(np.abs(i0 - i1)) < 1e-14


def test_sh_colour_is_direction_from_camera_centre():
    """Degree 1, coefficient only on Y_10 = sqrt(3/4pi) z: a primitive straight ahead of a camera
    looking down world +z has colour sqrt(3/4pi) * coefficient (direction (0, 0, 1)); moving the
    camera centre to the side changes the direction to the normalised offset."""
    K = 4
    sh = np.zeros((1, K, 3)); sh[0, 2, :] = [0.5, 1.0, 2.0]
    for cpos in ([0.0, 0.0, 0.0], [0.3, -0.2, 0.0]):
        V = np.eye(4); V[:3, 3] = -np.array(cpos)          # camera centre at cpos, axes aligned
        cam = O.Camera(width=16, height=16, fx=20.0, fy=20.0, cx=8.0, cy=8.0, viewmat=V)
        prims = p3([[0.0, 0.0, 2.0]], [0.9], [[0, 0, 0]], scale=[[0.05, 0.05, 0.05]], freq=[[0, 0, 0]])
        prims["sh"] = sh
        P = O.Params(mode=O.MODE_ALPHA3D, cov=O.COV_QUAT_SCALE, sh_degree=1)
        scr = O.project(P, prims, cam)[0]
        d = np.array([0.0, 0.0, 2.0]) - cpos
        zc = d[2] / np.linalg.norm(d)
        assert np.allclose(scr[[8, 9, 10]], math.sqrt(3 / (4 * math.pi)) * zc * np.array([0.5, 1.0, 2.0]),
                           rtol=1e-14)


@pytest.mark.parametrize("deg", [1, 3])
def test_fd_gradients_sh(deg):
    """Every gradient of an SH-coloured scene, including the mean's view-direction term, against
    central differences."""
    prims, cam = _alpha_scene(42)
    K = (deg + 1) ** 2
    prims["sh"] = np.random.default_rng(9).normal(0, 0.6, (6, K, 3))
    P = O.Params(mode=O.MODE_ALPHA3D, cov=O.COV_QUAT_SCALE, blur_eps=0.3, bg=(0.2, 0.1, 0.4), sh_degree=deg)
    # the loss is linear in sh, so the FD error there is pure rounding of the small steps the
    # near-zero coefficients get (h = 1e-8): 1e-5 still fails any wrong basis function or sign by O(1)
    _check_fd(P, prims, cam.width, cam.height, cam, ["sh", "mean", "velocity", "quat", "opacity"], rel=1e-5)
