"""Pins of the FP64 oracle against what the paper and the mathematics fix.

Nothing here compares the oracle with itself: every expected value comes
from a closed form (Poisson summation of the wavelet, Appendix-style
compositing identities), a library routine (scipy Gaussians, scipy rotations,
numpy stable sort), finite differences of the oracle's own forward, or a brute
force enumeration.  Each test names the mistake it is there to catch.
"""
import math

import numpy as np
import pytest
from scipy.spatial.transform import Rotation
from scipy.stats import multivariate_normal

import oracle as O


def p2(mean, cov, freq, color=None, opac=None):
    n = len(mean)
    return dict(mean=np.asarray(mean, float), cov=np.asarray(cov, float), freq=np.asarray(freq, float),
                color=np.asarray(color if color is not None else [[1.0, 0.0, 0.0]] * n, float),
                opacity=np.asarray(opac if opac is not None else [1.0] * n, float))


def gaussian_env(d, Sigma):
    """exp(-1/2 d^T Sigma^-1 d) through scipy's normal pdf (library routine)."""
    return multivariate_normal(mean=np.zeros(2), cov=Sigma).pdf(d) * 2.0 * math.pi * math.sqrt(np.linalg.det(Sigma))


# ----------------------------------------------------------------------------
# Closed forms of the 2D wavelet (Eq. 6-7) and additive blending (Eq. 4)
# ----------------------------------------------------------------------------

@pytest.mark.parametrize("theta", [0.0, 0.7])
def test_pixel_sum_matches_poisson_closed_form(theta):
    """sum_p W'(p) = pi sqrt(det Sigma) (1 + exp(-f^T Sigma f / 2)) for an untruncated,
    well-sampled wavelet (aliasing <= exp(-(2 pi - |f|)^2 sigma^2 / 2)).
    Catches: a dropped 1/2, cos vs 1+cos, conic not the inverse, wrong pixel centre."""
    s1, s2, f = 3.0, 4.5, np.array([1.1, -0.7])
    R = np.array([[math.cos(theta), -math.sin(theta)], [math.sin(theta), math.cos(theta)]])
    Sigma = R @ np.diag([s1 * s1, s2 * s2]) @ R.T
    P = O.Params(mode=O.MODE_ADD2D, cov=O.COV_RS, q_add=50.0)
    prims = p2([[80.3, 79.6]], [[s1, s2, theta]], [f], color=[[0.7, 0.0, 0.0]], opac=[0.9])
    scr = O.project(P, prims)
    img, _, _, _ = O.render_o1(P, 160, 160, scr)
    expect = 0.7 * 0.9 * math.pi * math.sqrt(np.linalg.det(Sigma)) * (1.0 + math.exp(-0.5 * f @ Sigma @ f))
    assert abs(img[:, 0].sum() - expect) < 1e-9 * expect
    assert np.all(img[:, 1:] == 0.0)


def test_pixel_sum_gradient_closed_form():
    """d/df' sum_p c o W' = -c o pi sqrt(det Sigma) exp(-f^T Sigma f/2) Sigma f, d/dmu' = 0,
    and d/d(conic) equals the derivative of the closed form in (a, b, c).
    Catches: sign of the carrier derivative, the 2b factor, a transposed conic gradient."""
    s1, s2, th, f = 3.2, 4.1, 0.4, np.array([0.9, 0.6])
    R = np.array([[math.cos(th), -math.sin(th)], [math.sin(th), math.cos(th)]])
    Sigma = R @ np.diag([s1 * s1, s2 * s2]) @ R.T
    P = O.Params(mode=O.MODE_ADD2D, cov=O.COV_RS, q_add=50.0)
    prims = p2([[70.2, 69.9]], [[s1, s2, th]], [f], color=[[1.0, 0.0, 0.0]], opac=[1.0])
    scr = O.project(P, prims)
    W = H = 140
    g = np.zeros((W * H, 3)); g[:, 0] = 1.0
    ds = O.render_bwd_o1(P, W, H, scr, g)[0]
    amp = math.pi * math.sqrt(np.linalg.det(Sigma))
    df = -amp * math.exp(-0.5 * f @ Sigma @ f) * (Sigma @ f)
    assert np.allclose(ds[[O.SG["fx"], O.SG["fy"]]], df, rtol=1e-8, atol=1e-10)
    assert np.all(np.abs(ds[[O.SG["mx"], O.SG["my"]]]) < 1e-8)

    def closed(a, b, c):
        A = np.array([[a, b], [b, c]])
        S = np.linalg.inv(A)
        return math.pi * math.sqrt(np.linalg.det(S)) * (1.0 + math.exp(-0.5 * f @ S @ f))

    A = np.linalg.inv(Sigma)
    abc = [A[0, 0], A[0, 1], A[1, 1]]
    for k, col in enumerate(["ca", "cb", "cc"]):
        h = 1e-6 * abs(abc[k]) + 1e-9
        up = list(abc); dn = list(abc)
        up[k] += h; dn[k] -= h
        fd = (closed(*up) - closed(*dn)) / (2 * h)
        assert abs(ds[O.SG[col]] - fd) < 1e-5 * abs(fd) + 1e-8, col
    # opacity and colour: d/do = sum W', d/dc_r = o sum W'
    total = amp * (1.0 + math.exp(-0.5 * f @ Sigma @ f))
    assert abs(ds[O.SG["op"]] - total) < 1e-8 * total
    assert abs(ds[O.SG["r"]] - total) < 1e-8 * total


def test_wavelet_pointwise_identities():
    """W'(mu') = 1; W' = G' along d perpendicular to f; W' = 0 where f.d = pi; 0 <= W' <= G'.
    Catches: phase measured from the wrong origin, missing +1, carrier on the envelope."""
    s1, s2, th = 2.5, 4.0, 0.3
    R = np.array([[math.cos(th), -math.sin(th)], [math.sin(th), math.cos(th)]])
    Sigma = R @ np.diag([s1 * s1, s2 * s2]) @ R.T
    mu = np.array([20.5, 18.5])        # a pixel centre
    f = np.array([math.pi / 3.0, 0.0])  # f.d = pi at dx = 3
    P = O.Params(mode=O.MODE_ADD2D, cov=O.COV_RS, q_add=1e9)
    prims = p2([mu], [[s1, s2, th]], [f])
    scr = O.project(P, prims)
    W, H = 41, 40
    img, _, _, _ = O.render_o1(P, W, H, scr)
    val = img[:, 0].reshape(H, W)
    assert abs(val[18, 20] - 1.0) < 1e-15
    assert abs(val[18, 23]) < 1e-15 and abs(val[18, 17]) < 1e-15
    for dy in (-5, -2, 1, 4, 7):
        d = np.array([0.0, float(dy)])
        assert abs(val[18 + dy, 20] - gaussian_env(d, Sigma)) < 1e-12
    ys, xs = np.mgrid[0:H, 0:W]
    d = np.stack([xs + 0.5 - mu[0], ys + 0.5 - mu[1]], -1).reshape(-1, 2)
    G = multivariate_normal(mean=np.zeros(2), cov=Sigma).pdf(d) * 2 * math.pi * math.sqrt(np.linalg.det(Sigma))
    assert np.all(val.reshape(-1) >= -1e-15) and np.all(val.reshape(-1) <= G + 1e-15)


def test_zero_frequency_is_gaussian_image():
    """f = 0 turns every wavelet into its Gaussian (Sec. 4.1), so the additive image is
    sum c o G' over q <= 9, with G' and q from scipy.  Catches: a wrong support test,
    a wrong Cholesky assembly, colour/opacity mixed up."""
    g = np.random.default_rng(7)
    n, W, H = 6, 48, 40
    mean = np.stack([g.uniform(5, 43, n), g.uniform(5, 35, n)], 1)
    L = [np.array([[g.uniform(1.5, 4), 0.0], [g.normal(0, 1.5), g.uniform(1.5, 4)]]) for _ in range(n)]
    covp = [[l[0, 0], l[1, 0], l[1, 1]] for l in L]
    color = g.uniform(0, 1, (n, 3)); opac = g.uniform(0.3, 1.0, n)
    P = O.Params(mode=O.MODE_ADD2D, cov=O.COV_CHOLESKY)
    scr = O.project(P, p2(mean, covp, np.zeros((n, 2)), color, opac))
    img, _, _, _ = O.render_o1(P, W, H, scr)
    ys, xs = np.mgrid[0:H, 0:W]
    pts = np.stack([xs + 0.5, ys + 0.5], -1).reshape(-1, 2)
    ref = np.zeros((W * H, 3))
    for i in range(n):
        S = L[i] @ L[i].T
        d = pts - mean[i]
        Gi = gaussian_env(d, S)
        q = np.einsum("pi,ij,pj->p", d, np.linalg.inv(S), d)
        ref += (Gi * (q <= 9.0))[:, None] * color[i] * opac[i]
    assert np.max(np.abs(img - ref)) < 1e-12


def test_additive_is_permutation_invariant_and_linear():
    """Eq. 4 is a plain sum: shuffling primitives changes nothing beyond rounding and
    render(A u B) = render(A) + render(B).  Catches: order-dependent state in the additive path."""
    g = np.random.default_rng(3)
    n, W, H = 40, 64, 48
    prims = dict(mean=np.stack([g.uniform(0, W, n), g.uniform(0, H, n)], 1),
                 cov=np.stack([g.uniform(1, 6, n), g.uniform(1, 6, n), g.uniform(0, math.pi, n)], 1),
                 freq=g.normal(0, 1, (n, 2)), color=g.uniform(0, 1, (n, 3)), opacity=g.uniform(0.2, 1, n))
    P = O.Params(mode=O.MODE_ADD2D, cov=O.COV_RS)
    full, _, _, _ = O.render_o1(P, W, H, O.project(P, prims))
    perm = g.permutation(n)
    shuf = {k: v[perm] for k, v in prims.items()}
    img2, _, _, _ = O.render_o1(P, W, H, O.project(P, shuf))
    assert np.max(np.abs(full - img2)) < 1e-12
    a = {k: v[: n // 2] for k, v in prims.items()}
    b = {k: v[n // 2:] for k, v in prims.items()}
    ia, _, _, _ = O.render_o1(P, W, H, O.project(P, a))
    ib, _, _, _ = O.render_o1(P, W, H, O.project(P, b))
    assert np.max(np.abs(full - ia - ib)) < 1e-12


# ----------------------------------------------------------------------------
# Alpha compositing (Eq. 3 with W') closed forms
# ----------------------------------------------------------------------------

def cam_identity(W=33, H=33):
    # principal point on the centre of pixel (16, 16)
    return O.Camera(width=W, height=H, fx=50.0, fy=50.0, cx=16.5, cy=16.5, viewmat=np.eye(4))


def p3(mean, opac, color, scale=None, freq=None, quat=None):
    n = len(mean)
    return dict(mean=np.asarray(mean, float), quat=np.asarray(quat if quat is not None else [[1, 0, 0, 0]] * n, float),
                scale=np.asarray(scale if scale is not None else [[0.05, 0.05, 0.05]] * n, float),
                freq=np.asarray(freq if freq is not None else [[0.0, 0.0, 0.0]] * n, float),
                color=np.asarray(color, float), opacity=np.asarray(opac, float))


def alpha_render(prims, cam, bg=(0.2, 0.3, 0.4), pix=None):
    P = O.Params(mode=O.MODE_ALPHA3D, cov=O.COV_QUAT_SCALE, blur_eps=0.3, bg=bg)
    scr = O.project(P, prims, cam)
    keys = O.depth_keys(prims, cam)
    return O.render_o1(P, cam.width, cam.height, scr, keys, pix=pix)


def test_alpha_single_primitive_centre():
    """At mu' (W' = 1): C = c alpha + (1 - alpha) bg, T = 1 - alpha, alpha = min(o, 0.99)."""
    cam = cam_identity()
    bg = np.array([0.2, 0.3, 0.4])
    for o in (0.37, 0.995):
        c = np.array([0.9, 0.1, 0.5])
        img, T, nc, _ = alpha_render(p3([[0, 0, 2.0]], [o], [c]), cam, pix=[16 * 33 + 16])
        a = min(o, 0.99)
        assert np.allclose(img[0], c * a + (1 - a) * bg, atol=1e-14)
        assert abs(T[0] - (1 - a)) < 1e-14 and nc[0] == 1


def test_alpha_two_primitives_order_and_ties():
    """Two primitives on the same pixel: C = c1 a1 + c2 a2 (1 - a1) + bg (1 - a1)(1 - a2) in depth
    order; swapping depths swaps the terms; equal depths composite in index order."""
    cam = cam_identity()
    bg = np.array([0.2, 0.3, 0.4])
    c1, c2 = np.array([1.0, 0.0, 0.2]), np.array([0.0, 1.0, 0.7])
    o1, o2 = 0.6, 0.45

    def expect(ca, aa, cb, ab):
        return ca * aa + cb * ab * (1 - aa) + bg * (1 - aa) * (1 - ab)

    img, _, _, _ = alpha_render(p3([[0, 0, 2.0], [0, 0, 3.0]], [o1, o2], [c1, c2]), cam, pix=[16 * 33 + 16])
    assert np.allclose(img[0], expect(c1, o1, c2, o2), atol=1e-14)
    img, _, _, _ = alpha_render(p3([[0, 0, 3.0], [0, 0, 2.0]], [o1, o2], [c1, c2]), cam, pix=[16 * 33 + 16])
    assert np.allclose(img[0], expect(c2, o2, c1, o1), atol=1e-14)
    img, _, _, _ = alpha_render(p3([[0, 0, 2.5], [0, 0, 2.5]], [o1, o2], [c1, c2]), cam, pix=[16 * 33 + 16])
    assert np.allclose(img[0], expect(c1, o1, c2, o2), atol=1e-14)


def test_alpha_termination_count():
    """n co-located primitives of constant alpha stop after n* = floor(ln T_min / ln(1 - alpha)) + 1
    (include-then-stop): C = c (1 - (1 - alpha)^n*) + bg (1 - alpha)^n*."""
    cam = cam_identity()
    bg = np.array([0.2, 0.3, 0.4])
    c = np.array([0.3, 0.6, 0.9])
    for alpha in (0.3, 0.55):
        nstar = math.floor(math.log(1e-4) / math.log(1 - alpha)) + 1
        m = nstar + 12
        prims = p3([[0, 0, 2.0 + 0.01 * k] for k in range(m)], [alpha] * m, [c] * m)
        img, T, nc, _ = alpha_render(prims, cam, pix=[16 * 33 + 16])
        rem = (1 - alpha) ** nstar
        assert nc[0] == nstar
        assert abs(T[0] - rem) < 1e-14
        assert np.allclose(img[0], c * (1 - rem) + bg * rem, atol=1e-13)


def test_alpha_skip_below_alpha_min():
    """A pair with o W' < alpha_min is skipped entirely (T unchanged)."""
    cam = cam_identity()
    prims = p3([[0, 0, 2.0]], [0.5], [[1.0, 1.0, 1.0]], scale=[[0.01, 0.01, 0.01]])
    # 6 px from the centre the wavelet is tiny
    img, T, nc, _ = alpha_render(prims, cam, pix=[16 * 33 + 22])
    assert nc[0] == 0 and T[0] == 1.0
    assert np.allclose(img[0], [0.2, 0.3, 0.4], atol=0)


# ----------------------------------------------------------------------------
# Projection (Eq. 2, Eq. 7 and the frequency transform)
# ----------------------------------------------------------------------------

def test_projection_on_axis_closed_form():
    """Camera at the origin looking down +z, primitive on the axis: mu' = (cx, cy),
    Sigma' = diag(fx^2 sx^2, fy^2 sy^2) / z^2 + eps I, f' = (fx nu_x, fy nu_y) / z (vector
    transform), f' = (z nu_x / fx, z nu_y / fy) (covector transform)."""
    cam = O.Camera(width=640, height=480, fx=500.0, fy=420.0, cx=320.0, cy=240.0, viewmat=np.eye(4))
    z, s, nu = 3.0, [0.02, 0.05, 0.03], np.array([1.5, -2.0, 0.7])
    prims = p3([[0, 0, z]], [0.8], [[1, 1, 1]], scale=[s], freq=[nu])
    for eps in (0.0, 0.3):
        P = O.Params(mode=O.MODE_ALPHA3D, cov=O.COV_QUAT_SCALE, blur_eps=eps)
        scr = O.project(P, prims, cam)[0]
        assert np.allclose(scr[[0, 1]], [320.0, 240.0], atol=1e-12)
        Sp = np.linalg.inv([[scr[2], scr[3]], [scr[3], scr[4]]])
        assert np.allclose(Sp, np.diag([(500 * s[0] / z) ** 2 + eps, (420 * s[1] / z) ** 2 + eps]), rtol=1e-12)
        assert np.allclose(scr[[5, 6]], [500 * nu[0] / z, 420 * nu[1] / z], rtol=1e-12)
        assert abs(scr[11] - z) < 1e-15
    P = O.Params(mode=O.MODE_ALPHA3D, cov=O.COV_QUAT_SCALE, freq_xform=O.FREQ_COVECTOR)
    scr = O.project(P, prims, cam)[0]
    assert np.allclose(scr[[5, 6]], [z * nu[0] / 500, z * nu[1] / 420], rtol=1e-12)


def _pinhole(t, cam):
    return np.array([cam.fx * t[0] / t[2] + cam.cx, cam.fy * t[1] / t[2] + cam.cy])


def test_projection_off_axis_matches_linearised_pinhole():
    """mu' is the pinhole image of the camera-space mean; Sigma' = M Sigma M^T + eps I and
    f' = M f where M is the numerical Jacobian of the pinhole map composed with the camera
    rotation, and Sigma = R(q) diag(s^2) R(q)^T with R from scipy (scalar-last there).
    Catches: a transposed rotation, the wrong J column, quaternion component order."""
    g = np.random.default_rng(11)
    ang = g.normal(0, 0.3, 3)
    Rw = Rotation.from_rotvec(ang).as_matrix()
    V = np.eye(4); V[:3, :3] = Rw; V[:3, 3] = [0.1, -0.2, 2.5]
    cam = O.Camera(width=800, height=600, fx=700.0, fy=650.0, cx=400.0, cy=300.0, viewmat=V)
    n = 8
    mean = g.uniform(-0.4, 0.4, (n, 3))
    quat = g.normal(0, 1, (n, 4))
    scale = g.uniform(0.01, 0.08, (n, 3))
    freq = g.normal(0, 3, (n, 3))
    prims = p3(mean, [0.9] * n, [[1, 1, 1]] * n, scale=scale, freq=freq, quat=quat)
    P = O.Params(mode=O.MODE_ALPHA3D, cov=O.COV_QUAT_SCALE, blur_eps=0.3)
    scr = O.project(P, prims, cam)
    for i in range(n):
        t = Rw @ mean[i] + V[:3, 3]
        assert np.allclose(scr[i, [0, 1]], _pinhole(t, cam), rtol=1e-13)
        Jn = np.zeros((2, 3))
        for k in range(3):
            h = 1e-6
            e = np.zeros(3); e[k] = h
            Jn[:, k] = (_pinhole(t + e, cam) - _pinhole(t - e, cam)) / (2 * h)
        M = Jn @ Rw
        q = quat[i] / np.linalg.norm(quat[i])
        Rq = Rotation.from_quat([q[1], q[2], q[3], q[0]]).as_matrix()
        S3 = Rq @ np.diag(scale[i] ** 2) @ Rq.T
        Sp = M @ S3 @ M.T + 0.3 * np.eye(2)
        Sp_or = np.linalg.inv([[scr[i, 2], scr[i, 3]], [scr[i, 3], scr[i, 4]]])
        assert np.allclose(Sp_or, Sp, rtol=1e-7)
        assert np.allclose(scr[i, [5, 6]], M @ freq[i], rtol=1e-7, atol=1e-9)
        assert abs(scr[i, 11] - t[2]) < 1e-13


def test_covector_transform_preserves_phase():
    """The covector variant keeps f'.(M d) = f.d for displacements d on which the third
    row of the ray-space Jacobian vanishes (to first order)."""
    g = np.random.default_rng(5)
    Rw = Rotation.from_rotvec(g.normal(0, 0.3, 3)).as_matrix()
    V = np.eye(4); V[:3, :3] = Rw; V[:3, 3] = [0.0, 0.0, 3.0]
    cam = O.Camera(width=800, height=600, fx=700.0, fy=650.0, cx=400.0, cy=300.0, viewmat=V)
    mean = np.array([[0.2, -0.1, 0.3]])
    f = np.array([[2.0, -1.0, 0.5]])
    prims = p3(mean, [0.9], [[1, 1, 1]], freq=f)
    P = O.Params(mode=O.MODE_ALPHA3D, cov=O.COV_QUAT_SCALE, freq_xform=O.FREQ_COVECTOR)
    scr = O.project(P, prims, cam)[0]
    t = Rw @ mean[0] + V[:3, 3]
    # displacement orthogonal to the viewing ray, expressed in world space
    ray = t / np.linalg.norm(t)
    dcam = np.cross(ray, [0.3, 0.8, 0.1]); dcam *= 1e-6 / np.linalg.norm(dcam)
    dworld = Rw.T @ dcam
    dscreen = _pinhole(t + dcam, cam) - _pinhole(t, cam)
    assert abs(scr[5] * dscreen[0] + scr[6] * dscreen[1] - f[0] @ dworld) < 1e-6 * abs(f[0] @ dworld) + 1e-14


# ----------------------------------------------------------------------------
# O1 == O2 (two organisations of one definition)
# ----------------------------------------------------------------------------

def scene2d(n, W, H, seed, cov):
    g = np.random.default_rng(seed)
    if cov == O.COV_RS:
        covp = np.stack([g.uniform(1, 7, n), g.uniform(1, 7, n), g.uniform(0, math.pi, n)], 1)
    else:
        covp = np.stack([g.uniform(1, 6, n), g.normal(0, 2, n), g.uniform(1, 6, n)], 1)
    return dict(mean=np.stack([g.uniform(-5, W + 5, n), g.uniform(-5, H + 5, n)], 1), cov=covp,
                freq=g.normal(0, 1.2, (n, 2)), color=g.uniform(0, 1, (n, 3)), opacity=g.uniform(0.3, 1, n))


def scene3d(n, seed):
    g = np.random.default_rng(seed)
    V = np.eye(4); V[:3, 3] = [-0.5, -0.5, 2.0]
    cam = O.Camera(width=64, height=48, fx=60.0, fy=60.0, cx=32.0, cy=24.0, viewmat=V)
    prims = p3(g.uniform(0.1, 0.9, (n, 3)), g.uniform(0.05, 0.99, n), g.uniform(0.05, 0.99, (n, 3)),
               scale=np.exp(g.uniform(np.log(0.01), np.log(0.08), (n, 3))), freq=g.normal(0, 20, (n, 3)),
               quat=g.normal(0, 1, (n, 4)))
    return prims, cam


@pytest.mark.parametrize("cov", [O.COV_RS, O.COV_CHOLESKY])
def test_o1_equals_o2_additive(cov):
    prims = scene2d(60, 70, 50, 21, cov)
    P = O.Params(mode=O.MODE_ADD2D, cov=cov)
    scr = O.project(P, prims)
    i1, _, _, t1 = O.render_o1(P, 70, 50, scr)
    i2, _, _, t2 = O.render_o2(P, 70, 50, scr)
    assert np.max(np.abs(i1 - i2.reshape(-1, 3))) < 1e-12
    g = np.random.default_rng(1).normal(0, 1, (50 * 70, 3))
    d1 = O.render_bwd_o1(P, 70, 50, scr, g)
    d2 = O.render_bwd_o2(P, 70, 50, scr, np.ones((50, 70)), np.zeros((50, 70), np.int32), g.reshape(50, 70, 3))
    assert np.max(np.abs(d1 - d2)) < 1e-9 * max(1.0, np.max(np.abs(d1)))


def test_o1_equals_o2_alpha():
    prims, cam = scene3d(2500, 4)
    P = O.Params(mode=O.MODE_ALPHA3D, cov=O.COV_QUAT_SCALE, blur_eps=0.3, bg=(0.1, 0.2, 0.3))
    scr = O.project(P, prims, cam)
    keys = O.depth_keys(prims, cam)
    W, H = cam.width, cam.height
    i1, T1, n1, _ = O.render_o1(P, W, H, scr, keys)
    i2, T2, last, _ = O.render_o2(P, W, H, scr, keys)
    assert np.max(np.abs(i1 - i2.reshape(-1, 3))) < 1e-12
    assert np.max(np.abs(T1 - T2.reshape(-1))) < 1e-12
    assert n1.max() > 5 and (T1 < 1e-4).any()          # some pixels terminate
    g = np.random.default_rng(2).normal(0, 1, (W * H, 3))
    d1 = O.render_bwd_o1(P, W, H, scr, g, keys)
    d2 = O.render_bwd_o2(P, W, H, scr, T2, last, g.reshape(H, W, 3), keys)
    assert np.max(np.abs(d1 - d2)) < 1e-8 * max(1.0, np.max(np.abs(d1)))


# ----------------------------------------------------------------------------
# Gradients by central finite differences of the FP64 forward
# ----------------------------------------------------------------------------

def _loss(P, prims, W, H, g, cam=None):
    scr = O.project(P, prims, cam)
    keys = O.depth_keys(prims, cam) if cam is not None else None
    img, _, _, tie = O.render_o1(P, W, H, scr, keys)
    return float(np.sum(img * g)), tie


def _check_fd(P, prims, W, H, cam, names, rel=1e-6, seed=0):
    g = np.random.default_rng(seed).normal(0, 1, (W * H, 3))
    scr = O.project(P, prims, cam)
    keys = O.depth_keys(prims, cam) if cam is not None else None
    _, _, _, tie = O.render_o1(P, W, H, scr, keys)
    assert not tie.any(), "test scene must sit away from every decision threshold"
    ds = O.render_bwd_o1(P, W, H, scr, g, keys)
    grads = O.project_bwd(P, prims, scr, ds, cam)
    for name in names:
        arr = prims[name]
        fd = np.zeros_like(arr, dtype=float)
        flat = arr.reshape(-1)
        for k in range(flat.size):
            # central differences at two steps; where they disagree a decision threshold lies
            # within the larger step, so the smaller one is used
            vals = []
            for h in (1e-6 * max(abs(flat[k]), 1e-2), 1e-7 * max(abs(flat[k]), 1e-2)):
                old = flat[k]
                flat[k] = old + h
                lp, _ = _loss(P, prims, W, H, g, cam)
                flat[k] = old - h
                lm, _ = _loss(P, prims, W, H, g, cam)
                flat[k] = old
                vals.append((lp - lm) / (2 * h))
            smooth = abs(vals[0] - vals[1]) <= 1e-4 * max(abs(vals[0]), abs(vals[1]), 1e-8)
            fd.reshape(-1)[k] = vals[0] if smooth else vals[1]
        an = grads[name].reshape(fd.shape)
        err = np.max(np.abs(an - fd)) / max(np.max(np.abs(fd)), 1e-12)
        assert err < rel, (name, err)


@pytest.mark.parametrize("cov", [O.COV_RS, O.COV_CHOLESKY])
def test_fd_gradients_additive(cov):
    prims = scene2d(5, 30, 26, 31 + cov, cov)
    P = O.Params(mode=O.MODE_ADD2D, cov=cov)
    _check_fd(P, prims, 30, 26, None, ["mean", "cov", "freq", "color", "opacity"], rel=1e-6)


def test_fd_gradients_alpha():
    # seed chosen so that no FD step crosses the alpha_min skip threshold
    g = np.random.default_rng(42)
    n = 6
    V = np.eye(4); V[:3, :3] = Rotation.from_rotvec([0.1, -0.2, 0.05]).as_matrix(); V[:3, 3] = [-0.5, -0.5, 2.0]
    cam = O.Camera(width=28, height=24, fx=30.0, fy=32.0, cx=14.0, cy=12.0, viewmat=V, time=0.4)
    prims = p3(g.uniform(0.3, 0.7, (n, 3)), g.uniform(0.3, 0.95, n), g.uniform(0.05, 0.99, (n, 3)),
               scale=g.uniform(0.03, 0.12, (n, 3)), freq=g.normal(0, 8, (n, 3)), quat=g.normal(0, 1, (n, 4)))
    prims["velocity"] = g.normal(0, 0.05, (n, 3))
    P = O.Params(mode=O.MODE_ALPHA3D, cov=O.COV_QUAT_SCALE, blur_eps=0.3, bg=(0.2, 0.1, 0.4))
    _check_fd(P, prims, cam.width, cam.height, cam,
              ["mean", "quat", "scale", "freq", "color", "opacity", "velocity"], rel=2e-6)


def test_fd_gradients_alpha_guard_band():
    """A primitive outside the guard band: the clamped x/z has zero derivative."""
    V = np.eye(4)
    cam = O.Camera(width=32, height=32, fx=20.0, fy=20.0, cx=16.0, cy=16.0, viewmat=V)
    # x/z = 1.9 > 1.3 * 16/20 = 1.04: clamped, yet its wide footprint reaches the image
    prims = p3([[1.9, 0.1, 1.0], [0.05, -0.05, 1.5]], [0.8, 0.7], [[0.9, 0.2, 0.1], [0.1, 0.5, 0.9]],
               scale=[[0.6, 0.2, 0.3], [0.05, 0.04, 0.06]], freq=[[1.0, -0.5, 0.3], [2.0, 1.0, -1.0]],
               quat=[[0.9, 0.1, 0.2, -0.1], [0.7, -0.3, 0.1, 0.2]])
    P = O.Params(mode=O.MODE_ALPHA3D, cov=O.COV_QUAT_SCALE, blur_eps=0.3)
    scr = O.project(P, prims, cam)
    assert scr[0, 15] == 1.0
    _check_fd(P, prims, 32, 32, cam, ["mean", "quat", "scale", "freq", "opacity"], rel=2e-6, seed=3)


# ----------------------------------------------------------------------------
# O-bin against brute-force enumeration and numpy's stable sort
# ----------------------------------------------------------------------------

@pytest.mark.parametrize("mode,tw,th", [(O.MODE_ALPHA3D, 16, 16), (O.MODE_ADD2D, 8, 8), (O.MODE_ALPHA3D, 32, 16)])
def test_binning_brute_force(mode, tw, th):
    """O-bin against brute force.  The pixel box: pixels whose centre lies within the FP32 half-extents
    (enumerated).  The tiles kept: a tile of a rectangle of at most 64 tiles is kept iff the support
    ellipse q <= Qs reaches its pixel-centre rectangle -- checked against the rectangle minimum of q
    found by scipy's bounded L-BFGS-B in FP64 (decisions within 1e-3 of Qs are ties and accept either
    outcome), and against pixel-centre enumeration (no tile holding a centre with q <= Qs is dropped).
    Keys, values and ranges: numpy's stable argsort of the kept instances."""
    from scipy.optimize import minimize
    from paper_2508_12615_amd import synth
    W, H = 150, 93
    n = 250
    r = synth.screen_records(n, W, H, seed=77)
    out = O.bin_tiles(W, H, tw, th, mode, r["mx"], r["my"], r["rx"], r["ry"], r["depth"], r["ca"], r["cb"], r["cc"],
                      r["Qs"])
    tiles_x = -(-W // tw)
    keys, vals, decided, dropped = [], [], 0, 0
    kept_ref = {}
    for i in range(n):
        mx, my, rx, ry = (np.float32(r[k][i]) for k in ("mx", "my", "rx", "ry"))
        ca, cb, cc, Qs = (float(r[k][i]) for k in ("ca", "cb", "cc", "Qs"))
        rect = set()
        if rx >= 0 and ry >= 0:
            lox, hix = (mx - rx) - np.float32(0.5), (mx + rx) - np.float32(0.5)
            loy, hiy = (my - ry) - np.float32(0.5), (my + ry) - np.float32(0.5)
            xs = [x for x in range(W) if lox <= x <= hix]
            ys = [y for y in range(H) if loy <= y <= hiy]
            for y in ys:
                for x in xs:
                    rect.add((y // th, x // tw))
            if xs and ys:
                assert tuple(out["box"][i]) == (xs[0], ys[0], xs[-1], ys[-1])
        q = lambda p: ca * (p[0] - float(mx)) ** 2 + 2 * cb * (p[0] - float(mx)) * (p[1] - float(my)) + \
            cc * (p[1] - float(my)) ** 2  # noqa: E731
        mine = set()
        for (ty, tx) in sorted(rect):
            b = out["box"][i]
            x0, x1 = max(tx * tw, b[0]) + 0.5, min(tx * tw + tw - 1, b[2]) + 0.5
            y0, y1 = max(ty * th, b[1]) + 0.5, min(ty * th + th - 1, b[3]) + 0.5
            if len(rect) > 64:
                mine.add((ty, tx))
                continue
            res = minimize(q, [(x0 + x1) / 2, (y0 + y1) / 2], method="L-BFGS-B", bounds=[(x0, x1), (y0, y1)],
                           options=dict(ftol=1e-15, gtol=1e-12))
            centres = [q((x + 0.5, y + 0.5)) for x in range(int(x0), int(x1) + 1) for y in range(int(y0), int(y1) + 1)]
            if min(centres) <= Qs * (1 - 1e-6):
                mine.add((ty, tx))                 # holds a supported pixel centre: must be kept
            elif res.fun > Qs * (1 + 1e-3):
                dropped += 1                       # ellipse misses the rectangle: must be dropped
            elif res.fun < Qs * (1 - 1e-3):
                mine.add((ty, tx))                 # ellipse reaches the rectangle: kept
            else:
                mine.add(None)                     # tie: either outcome
                continue
            decided += 1
        kept_ref[i] = mine
    # the oracle's instances per primitive, from its sorted output
    got = {}
    tile_of = out["keys"] >> np.uint64(32) if mode == O.MODE_ALPHA3D else out["keys"]
    for t, v in zip(tile_of.astype(np.int64), out["vals"]):
        got.setdefault(int(v), set()).add((int(t) // tiles_x, int(t) % tiles_x))
    for i in range(n):
        ref = kept_ref[i]
        have = got.get(i, set())
        assert out["count"][i] == len(have)
        assert {x for x in ref if x is not None} <= have, i
        if None not in ref:
            assert have == ref, i
    assert decided > 200 and dropped > 20, (decided, dropped)
    for i in sorted(got):
        for (ty, tx) in sorted(got[i]):
            t = ty * tiles_x + tx
            d = int(np.float32(r["depth"][i]).view(np.uint32))
            keys.append((t << 32) | d if mode == O.MODE_ALPHA3D else t)
            vals.append(i)
    keys = np.array(keys, np.uint64); vals = np.array(vals, np.uint32)
    order = np.argsort(keys, kind="stable")
    assert out["K"] == len(keys)
    assert np.array_equal(out["keys"], keys[order]) and np.array_equal(out["vals"], vals[order])
    for t in range(out["ranges"].shape[0]):
        lo = np.searchsorted(tile_of, t, "left"); hi = np.searchsorted(tile_of, t, "right")
        exp = (lo, hi) if hi > lo else (0, 0)
        assert tuple(out["ranges"][t]) == exp


# ----------------------------------------------------------------------------
# Work counts against a numpy brute force
# ----------------------------------------------------------------------------

def _support_counts_numpy(P, W, H, scr, keys):
    """Support pairs per pixel, written out from the definitions: a pair is in the support when
    q <= Q (Q = q_add, or 2 ln(o / alpha_min) in alpha mode); pairs are visited in compositing order
    ((depth key, index) in alpha mode, index order in additive mode); the forward count runs up to and
    including the stopping pair (the pair after which T < T_min), the backward count up to and
    including the last pair with o W' >= alpha_min before that stop."""
    valid = np.flatnonzero(scr[:, 15] != 0)
    if P.mode == O.MODE_ALPHA3D:
        valid = valid[np.lexsort((valid, np.asarray(keys)[valid]))]
    fwd = np.zeros(W * H, np.int64)
    bwd = np.zeros(W * H, np.int64)
    ys, xs = np.divmod(np.arange(W * H), W)
    px, py = xs + 0.5, ys + 0.5
    q = np.zeros((valid.size, W * H))
    a = np.zeros_like(q)
    for j, i in enumerate(valid):
        s = scr[i]
        dx, dy = px - s[0], py - s[1]
        q[j] = s[2] * dx * dx + 2 * s[3] * dx * dy + s[4] * dy * dy
        a[j] = s[7] * 0.5 * (1 + np.cos(s[5] * dx + s[6] * dy + s[16])) * np.exp(-0.5 * q[j])
    insup = q <= scr[valid, 14][:, None]
    for p in range(W * H):
        if P.mode == O.MODE_ADD2D:
            fwd[p] = bwd[p] = insup[:, p].sum()
            continue
        T, stop, last = 1.0, valid.size - 1, -1
        for j in range(valid.size):
            if a[j, p] < P.alpha_min:
                continue
            last = j
            T *= 1.0 - min(a[j, p], P.alpha_max)
            if T < P.T_min:
                stop = j
                break
        fwd[p] = insup[: stop + 1, p].sum()
        bwd[p] = insup[: last + 1, p].sum()
    return fwd, bwd


@pytest.mark.parametrize("mode", [O.MODE_ADD2D, O.MODE_ALPHA3D])
def test_support_counts_brute_force(mode):
    """The oracle's support-pair counts (the roofline numerator) against the numpy brute force above,
    on scenes where pixels stop, pairs are skipped, and supports overlap; catches an off-by-one in
    the stop or last rule."""
    if mode == O.MODE_ADD2D:
        prims = scene2d(40, 36, 30, 5, O.COV_RS)
        P = O.Params(mode=O.MODE_ADD2D, cov=O.COV_RS)
        W, H, cam, keys = 36, 30, None, None
    else:
        prims, cam = scene3d(900, 6)
        cam = O.Camera(width=40, height=30, fx=40.0, fy=40.0, cx=20.0, cy=15.0, viewmat=cam.viewmat)
        prims["opacity"] = np.clip(prims["opacity"] * 1.2, 0, 0.995)
        P = O.Params(mode=O.MODE_ALPHA3D, cov=O.COV_QUAT_SCALE, blur_eps=0.3)
        W, H = cam.width, cam.height
        keys = O.depth_keys(prims, cam)
    scr = O.project(P, prims, cam)
    cf, cb = O.support_counts(P, W, H, scr, keys)
    nf, nb = _support_counts_numpy(P, W, H, scr, keys)
    assert np.array_equal(cf, nf) and np.array_equal(cb, nb)
    if mode == O.MODE_ALPHA3D:
        _, T, _, _ = O.render_o1(P, W, H, scr, keys)
        assert (T < P.T_min).sum() > 20 and (cb < cf).sum() > 20      # stops and skipped tails occur


# ----------------------------------------------------------------------------
# O-bin kept tiles against pixel-centre enumeration (no tile-count rule)
# ----------------------------------------------------------------------------

@pytest.mark.parametrize("tw,th", [(8, 8), (16, 16)])
def test_binning_keeps_every_supported_tile(tw, th):
    """Large, anisotropic supports (tile rectangles of up to several hundred tiles, so both sides of
    the binning's 64-tile rule occur): every tile holding a pixel centre with q <= Qs is kept, no kept
    tile lies outside the tile rectangle of the enumerated pixel box, and count is the number kept.
    Checked by enumerating every pixel centre of the image; nothing here depends on the tile-count
    rule, so it pins the rule's large-rectangle branch as well as the culled one."""
    g = np.random.default_rng(123)
    W, H, n = 240, 200, 60
    sig = np.exp(g.uniform(np.log(2.0), np.log(70.0), (n, 2)))
    th_ = g.uniform(0, math.pi, n)
    c, s_ = np.cos(th_), np.sin(th_)
    Sxx = c * c * sig[:, 0] ** 2 + s_ * s_ * sig[:, 1] ** 2
    Syy = s_ * s_ * sig[:, 0] ** 2 + c * c * sig[:, 1] ** 2
    Sxy = c * s_ * (sig[:, 0] ** 2 - sig[:, 1] ** 2)
    det = Sxx * Syy - Sxy ** 2
    Qs = np.full(n, 9.0 * 1.001 + 1e-3)
    r = dict(mx=g.uniform(-20, W + 20, n), my=g.uniform(-20, H + 20, n), ca=Syy / det, cb=-Sxy / det, cc=Sxx / det,
             rx=np.sqrt(Qs * Sxx) * 1.0002, ry=np.sqrt(Qs * Syy) * 1.0002, depth=g.uniform(1, 2, n), Qs=Qs)
    r = {k: np.asarray(v, np.float32) for k, v in r.items()}
    out = O.bin_tiles(W, H, tw, th, O.MODE_ALPHA3D, r["mx"], r["my"], r["rx"], r["ry"], r["depth"], r["ca"], r["cb"],
                      r["cc"], r["Qs"])
    tiles_x = -(-W // tw)
    got = {}
    for t, v in zip((out["keys"] >> np.uint64(32)).astype(np.int64), out["vals"]):
        got.setdefault(int(v), set()).add((int(t) // tiles_x, int(t) % tiles_x))
    ys, xs = np.mgrid[0:H, 0:W]
    big = 0
    for i in range(n):
        mx, my, rx, ry = (np.float32(r[k][i]) for k in ("mx", "my", "rx", "ry"))
        dx, dy = xs + 0.5 - float(mx), ys + 0.5 - float(my)
        q = float(r["ca"][i]) * dx * dx + 2 * float(r["cb"][i]) * dx * dy + float(r["cc"][i]) * dy * dy
        inbox = ((mx - rx) - np.float32(0.5) <= xs) & (xs <= (mx + rx) - np.float32(0.5)) & \
                ((my - ry) - np.float32(0.5) <= ys) & (ys <= (my + ry) - np.float32(0.5))
        need = {(int(y) // th, int(x) // tw) for y, x in zip(*np.nonzero(inbox & (q <= float(r["Qs"][i]) * (1 - 1e-6))))}
        rect = {(int(y) // th, int(x) // tw) for y, x in zip(*np.nonzero(inbox))}
        have = got.get(i, set())
        assert need <= have, i
        assert have <= rect, i
        assert out["count"][i] == len(have)
        big += len(rect) > 64
    assert big >= 5


# ----------------------------------------------------------------------------
# The tie protocol itself (tests/helpers.compare_image)
# ----------------------------------------------------------------------------

def test_tie_protocol_accepts_flipped_ties_and_catches_wrong_decisions():
    """Renders whose support threshold moves by 3e-6 relative flip only decisions the oracle flags as
    ties: compare_image accepts them (each flip stays within its jump bound).  A threshold moved by
    1e-3 flips decisions that are not ties: compare_image rejects it.  A tie pixel moved beyond its
    jump bound is rejected too."""
    from helpers import compare_image
    W, H = 150, 118
    prims = scene2d(900, W, H, 8, O.COV_RS)
    P = O.Params(mode=O.MODE_ADD2D, cov=O.COV_RS)
    scr = O.project(P, prims)
    ref, _, _, tie, jb = O.render_o1(P, W, H, scr, jump=True)
    assert tie.sum() > 0
    flipped = scr.copy(); flipped[:, 14] *= 1 + 3e-6
    img2, _, _, _ = O.render_o1(P, W, H, flipped)
    assert np.abs(img2 - ref).max() > 1e-4            # some tie pixel really moved
    compare_image(img2, ref, tie, jb, max_tie_frac=1e-2)
    wrong = scr.copy(); wrong[:, 14] *= 1 + 1e-3
    img3, _, _, _ = O.render_o1(P, W, H, wrong)
    with pytest.raises(AssertionError):
        compare_image(img3, ref, tie, jb, max_tie_frac=1e-2)
    k = int(np.flatnonzero(tie)[0])
    bad = ref.copy(); bad[k, 0] += jb[k, 0] + 3e-4
    with pytest.raises(AssertionError):
        compare_image(bad, ref, tie, jb, max_tie_frac=1e-2)
