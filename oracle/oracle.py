"""FP64 reference oracle for the WIPES wavelet rasterizer -- TEST INFRASTRUCTURE ONLY.

Thin ctypes harness around ``wipes_oracle.c`` (plain C, FP64).  Only the test
suite, the smoke check and the CPU-baseline leg of the benchmark may import
this module; the rasterizer library never does.  It shares no code with the
HIP library: inputs are plain numpy arrays produced by the seeded generators.

Paper: arXiv 2508.12615, "WIPES: Wavelet-based Visual Primitives".
  * Eq. 6  wavelet W = 1/2 [cos(f.(x - mu)) + 1] G(x; mu, Sigma)
  * Eq. 7  screen-space wavelet W'(x'; mu', f', Sigma')
  * Eq. 2  EWA projection Sigma' = 2x2 block of J W Sigma W^T J^T
  * Eq. 3  front-to-back alpha blending, Eq. 4 additive blending
The readings the paper leaves open (support, clamp, termination, pixel
centres, key layout) are documented in wipes_oracle.c where they are used.

Functions: project, depth_keys, render_o1, render_bwd_o1, render_o2,
render_bwd_o2, project_bwd, bin_tiles, support_counts, sh_basis.  All are
pinned by tests/test_oracle_*.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from dataclasses import dataclass, field

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "wipes_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

MODE_ADD2D, MODE_ALPHA3D = 0, 1
COV_CHOLESKY, COV_RS, COV_QUAT_SCALE = 0, 1, 2
FREQ_VECTOR, FREQ_COVECTOR = 0, 1

# screen record columns (FP64)
SR = dict(mx=0, my=1, ca=2, cb=3, cc=4, fx=5, fy=6, op=7, r=8, g=9, b=10, depth=11, rx=12, ry=13, Q=14, valid=15,
          phase=16)
SR_N = 17
# screen-space gradient columns
SG = dict(mx=0, my=1, ca=2, cb=3, cc=4, fx=5, fy=6, op=7, r=8, g=9, b=10, phase=11)
SG_N = 12

TIE_SUPPORT, TIE_SKIP, TIE_STOP, TIE_CLAMP, TIE_CULL = 1, 2, 4, 8, 16


def build(force: bool = False) -> str:
    """Compile the oracle with gcc (FP64 C, no FMA contraction)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(
            ["gcc", "-O2", "-fopenmp", "-ffp-contract=off", "-fno-fast-math", "-fPIC", "-shared",
             "-std=c99", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


class _Params(C.Structure):
    _fields_ = [("mode", C.c_int32), ("cov", C.c_int32), ("freq_xform", C.c_int32), ("sh_degree", C.c_int32),
                ("alpha_min", C.c_double), ("alpha_max", C.c_double), ("T_min", C.c_double),
                ("q_add", C.c_double), ("blur_eps", C.c_double), ("near_plane", C.c_double),
                ("fov_guard", C.c_double), ("bg", C.c_double * 3)]


class _Camera(C.Structure):
    _fields_ = [("width", C.c_int32), ("height", C.c_int32), ("fx", C.c_double), ("fy", C.c_double),
                ("cx", C.c_double), ("cy", C.c_double), ("viewmat", C.c_double * 16), ("time", C.c_double)]


@dataclass
class Params:
    """Rasterizer constants.  Defaults are the readings the oracle documents."""
    mode: int = MODE_ADD2D
    cov: int = COV_RS
    freq_xform: int = FREQ_VECTOR
    sh_degree: int = -1          # < 0: direct RGB colour; 0..3: spherical-harmonic colour
    alpha_min: float = 1.0 / 255.0
    alpha_max: float = 0.99
    T_min: float = 1e-4
    q_add: float = 9.0
    blur_eps: float = 0.0
    near_plane: float = 0.01
    fov_guard: float = 1.3
    bg: tuple = (0.0, 0.0, 0.0)

    def c(self) -> _Params:
        p = _Params()
        p.mode, p.cov, p.freq_xform, p.sh_degree = self.mode, self.cov, self.freq_xform, self.sh_degree
        p.alpha_min, p.alpha_max, p.T_min = self.alpha_min, self.alpha_max, self.T_min
        p.q_add, p.blur_eps, p.near_plane, p.fov_guard = self.q_add, self.blur_eps, self.near_plane, self.fov_guard
        for k in range(3):
            p.bg[k] = float(self.bg[k])
        return p


@dataclass
class Camera:
    width: int
    height: int
    fx: float
    fy: float
    cx: float
    cy: float
    viewmat: np.ndarray = field(default_factory=lambda: np.eye(4))
    time: float = 0.0

    def c(self) -> _Camera:
        cam = _Camera()
        cam.width, cam.height = int(self.width), int(self.height)
        cam.fx, cam.fy, cam.cx, cam.cy = float(self.fx), float(self.fy), float(self.cx), float(self.cy)
        vm = np.asarray(self.viewmat, dtype=np.float64).reshape(16)
        for k in range(16):
            cam.viewmat[k] = float(vm[k])
        cam.time = float(self.time)
        return cam


_lib = None


def lib():
    global _lib
    if _lib is None:
        # WIPES_ORACLE_LIB points the harness at another build of the same source
        # (used by the mutation tests, which plant mistakes in a temporary copy)
        alt = os.environ.get("WIPES_ORACLE_LIB")
        _lib = C.CDLL(alt if alt else build())
        P = C.c_void_p
        _lib.or_project.argtypes = [C.POINTER(_Params), C.POINTER(_Camera), C.c_int64] + [P] * 10 + [P]
        _lib.or_depth_keys.argtypes = [C.c_int64, P, P, C.c_float, P, P]
        _lib.or_render_o1.argtypes = [C.POINTER(_Params), C.c_int32, C.c_int32, C.c_int64, P, P, C.c_int64,
                                      P, P, P, P, P, P]
        _lib.or_render_bwd_o1.argtypes = [C.POINTER(_Params), C.c_int32, C.c_int32, C.c_int64, P, P, C.c_int64,
                                          P, P, P, C.c_int32]
        _lib.or_render_o2.argtypes = [C.POINTER(_Params), C.c_int32, C.c_int32, C.c_int64, P, P, P, P, P, P, P]
        _lib.or_render_bwd_o2.argtypes = [C.POINTER(_Params), C.c_int32, C.c_int32, C.c_int64, P, P, P, P, P, P,
                                          C.c_int32]
        _lib.or_project_bwd.argtypes = [C.POINTER(_Params), C.POINTER(_Camera), C.c_int64] + [P] * 8 + [P] * 12
        _lib.or_sh_basis.argtypes = [C.c_int32, C.c_int64, P, P, P]
        _lib.or_support_counts.argtypes = [C.POINTER(_Params), C.c_int32, C.c_int32, C.c_int64, P, P, C.c_int64,
                                           P, P, P]
        _lib.or_bin.argtypes = [C.c_int32] * 5 + [C.c_int64] + [P] * 9 + [P, P, P, P, P, P]
    return _lib


def _p(a):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


def _f32(a, shape=None):
    if a is None:
        return None
    a = np.ascontiguousarray(np.asarray(a, dtype=np.float32))
    if shape is not None:
        a = a.reshape(shape)
    return a


def _f64(a, shape=None):
    if a is None:
        return None
    a = np.ascontiguousarray(np.asarray(a, dtype=np.float64))
    if shape is not None:
        a = a.reshape(shape)
    return a


def _prims(prims: dict, n: int, three_d: bool):
    """Parameters as FP64 arrays (exact widening of the FP32 inputs)."""
    d = 3 if three_d else 2
    sh = prims.get("sh")
    return dict(
        phase=_f64(prims.get("phase"), (n,)) if prims.get("phase") is not None else None,
        sh=_f64(sh) if sh is not None and three_d else None,
        mean=_f64(prims["mean"], (n, d)),
        cov=_f64(prims.get("cov"), (n, 3)) if not three_d else None,
        quat=_f64(prims.get("quat"), (n, 4)) if three_d else None,
        scale=_f64(prims.get("scale"), (n, 3)) if three_d else None,
        freq=_f64(prims["freq"], (n, d)),
        color=_f64(prims["color"], (n, 3)),
        opacity=_f64(prims["opacity"], (n,)),
        velocity=_f64(prims.get("velocity"), (n, 3)) if three_d and prims.get("velocity") is not None else None,
    )


def project(params: Params, prims: dict, cam: Camera | None = None) -> np.ndarray:
    """FP64 screen records [n, SR_N] (columns in SR)."""
    n = int(np.asarray(prims["opacity"]).shape[0])
    three_d = params.mode == MODE_ALPHA3D
    q = _prims(prims, n, three_d)
    _check_sh(params, q, n)
    out = np.zeros((n, SR_N), dtype=np.float64)
    cp = params.c()
    cc = cam.c() if cam is not None else None
    lib().or_project(C.byref(cp), C.byref(cc) if cc is not None else None, n, _p(q["mean"]), _p(q["cov"]),
                     _p(q["quat"]), _p(q["scale"]), _p(q["freq"]), _p(q["color"]), _p(q["opacity"]),
                     _p(q["velocity"]), _p(q["phase"]), _p(q["sh"]), _p(out))
    return out


def _check_sh(params: Params, q: dict, n: int):
    if params.sh_degree >= 0:
        if params.mode != MODE_ALPHA3D:
            raise ValueError("spherical-harmonic colour is defined for 3D primitives")
        K = (params.sh_degree + 1) ** 2
        if q["sh"] is None or q["sh"].shape != (n, K, 3):
            raise ValueError("sh must be [n, %d, 3] for degree %d" % (K, params.sh_degree))


def sh_basis(degree: int, dirs) -> np.ndarray:
    """Real spherical harmonics (Condon-Shortley phase) of unit directions [n, 3]: [n, (degree+1)^2],
    and their polynomial gradients [n, (degree+1)^2, 3]."""
    d = _f64(dirs, (-1, 3))
    n = d.shape[0]
    K = (degree + 1) ** 2
    Y = np.zeros((n, K)); G = np.zeros((n, K, 3))
    lib().or_sh_basis(degree, n, _p(d), _p(Y), _p(G))
    return Y, G


def depth_keys(prims: dict, cam: Camera) -> np.ndarray:
    """FP32 depth keys (uint32 bit patterns) defining the alpha compositing order."""
    n = int(np.asarray(prims["opacity"]).shape[0])
    mean = _f32(prims["mean"], (n, 3))
    vel = _f32(prims.get("velocity"), (n, 3)) if prims.get("velocity") is not None else None
    W = np.ascontiguousarray(np.asarray(cam.viewmat, dtype=np.float64).reshape(16).astype(np.float32))
    out = np.zeros(n, dtype=np.uint32)
    lib().or_depth_keys(n, _p(mean), _p(vel), C.c_float(np.float32(cam.time)), _p(W), _p(out))
    return out


def _keys_or_none(params, keys):
    if params.mode != MODE_ALPHA3D:
        return None
    return np.ascontiguousarray(np.asarray(keys, dtype=np.uint32))


def render_o1(params: Params, W: int, H: int, screen: np.ndarray, keys=None, pix=None, jump: bool = False):
    """O1 brute force.  Returns (image [npix,3], T_final [npix], n_contrib [npix], tie [npix]) and, with
    jump=True, the tie jump bounds [npix, 2] (image value, final T) as a fifth item."""
    screen = np.ascontiguousarray(screen, dtype=np.float64)
    n = screen.shape[0]
    pix = None if pix is None else np.ascontiguousarray(np.asarray(pix, dtype=np.int64))
    npix = W * H if pix is None else pix.shape[0]
    img = np.zeros((npix, 3)); T = np.zeros(npix); nc = np.zeros(npix, np.int32); tie = np.zeros(npix, np.uint8)
    jb = np.zeros((npix, 2))
    k = _keys_or_none(params, keys)
    cp = params.c()
    lib().or_render_o1(C.byref(cp), W, H, n, _p(screen), _p(k), npix, _p(pix), _p(img), _p(T), _p(nc), _p(tie),
                       _p(jb))
    return (img, T, nc, tie, jb) if jump else (img, T, nc, tie)


def render_bwd_o1(params: Params, W: int, H: int, screen: np.ndarray, dLdC, keys=None, pix=None, max_threads=0):
    """O1 backward.  dLdC is [npix, 3] for the listed pixels.  Returns dscreen [n, 11]."""
    screen = np.ascontiguousarray(screen, dtype=np.float64)
    n = screen.shape[0]
    pix = None if pix is None else np.ascontiguousarray(np.asarray(pix, dtype=np.int64))
    npix = W * H if pix is None else pix.shape[0]
    g = np.ascontiguousarray(np.asarray(dLdC, dtype=np.float64).reshape(npix, 3))
    out = np.zeros((n, SG_N))
    k = _keys_or_none(params, keys)
    cp = params.c()
    lib().or_render_bwd_o1(C.byref(cp), W, H, n, _p(screen), _p(k), npix, _p(pix), _p(g), _p(out), max_threads)
    return out


def render_o2(params: Params, W: int, H: int, screen: np.ndarray, keys=None, jump: bool = False):
    """O2 support scatter over the full image.  Returns (image [H,W,3], T [H,W], last_id [H,W], tie [H,W])
    and, with jump=True, the tie jump bounds [H,W,2] as a fifth item."""
    screen = np.ascontiguousarray(screen, dtype=np.float64)
    n = screen.shape[0]
    img = np.zeros((H, W, 3)); T = np.zeros((H, W)); last = np.zeros((H, W), np.int32)
    tie = np.zeros((H, W), np.uint8)
    jb = np.zeros((H, W, 2))
    k = _keys_or_none(params, keys)
    cp = params.c()
    lib().or_render_o2(C.byref(cp), W, H, n, _p(screen), _p(k), _p(img), _p(T), _p(last), _p(tie), _p(jb))
    return (img, T, last, tie, jb) if jump else (img, T, last, tie)


def render_bwd_o2(params: Params, W: int, H: int, screen: np.ndarray, T_final, last_id, dLdC, keys=None,
                  max_threads=0):
    """O2 backward over the full image (dLdC [H,W,3]).  Returns dscreen [n, 11]."""
    screen = np.ascontiguousarray(screen, dtype=np.float64)
    n = screen.shape[0]
    T = np.ascontiguousarray(np.asarray(T_final, dtype=np.float64).reshape(H * W))
    last = np.ascontiguousarray(np.asarray(last_id, dtype=np.int32).reshape(H * W))
    g = np.ascontiguousarray(np.asarray(dLdC, dtype=np.float64).reshape(H * W, 3))
    out = np.zeros((n, SG_N))
    k = _keys_or_none(params, keys)
    cp = params.c()
    lib().or_render_bwd_o2(C.byref(cp), W, H, n, _p(screen), _p(k), _p(T), _p(last), _p(g), _p(out), max_threads)
    return out


def project_bwd(params: Params, prims: dict, screen: np.ndarray, dscreen: np.ndarray, cam: Camera | None = None):
    """Chain rule from screen-space gradients to parameter gradients (dict of FP64 arrays)."""
    n = int(np.asarray(prims["opacity"]).shape[0])
    three_d = params.mode == MODE_ALPHA3D
    q = _prims(prims, n, three_d)
    d = 3 if three_d else 2
    _check_sh(params, q, n)
    out = dict(mean=np.zeros((n, d)), freq=np.zeros((n, d)), color=np.zeros((n, 3)), opacity=np.zeros(n),
               phase=np.zeros(n))
    if q["sh"] is not None and params.sh_degree >= 0:
        out["sh"] = np.zeros_like(q["sh"])
    if three_d:
        out.update(quat=np.zeros((n, 4)), scale=np.zeros((n, 3)))
        if q["velocity"] is not None:
            out["velocity"] = np.zeros((n, 3))
    else:
        out["cov"] = np.zeros((n, 3))
    screen = np.ascontiguousarray(screen, dtype=np.float64)
    dscreen = np.ascontiguousarray(dscreen, dtype=np.float64)
    if dscreen.shape[1] < SG_N:   # screen gradients without the phase column
        dscreen = np.ascontiguousarray(np.concatenate([dscreen, np.zeros((n, SG_N - dscreen.shape[1]))], 1))
    cp = params.c()
    cc = cam.c() if cam is not None else None
    lib().or_project_bwd(C.byref(cp), C.byref(cc) if cc is not None else None, n, _p(q["mean"]), _p(q["cov"]),
                         _p(q["quat"]), _p(q["scale"]), _p(q["freq"]), _p(q["opacity"]), _p(q["velocity"]),
                         _p(q["sh"]), _p(screen), _p(dscreen), _p(out["mean"]), _p(out.get("cov")),
                         _p(out.get("quat")), _p(out.get("scale")), _p(out["freq"]), _p(out["color"]),
                         _p(out["opacity"]), _p(out.get("velocity")), _p(out["phase"]), _p(out.get("sh")))
    if "sh" in out:
        out["sh"] = out["sh"].reshape(np.asarray(prims["sh"]).shape)
    return out


def bin_tiles(W: int, H: int, tw: int, th: int, mode: int, mx, my, rx, ry, depth, ca, cb, cc, Qs):
    """O-bin (FP32 rule: pixel box, then the tiles of its rectangle whose pixel-centre rectangle the
    padded support ellipse q <= Qs reaches, conic (ca, cb, cc); rectangles of more than 64 tiles keep
    every tile).  Returns dict(box [n,4], count [n], K, keys u64 [K], vals u32 [K], ranges [T,2])."""
    mx, my, rx, ry, depth, ca, cb, cc, Qs = (np.ascontiguousarray(np.asarray(a, dtype=np.float32))
                                             for a in (mx, my, rx, ry, depth, ca, cb, cc, Qs))
    n = mx.shape[0]
    box = np.zeros((n, 4), np.int32)
    count = np.zeros(n, np.int32)
    K = C.c_int64(0)
    L = lib()
    args = [_p(mx), _p(my), _p(rx), _p(ry), _p(depth), _p(ca), _p(cb), _p(cc), _p(Qs)]
    L.or_bin(W, H, tw, th, mode, n, *args, _p(box), _p(count), C.byref(K), None, None, None)
    Kv = K.value
    tiles = ((W + tw - 1) // tw) * ((H + th - 1) // th)
    keys = np.zeros(max(Kv, 1), np.uint64)
    vals = np.zeros(max(Kv, 1), np.uint32)
    ranges = np.zeros((tiles, 2), np.uint32)
    L.or_bin(W, H, tw, th, mode, n, *args, _p(box), _p(count), C.byref(K), _p(keys), _p(vals), _p(ranges))
    return dict(box=box, count=count, K=Kv, keys=keys[:Kv], vals=vals[:Kv], ranges=ranges)


def support_counts(params: Params, W: int, H: int, screen: np.ndarray, keys=None, pix=None):
    """Per listed pixel: (support pairs the forward evaluates, support pairs the backward revisits)."""
    screen = np.ascontiguousarray(screen, dtype=np.float64)
    n = screen.shape[0]
    pix = None if pix is None else np.ascontiguousarray(np.asarray(pix, dtype=np.int64))
    npix = W * H if pix is None else pix.shape[0]
    fwd = np.zeros(npix, np.int64)
    bwd = np.zeros(npix, np.int64)
    k = _keys_or_none(params, keys)
    cp = params.c()
    lib().or_support_counts(C.byref(cp), W, H, n, _p(screen), _p(k), npix, _p(pix), _p(fwd), _p(bwd))
    return fwd, bwd
