"""FP64 reference of the deformation network of Eq. 8 -- TEST INFRASTRUCTURE ONLY.

Only the test suite, the smoke check and the CPU-baseline leg of the
benchmark may import this module; the library never does.  Plain numpy in
FP64; a matrix product is the one library primitive used.

Paper: arXiv 2508.12615, Sec. 4.3, Eq. 8: for dynamic scenes a network F_theta
maps the positional encodings of a primitive's position and of the time to
offsets of its position, frequency and covariance, (dx, df, dSigma) =
F_theta(gamma(x), gamma(t)); the same form as the D-3DGS deformation field of
Sec. 3.2, whose configuration the paper keeps for its other settings (Sec. 5.3).

Readings (the paper prints no architecture; D-3DGS's is taken):
  * gamma(p) = (p, sin(2^0 pi p), cos(2^0 pi p), ..., sin(2^(L-1) pi p),
    cos(2^(L-1) pi p)) with the d components of p kept together inside each
    block; L = 10 for the position (3 -> 63), L = 6 for the time (1 -> 13);
    e = (gamma(x), gamma(t)), 76 values;
  * 8 hidden layers of 256 units with ReLU; the encoding e is concatenated to
    the output of the fifth layer (the sixth layer reads 256 + 76 inputs);
  * one linear output layer of 13 values: dx (3), df (3), dq (4, added to the
    quaternion), ds (3, added to the linear scales) -- dSigma in the
    rotation/scale form the covariance is parameterised by (Sec. 3.1).
Parameters are one flat float array: W0 [256, 76], b0 [256], W1..W4 [256, 256]
with their biases, W5 [256, 332], b5, W6, W7 [256, 256] with their biases,
Wo [13, 256], bo [13]; a weight matrix is row-major [out, in].
"""
from __future__ import annotations

import numpy as np

LX, LT = 10, 6
WIDTH, DEPTH, SKIP = 256, 8, 5     # SKIP: index of the layer that also reads the encoding
N_IN = 3 * (1 + 2 * LX) + 1 * (1 + 2 * LT)   # 76
N_OUT = 13


def layer_shapes():
    """(out, in) of every layer, the output layer last."""
    shapes = []
    for l in range(DEPTH):
        fan_in = N_IN if l == 0 else WIDTH + (N_IN if l == SKIP else 0)
        shapes.append((WIDTH, fan_in))
    shapes.append((N_OUT, WIDTH))
    return shapes


def param_count() -> int:
    return sum(o * i + o for o, i in layer_shapes())


def unpack(params):
    """List of (W, b) views into the flat parameter array (FP64 copy)."""
    p = np.asarray(params, dtype=np.float64).reshape(-1)
    assert p.size == param_count()
    out, o = [], 0
    for (m, k) in layer_shapes():
        W = p[o:o + m * k].reshape(m, k)
        o += m * k
        b = p[o:o + m]
        o += m
        out.append((W, b))
    return out


def _gamma(p, L):
    """gamma of an [n, d] array: [n, d (1 + 2L)]."""
    p = np.asarray(p, dtype=np.float64)
    parts = [p]
    for k in range(L):
        a = (2.0 ** k) * np.pi * p
        parts += [np.sin(a), np.cos(a)]
    return np.concatenate(parts, axis=1)


def _dgamma(p, L):
    """d gamma / d p per component: [n, d (1 + 2L)] (each entry depends on one component of p)."""
    p = np.asarray(p, dtype=np.float64)
    parts = [np.ones_like(p)]
    for k in range(L):
        w = (2.0 ** k) * np.pi
        a = w * p
        parts += [w * np.cos(a), -w * np.sin(a)]
    return np.concatenate(parts, axis=1)


def encode(x, t):
    """e = (gamma(x), gamma(t)) for positions x [n, 3] and one time t: [n, 76]."""
    x = np.asarray(x, dtype=np.float64).reshape(-1, 3)
    tt = np.full((x.shape[0], 1), float(t))
    return np.concatenate([_gamma(x, LX), _gamma(tt, LT)], axis=1)


def forward(params, x, t, keep=False):
    """Offsets [n, 13] = (dx, df, dq, ds); with keep=True also the layer inputs and
    pre-activations the backward needs."""
    layers = unpack(params)
    e = encode(x, t)
    h = e
    saved = []
    for l in range(DEPTH):
        W, b = layers[l]
        inp = np.concatenate([h, e], axis=1) if l == SKIP else h
        z = inp @ W.T + b
        saved.append((inp, z))
        h = np.maximum(z, 0.0)
    Wo, bo = layers[DEPTH]
    out = h @ Wo.T + bo
    return (out, (e, saved, h)) if keep else out


def backward(params, x, t, dout):
    """Gradients for the upstream dL/d(offsets) [n, 13]: (d params (flat, like params),
    dL/dx [n, 3], dL/dt (scalar))."""
    layers = unpack(params)
    out, (e, saved, hL) = forward(params, x, t, keep=True)
    dout = np.asarray(dout, dtype=np.float64).reshape(-1, N_OUT)
    grads = [None] * (DEPTH + 1)
    Wo, bo = layers[DEPTH]
    grads[DEPTH] = (dout.T @ hL, dout.sum(axis=0))
    dh = dout @ Wo
    de = np.zeros_like(e)
    for l in range(DEPTH - 1, -1, -1):
        inp, z = saved[l]
        W, b = layers[l]
        dz = dh * (z > 0.0)
        grads[l] = (dz.T @ inp, dz.sum(axis=0))
        dinp = dz @ W
        if l == SKIP:
            dh = dinp[:, :WIDTH]
            de += dinp[:, WIDTH:]
        elif l == 0:
            de += dinp
        else:
            dh = dinp
    x = np.asarray(x, dtype=np.float64).reshape(-1, 3)
    nx = 3 * (1 + 2 * LX)
    gx = de[:, :nx] * _dgamma(x, LX)
    dx = np.zeros_like(x)
    for c in range(3):   # entries c, c + 3, c + 6, ... belong to component c
        dx[:, c] = gx[:, c::3].sum(axis=1)
    tt = np.full((x.shape[0], 1), float(t))
    dt = float((de[:, nx:] * _dgamma(tt, LT)).sum())
    flat = np.concatenate([np.concatenate([g[0].reshape(-1), g[1]]) for g in grads])
    return flat, dx, dt


def apply(prims, offsets):
    """Deformed primitives: mean + dx, freq + df, quat + dq, scale + ds (other keys unchanged)."""
    d = np.asarray(offsets, dtype=np.float64)
    out = dict(prims)
    out["mean"] = np.asarray(prims["mean"], np.float64) + d[:, 0:3]
    out["freq"] = np.asarray(prims["freq"], np.float64) + d[:, 3:6]
    out["quat"] = np.asarray(prims["quat"], np.float64) + d[:, 6:10]
    out["scale"] = np.asarray(prims["scale"], np.float64) + d[:, 10:13]
    return out
