"""Pins of the FP64 deformation-network oracle (Eq. 8, oracle/deform.py), each
against something other than the oracle itself:

* the encoding: its first block is the input, every frequency block satisfies
  sin^2 + cos^2 = 1, consecutive blocks satisfy the double-angle identities
  (a wrong exponent or a missing pi breaks them), and gamma(0) is known;
* the architecture: parameter sets for which the network computes a closed
  form -- identity hidden layers pass one encoding entry through every layer,
  and the skip layer routes a chosen encoding entry straight to the output --
  so a wrong depth, skip position or concatenation order changes the value;
* the backward: FP64 central finite differences of the forward for the
  parameters, the position and the time;
* planted mistakes in a patched copy of the module are caught by these pins.
"""
import importlib.util
import math
import os

import numpy as np
import pytest

import deform as D

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _params(seed, head=0.05):
    g = np.random.default_rng(seed)
    parts = []
    for l, (m, k) in enumerate(D.layer_shapes()):
        s = 1.0 / math.sqrt(k)
        W = g.uniform(-s, s, (m, k)) * (head if l == D.DEPTH else 1.0)
        b = g.uniform(-s, s, m) * (head if l == D.DEPTH else 1.0)
        parts += [W.reshape(-1), b]
    return np.concatenate(parts)


# the reading: the encoding joins the output of the fifth layer, so layer index 5 reads 256 + 76
SKIP_LAYER = 5


def test_architecture_size():
    shapes = D.layer_shapes()
    assert D.N_IN == 76 and shapes[0] == (256, 76) and shapes[SKIP_LAYER] == (256, 332)
    assert all(shapes[l] == (256, 256) for l in range(1, 8) if l != SKIP_LAYER) and shapes[8] == (13, 256)
    assert D.param_count() == 256 * 76 + 256 + 6 * (256 * 256 + 256) + 256 * 332 + 256 + 13 * 256 + 13


def test_encoding_identities():
    g = np.random.default_rng(1)
    x = g.uniform(-1, 2, (50, 3))
    t = 0.37
    e = D.encode(x, t)
    assert e.shape == (50, 76)
    np.testing.assert_array_equal(e[:, :3], x)
    for k in range(D.LX):
        s = e[:, 3 + 6 * k: 6 + 6 * k]
        c = e[:, 6 + 6 * k: 9 + 6 * k]
        np.testing.assert_allclose(s * s + c * c, 1.0, atol=1e-14)
        np.testing.assert_allclose(s, np.sin((2.0 ** k) * math.pi * x), atol=1e-12)
        if k + 1 < D.LX:   # double angle: sin 2a = 2 sin a cos a, cos 2a = cos^2 a - sin^2 a
            s2 = e[:, 3 + 6 * (k + 1): 6 + 6 * (k + 1)]
            c2 = e[:, 6 + 6 * (k + 1): 9 + 6 * (k + 1)]
            np.testing.assert_allclose(s2, 2 * s * c, atol=1e-12)
            np.testing.assert_allclose(c2, c * c - s * s, atol=1e-12)
    te = e[:, 63:]
    assert np.all(te[:, 0] == t)
    np.testing.assert_allclose(te[:, 1], math.sin(math.pi * t), atol=1e-15)
    np.testing.assert_allclose(te[:, 2], math.cos(math.pi * t), atol=1e-15)
    e0 = D.encode(np.zeros((1, 3)), 0.0)[0]
    expect = np.concatenate([np.zeros(3)] + [np.r_[np.zeros(3), np.ones(3)] for _ in range(D.LX)] +
                            [np.zeros(1)] + [np.r_[0.0, 1.0] for _ in range(D.LT)])
    np.testing.assert_array_equal(e0, expect)


def _identity_net(src, dst_unit=0, skip_src=None):
    """Hidden layers pass unit dst_unit through unchanged (identity rows), layer 0 copies encoding
    entry src into it; the skip layer's encoding block is zero unless skip_src is given, in which
    case it routes that encoding entry into unit 1, which the output's row 1 reads."""
    shapes = D.layer_shapes()
    Ws = [np.zeros(s) for s in shapes]
    bs = [np.zeros(s[0]) for s in shapes]
    Ws[0][dst_unit, src] = 1.0
    for l in range(1, D.DEPTH):
        Ws[l][:, :D.WIDTH] = np.eye(D.WIDTH)
    if skip_src is not None:
        Ws[SKIP_LAYER][1, :D.WIDTH] = 0.0
        Ws[SKIP_LAYER][1, D.WIDTH + skip_src] = 1.0
    Ws[D.DEPTH][0, dst_unit] = 1.0
    Ws[D.DEPTH][1, 1] = 1.0
    bs[D.DEPTH][2] = 0.25
    return np.concatenate([np.concatenate([W.reshape(-1), b]) for W, b in zip(Ws, bs)])


def test_closed_form_networks():
    g = np.random.default_rng(2)
    x = g.uniform(0.05, 0.95, (20, 3))
    t = 0.6
    # one positive encoding entry (x_1) through all eight ReLU layers and the output
    out = D.forward(_identity_net(1), x, t)
    np.testing.assert_allclose(out[:, 0], x[:, 1], atol=1e-15)
    np.testing.assert_allclose(out[:, 2], 0.25, atol=1e-15)
    assert np.all(out[:, 3:] == 0.0)
    # a negative input is cut by the first ReLU
    out = D.forward(_identity_net(1), -x, t)
    assert np.all(out[:, 0] == 0.0)
    # the skip layer reads the encoding after the 256 hidden units: entry 63 is t itself,
    # entry 64 is sin(pi t) (positive for t in (0, 1))
    out = D.forward(_identity_net(0, skip_src=63), x, t)
    np.testing.assert_allclose(out[:, 1], t, atol=1e-15)
    out = D.forward(_identity_net(0, skip_src=64), x, t)
    np.testing.assert_allclose(out[:, 1], math.sin(math.pi * t), atol=1e-15)


def test_fd_backward():
    g = np.random.default_rng(3)
    p = _params(4, head=0.3)
    x = g.uniform(0, 1, (5, 3))
    t = 0.41
    dout = g.normal(0, 1, (5, D.N_OUT))
    dp, dx, dt = D.backward(p, x, t, dout)
    L = lambda pp, xx, tt: float((D.forward(pp, xx, tt) * dout).sum())  # noqa: E731
    h = 1e-6
    # parameters: a sample from every layer's weights and biases
    o = 0
    idx = []
    for (m, k) in D.layer_shapes():
        idx += list(g.integers(o, o + m * k, 4)) + list(g.integers(o + m * k, o + m * k + m, 2))
        o += m * k + m
    for i in idx:
        e = np.zeros_like(p); e[i] = h
        fd = (L(p + e, x, t) - L(p - e, x, t)) / (2 * h)
        assert abs(fd - dp[i]) <= 1e-6 * max(1.0, abs(fd)), (i, fd, dp[i])
    hx = 1e-8   # the encoding reaches 2^9 pi rad per unit: a small step keeps the FD truncation low
    for i in range(5):
        for c in range(3):
            e = np.zeros_like(x); e[i, c] = hx
            fd = (L(p, x + e, t) - L(p, x - e, t)) / (2 * hx)
            assert abs(fd - dx[i, c]) <= 1e-6 * max(1.0, abs(fd)), (i, c, fd, dx[i, c])
    fd = (L(p, x, t + hx) - L(p, x, t - hx)) / (2 * hx)
    assert abs(fd - dt) <= 1e-6 * max(1.0, abs(fd))


def test_apply_offsets():
    g = np.random.default_rng(5)
    prims = dict(mean=g.normal(0, 1, (4, 3)), freq=g.normal(0, 1, (4, 3)), quat=g.normal(0, 1, (4, 4)),
                 scale=g.uniform(0, 1, (4, 3)), opacity=np.ones(4))
    d = g.normal(0, 1, (4, 13))
    q = D.apply(prims, d)
    np.testing.assert_array_equal(q["mean"], prims["mean"] + d[:, :3])
    np.testing.assert_array_equal(q["freq"], prims["freq"] + d[:, 3:6])
    np.testing.assert_array_equal(q["quat"], prims["quat"] + d[:, 6:10])
    np.testing.assert_array_equal(q["scale"], prims["scale"] + d[:, 10:13])


# ---------------------------------------------------------------- mutations

MUTATIONS = {
    "skip one layer late": ("WIDTH, DEPTH, SKIP = 256, 8, 5", "WIDTH, DEPTH, SKIP = 256, 8, 6",
                            ["test_architecture_size", "test_closed_form_networks"]),
    "encoding without pi": ("a = (2.0 ** k) * np.pi * p", "a = (2.0 ** k) * p", ["test_encoding_identities"]),
    "encoding frequencies off by one": ("a = (2.0 ** k) * np.pi * p", "a = (2.0 ** (k + 1)) * np.pi * p",
                                        ["test_encoding_identities"]),
    "ReLU derivative passes negatives": ("dz = dh * (z > 0.0)", "dz = dh", ["test_fd_backward"]),
    "encoding derivative sign": ("parts += [w * np.cos(a), -w * np.sin(a)]", "parts += [w * np.cos(a), w * np.sin(a)]",
                                 ["test_fd_backward"]),
    "skip gradient dropped": ("de += dinp[:, WIDTH:]", "pass", ["test_fd_backward"]),
}


@pytest.mark.parametrize("name", sorted(MUTATIONS))
def test_pins_catch_planted_mistake(name):
    old, new, tests = MUTATIONS[name]
    src = open(os.path.join(ROOT, "oracle", "deform.py")).read()
    assert src.count(old) == 1, name
    spec = importlib.util.spec_from_loader("deform_mutant", loader=None)
    mod = importlib.util.module_from_spec(spec)
    exec(compile(src.replace(old, new), "deform_mutant", "exec"), mod.__dict__)
    caught = False
    for tname in tests:
        fn = globals()[tname]
        fn.__globals__["D"] = mod
        try:
            fn()
        except (AssertionError, IndexError, ValueError):   # a pin failing, or unable to run, on the mutant
            caught = True
        finally:
            fn.__globals__["D"] = D
    assert caught, name
