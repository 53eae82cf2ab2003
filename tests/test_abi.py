"""The C-ABI library loads and exports every entry point include/wipes.h
declares; host-only calls (defaults, workspace sizing, argument validation)
behave as documented.  No device work is issued, so this runs without a GPU."""
import ctypes as C
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "wipes.h")


def declared():
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(wipes_[a-z_0-9]+)\s*\(", txt)))


@pytest.fixture(scope="module")
def B():
    from paper_2508_12615_amd import binding
    try:
        binding.lib()
    except ImportError as e:  # pragma: no cover
        pytest.fail(str(e))
    return binding


def test_every_declared_symbol_is_exported(B):
    names = declared()
    assert "wipes_render_bwd" in names and len(names) >= 11
    out = subprocess.run(["nm", "-D", "--defined-only", B.LIB_PATH], capture_output=True, text=True).stdout
    exported = set(re.findall(r" T (wipes_\w+)", out))
    missing = [n for n in names if n not in exported]
    assert not missing, missing


def test_params_default(B):
    p = B.wipes_params_default(B.WIPES_3D_ALPHA)
    assert (p.tile_w, p.tile_h, p.cov, p.persistent) == (16, 16, B.WIPES_COV_QUAT_SCALE, 3)
    assert abs(p.alpha_min - 1 / 255) < 1e-9 and abs(p.alpha_max - 0.99) < 1e-7 and abs(p.T_min - 1e-4) < 1e-10
    assert abs(p.blur_eps - 0.3) < 1e-7 and p.q_add == 9.0
    q = B.wipes_params_default(B.WIPES_2D_ADDITIVE)
    assert q.blur_eps == 0.0 and q.cov == B.WIPES_COV_RS


def _batch(B, n, W=64, H=48, fx=1.0):
    img = B.wipes_image()
    img.cam.width, img.cam.height, img.cam.fx, img.cam.fy = W, H, fx, fx
    img.prims.n = n
    for k in ("mean", "cov", "quat", "scale", "freq", "color", "opacity"):
        setattr(img.prims, k, 0x1000)   # never dereferenced by host-only calls
    arr = (B.wipes_image * 1)(img)
    return B.wipes_batch(1, arr), arr


def test_workspace_size_grows_with_inputs(B):
    p = B.wipes_params_default(B.WIPES_3D_ALPHA)
    b, keep = _batch(B, 1000)
    s0, b0 = B.wipes_workspace_size(p, b, 10_000, False)
    s1, b1 = B.wipes_workspace_size(p, b, 20_000, True)
    assert s0 == s1 and b1 > b0 + 10_000 * 48
    b2, keep2 = _batch(B, 5000)
    s2, _ = B.wipes_workspace_size(p, b2, 10_000, False)
    assert s2 >= s0 + 4000 * (64 + 16)


@pytest.mark.parametrize("bad", ["tile", "cov", "alpha", "size", "freq", "sh_degree", "sh_missing", "sh_2d",
                                 "lds_batch", "launch_form"])
def test_validation_rejects_bad_arguments(B, bad):
    p = B.wipes_params_default(B.WIPES_3D_ALPHA if bad != "sh_2d" else B.WIPES_2D_ADDITIVE)
    b, keep = _batch(B, 10)
    if bad == "tile":
        p.tile_w = 12
    elif bad == "cov":
        p.cov = B.WIPES_COV_RS
    elif bad == "alpha":
        p.alpha_max = 1.5
    elif bad == "size":
        b.images[0].cam.width = 0
    elif bad == "freq":
        p.freq_xform = 7
    elif bad == "sh_degree":
        p.sh_degree = 4
    elif bad == "sh_missing":   # spherical-harmonic colour without coefficients
        p.sh_degree = 1
    elif bad == "sh_2d":
        p.sh_degree = 0
    elif bad == "lds_batch":
        p.lds_batch = 128
    elif bad == "launch_form":
        p.persistent = 4
    sb, bb = C.c_size_t(), C.c_size_t()
    st = B.lib().wipes_workspace_size(C.byref(p), C.byref(b), 100, 0, C.byref(sb), C.byref(bb))
    assert st == B.WIPES_ERR_INVALID
    assert B.last_error(None)


def test_null_context_is_rejected_before_any_device_work(B):
    p = B.wipes_params_default(B.WIPES_2D_ADDITIVE)
    b, keep = _batch(B, 10)
    buf = B.wipes_buffer(0x1000, 1 << 20, 0, 0, 0)
    assert B.lib().wipes_project(None, C.byref(p), C.byref(b), C.byref(buf), None) == B.WIPES_ERR_INVALID
    k = C.c_int64()
    assert B.lib().wipes_bin_sort(None, C.byref(p), C.byref(b), C.byref(buf), C.byref(buf), C.byref(k),
                                  None) == B.WIPES_ERR_INVALID


def test_missing_library_raises(monkeypatch):
    """Without the built library the binding refuses to load: there is no fallback path."""
    from paper_2508_12615_amd import binding
    monkeypatch.setattr(binding, "_lib", None)
    monkeypatch.setattr(binding, "LIB_PATH", os.path.join(os.path.dirname(binding.LIB_PATH), "no_such_libwipes.so"))
    with pytest.raises(ImportError):
        binding.lib()
