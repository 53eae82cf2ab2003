"""ctypes binding of libwipes.so: the C ABI of include/wipes.h, one Python
function per entry point with the same name.  Argument marshalling only --
every step of the render path runs in the HIP library.  Importing this module
fails loudly if the library has not been built (there is no fallback).
"""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libwipes.so")

WIPES_OK, WIPES_ERR_INVALID, WIPES_ERR_NOMEM, WIPES_ERR_CAPACITY = 0, 1, 2, 3
WIPES_ERR_DEVICE, WIPES_ERR_BUSY, WIPES_ERR_NOTFOUND = 4, 5, 6
WIPES_2D_ADDITIVE, WIPES_3D_ALPHA = 0, 1
WIPES_COV_CHOLESKY, WIPES_COV_RS, WIPES_COV_QUAT_SCALE = 0, 1, 2
WIPES_FREQ_VECTOR, WIPES_FREQ_COVECTOR = 0, 1

STATUS_NAMES = {0: "OK", 1: "INVALID", 2: "NOMEM", 3: "CAPACITY", 4: "DEVICE", 5: "BUSY", 6: "NOTFOUND"}


class WipesError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__("wipes status %s: %s" % (STATUS_NAMES.get(status, status), msg))
        self.status = status


class wipes_params(C.Structure):
    _fields_ = [("mode", C.c_int32), ("cov", C.c_int32), ("freq_xform", C.c_int32), ("tile_w", C.c_int32),
                ("tile_h", C.c_int32), ("persistent", C.c_int32), ("alpha_min", C.c_float),
                ("alpha_max", C.c_float), ("T_min", C.c_float), ("q_add", C.c_float), ("blur_eps", C.c_float),
                ("near_plane", C.c_float), ("fov_guard", C.c_float), ("bg", C.c_float * 3),
                ("sh_degree", C.c_int32), ("lds_batch", C.c_int32)]


class wipes_camera(C.Structure):
    _fields_ = [("width", C.c_int32), ("height", C.c_int32), ("fx", C.c_float), ("fy", C.c_float),
                ("cx", C.c_float), ("cy", C.c_float), ("viewmat", C.c_float * 16), ("time", C.c_float)]


_PRIM_FIELDS = ["mean", "cov", "quat", "scale", "freq", "color", "opacity", "velocity", "phase", "sh"]


class wipes_prims(C.Structure):
    _fields_ = [("n", C.c_int64)] + [(f, C.c_void_p) for f in _PRIM_FIELDS]


class wipes_prims_grad(C.Structure):
    _fields_ = [(f, C.c_void_p) for f in _PRIM_FIELDS]


class wipes_image(C.Structure):
    _fields_ = [("cam", wipes_camera), ("prims", wipes_prims), ("grads", wipes_prims_grad), ("out_image", C.c_void_p)]


class wipes_batch(C.Structure):
    _fields_ = [("n_images", C.c_int32), ("images", C.POINTER(wipes_image))]


class wipes_buffer(C.Structure):
    _fields_ = [("base", C.c_void_p), ("bytes", C.c_size_t), ("capacity", C.c_int64),
                ("with_backward", C.c_int32), ("reserved", C.c_int32)]


_lib = None


def lib() -> C.CDLL:
    """Load libwipes.so (built in-tree).  Raises if it is missing."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError("libwipes.so is not built (%s); run `python -m paper_2508_12615_amd.build`" % LIB_PATH)
    L = C.CDLL(LIB_PATH)
    P, PP = C.c_void_p, C.POINTER
    sig = {
        "wipes_params_default": (None, [C.c_int32, PP(wipes_params)]),
        "wipes_ctx_create": (C.c_int, [C.c_int32, PP(C.c_void_p)]),
        "wipes_ctx_destroy": (None, [P]),
        "wipes_last_error": (C.c_char_p, [P]),
        "wipes_workspace_size": (C.c_int, [PP(wipes_params), PP(wipes_batch), C.c_int64, C.c_int32,
                                           PP(C.c_size_t), PP(C.c_size_t)]),
        "wipes_project": (C.c_int, [P, PP(wipes_params), PP(wipes_batch), PP(wipes_buffer), P]),
        "wipes_bin_sort": (C.c_int, [P, PP(wipes_params), PP(wipes_batch), PP(wipes_buffer), PP(wipes_buffer),
                                     PP(C.c_int64), P]),
        "wipes_render_fwd": (C.c_int, [P, PP(wipes_params), PP(wipes_batch), PP(wipes_buffer), PP(wipes_buffer),
                                       P, P, P, P]),
        "wipes_render_bwd": (C.c_int, [P, PP(wipes_params), PP(wipes_batch), PP(wipes_buffer), PP(wipes_buffer),
                                       P, P, P, P, P]),
        "wipes_check_overflow": (C.c_int, [P, PP(wipes_params), PP(wipes_batch), PP(wipes_buffer), PP(C.c_int64),
                                           P]),
        "wipes_bins_view": (C.c_int, [PP(wipes_params), PP(wipes_batch), PP(wipes_buffer), PP(wipes_buffer),
                                      PP(C.c_void_p), PP(C.c_void_p), PP(C.c_void_p), PP(C.c_int64)]),
    }
    sig.update({
        "wipes_render_fwd_noalloc": (C.c_int, [P, PP(wipes_params), PP(wipes_batch), P, P, P, PP(C.c_int64), P]),
        "wipes_stage_name": (C.c_char_p, [C.c_int32]),
        "wipes_probe_issue_rate": (C.c_int, [P, C.c_int32, PP(C.c_double), P]),
        "wipes_deform_param_count": (C.c_int64, []),
        "wipes_deform_workspace_size": (C.c_int, [C.c_int64, C.c_int32, PP(C.c_size_t)]),
        "wipes_deform_fwd": (C.c_int, [P, C.c_int32, P, C.c_int64, P, C.c_float, P, P, C.c_size_t, C.c_int32, P]),
        "wipes_deform_bwd": (C.c_int, [P, C.c_int32, P, C.c_int64, P, C.c_float, P, P, C.c_size_t, P, P, P]),
        "wipes_deform_apply": (C.c_int, [P, C.c_int64, P, P, P, P, P, P, P, P, P, P]),
        "wipes_profile_enable": (C.c_int, [P, C.c_int32]),
        "wipes_profile_read": (C.c_int, [P, PP(C.c_double), PP(C.c_int64), C.c_int32]),
        "wipes_render_stats": (C.c_int, [P, PP(wipes_params), PP(wipes_batch), PP(wipes_buffer), PP(wipes_buffer),
                                         P, P, PP(C.c_uint64), P]),
    })
    for name, (res, args) in sig.items():
        f = getattr(L, name)
        f.restype = res
        f.argtypes = args
    _extra_signatures(L)
    _lib = L
    return L


def _extra_signatures(L):
    """Signatures of the graph, autotune and serving entry points."""
    from . import binding_ext
    binding_ext.declare(L)


def last_error(ctx) -> str:
    s = lib().wipes_last_error(ctx)
    return s.decode() if s else ""


def check(status: int, ctx=None, allow=()):
    if status != WIPES_OK and status not in allow:
        raise WipesError(status, last_error(ctx))
    return status


# --------------------------------------------------------------- entry points

def wipes_params_default(mode: int) -> wipes_params:
    p = wipes_params()
    lib().wipes_params_default(mode, C.byref(p))
    return p


def wipes_ctx_create(device: int = 0):
    ctx = C.c_void_p()
    check(lib().wipes_ctx_create(device, C.byref(ctx)))
    return ctx


def wipes_ctx_destroy(ctx) -> None:
    lib().wipes_ctx_destroy(ctx)


def wipes_workspace_size(params: wipes_params, batch: wipes_batch, capacity: int, with_backward: bool):
    sb, bb = C.c_size_t(), C.c_size_t()
    check(lib().wipes_workspace_size(C.byref(params), C.byref(batch), int(capacity), int(bool(with_backward)),
                                     C.byref(sb), C.byref(bb)))
    return sb.value, bb.value


def wipes_project(ctx, params, batch, screen: wipes_buffer, stream: int = 0) -> None:
    check(lib().wipes_project(ctx, C.byref(params), C.byref(batch), C.byref(screen), stream), ctx)


def wipes_bin_sort(ctx, params, batch, screen: wipes_buffer, bins: wipes_buffer, stream: int = 0, sync: bool = True):
    """Returns (status, K): status is WIPES_OK or WIPES_ERR_CAPACITY (K = required instances)."""
    k = C.c_int64(-1)
    st = lib().wipes_bin_sort(ctx, C.byref(params), C.byref(batch), C.byref(screen), C.byref(bins),
                              C.byref(k) if sync else None, stream)
    check(st, ctx, allow=(WIPES_ERR_CAPACITY,))
    return st, k.value


def wipes_render_fwd(ctx, params, batch, screen, bins, image: int, T_final: int, last: int, stream: int = 0) -> None:
    check(lib().wipes_render_fwd(ctx, C.byref(params), C.byref(batch), C.byref(screen), C.byref(bins), image,
                                 T_final, last, stream), ctx)


def wipes_render_bwd(ctx, params, batch, screen, bins, T_final: int, last: int, dL_dimage: int, dscreen: int,
                     stream: int = 0) -> None:
    check(lib().wipes_render_bwd(ctx, C.byref(params), C.byref(batch), C.byref(screen), C.byref(bins), T_final,
                                 last, dL_dimage, dscreen, stream), ctx)


def wipes_render_fwd_noalloc(ctx, params, batch, image: int, T_final: int, last: int, stream: int = 0,
                             sync: bool = True):
    """Returns (status, K): status is WIPES_OK or WIPES_ERR_CAPACITY (K = required instances; -1 when
    sync is False, i.e. no host synchronisation)."""
    k = C.c_int64(-1)
    st = lib().wipes_render_fwd_noalloc(ctx, C.byref(params), C.byref(batch), image, T_final, last,
                                        C.byref(k) if sync else None, stream)
    check(st, ctx, allow=(WIPES_ERR_CAPACITY,))
    return st, k.value


def wipes_check_overflow(ctx, params, batch, screen, stream: int = 0):
    k = C.c_int64(-1)
    st = lib().wipes_check_overflow(ctx, C.byref(params), C.byref(batch), C.byref(screen), C.byref(k), stream)
    check(st, ctx, allow=(WIPES_ERR_CAPACITY,))
    return st, k.value


def wipes_bins_view(params, batch, screen, bins):
    keys, vals, ranges, nt = C.c_void_p(), C.c_void_p(), C.c_void_p(), C.c_int64()
    check(lib().wipes_bins_view(C.byref(params), C.byref(batch), C.byref(screen), C.byref(bins), C.byref(keys),
                                C.byref(vals), C.byref(ranges), C.byref(nt)))
    return keys.value, vals.value, ranges.value, nt.value


WIPES_N_STAGES = 11


def wipes_stage_name(stage: int) -> str:
    return lib().wipes_stage_name(stage).decode()


def wipes_profile_enable(ctx, enable: bool) -> None:
    check(lib().wipes_profile_enable(ctx, int(bool(enable))), ctx)


def wipes_profile_read(ctx):
    """{stage name: (total ms, launches)} since the last read."""
    ms = (C.c_double * WIPES_N_STAGES)()
    n = (C.c_int64 * WIPES_N_STAGES)()
    check(lib().wipes_profile_read(ctx, ms, n, WIPES_N_STAGES), ctx)
    return {wipes_stage_name(i): (ms[i], n[i]) for i in range(WIPES_N_STAGES)}


PROBE_OPS = ("fma", "exp2", "cos", "sin", "rcp")


def wipes_probe_issue_rate(ctx, op: str, stream: int = 0) -> float:
    """Sustained lane operations per second of one instruction (see wipes.h)."""
    r = C.c_double()
    check(lib().wipes_probe_issue_rate(ctx, PROBE_OPS.index(op), C.byref(r), stream), ctx)
    return r.value


WIPES_DEFORM_BF16X3, WIPES_DEFORM_BF16 = 0, 1


def wipes_deform_param_count() -> int:
    return int(lib().wipes_deform_param_count())


def wipes_deform_workspace_size(n: int, with_backward: bool) -> int:
    b = C.c_size_t()
    check(lib().wipes_deform_workspace_size(n, int(with_backward), C.byref(b)))
    return b.value


def wipes_deform_fwd(ctx, precision: int, params: int, n: int, mean: int, time: float, offsets: int,
                     workspace: int, workspace_bytes: int, keep_for_backward: bool, stream: int = 0) -> None:
    check(lib().wipes_deform_fwd(ctx, precision, params, n, mean, time, offsets, workspace, workspace_bytes,
                                 int(keep_for_backward), stream), ctx)


def wipes_deform_bwd(ctx, precision: int, params: int, n: int, mean: int, time: float, d_offsets: int,
                     workspace: int, workspace_bytes: int, d_params: int, d_mean: int, stream: int = 0) -> None:
    check(lib().wipes_deform_bwd(ctx, precision, params, n, mean, time, d_offsets, workspace, workspace_bytes,
                                 d_params, d_mean, stream), ctx)


def wipes_deform_apply(ctx, n: int, offsets: int, mean: int, freq: int, quat: int, scale: int, out_mean: int,
                       out_freq: int, out_quat: int, out_scale: int, stream: int = 0) -> None:
    check(lib().wipes_deform_apply(ctx, n, offsets, mean, freq, quat, scale, out_mean, out_freq, out_quat, out_scale,
                                   stream), ctx)


def wipes_render_stats(ctx, params, batch, screen, bins, T_final: int, last: int, stream: int = 0):
    out = (C.c_uint64 * 4)()
    check(lib().wipes_render_stats(ctx, C.byref(params), C.byref(batch), C.byref(screen), C.byref(bins), T_final,
                                   last, out, stream), ctx)
    return dict(support_fwd=out[0], support_bwd=out[1], tile_pairs=out[2], subblock_pairs=out[3])


def wipes_l2_grad(ctx, params, batch, screen, image: int, target: int, dL_dimage: int, stream: int = 0) -> None:
    check(lib().wipes_l2_grad(ctx, C.byref(params), C.byref(batch), C.byref(screen), image, target, dL_dimage,
                              stream), ctx)


def wipes_adam(ctx, groups, beta1: float, beta2: float, eps: float, step: int, params=None, batch=None,
               screen=None, stream: int = 0) -> None:
    """One Adam step over groups = [(param, grad, m, v, lr)] of float32 CUDA tensors (see wipes.h);
    step: device address of the uint32 step counter.  With (params, batch, screen) the step is
    skipped on the device when the last bin_sort on that screen buffer overflowed."""
    from .binding_ext import wipes_adam_group
    arr = (wipes_adam_group * len(groups))()
    for i, (p, g, m, v, lr) in enumerate(groups):
        for t in (p, g, m, v):
            if t.dtype != torch_float32() or not t.is_cuda or not t.is_contiguous() or t.numel() != p.numel():
                raise ValueError("Adam group %d: param, grad, m, v must be contiguous float32 CUDA tensors "
                                 "of equal size" % i)
        arr[i] = wipes_adam_group(p.data_ptr(), g.data_ptr(), m.data_ptr(), v.data_ptr(), p.numel(), float(lr))
    check(lib().wipes_adam(ctx, len(groups), arr, float(beta1), float(beta2), float(eps), step,
                           C.byref(params) if params is not None else None,
                           C.byref(batch) if batch is not None else None,
                           C.byref(screen) if screen is not None else None, stream), ctx)


def torch_float32():
    import torch
    return torch.float32


def wipes_graph_capture(ctx, params, batch, screen, bins, image: int, T_final, last, target, dL_dimage,
                        backward: bool):
    g = C.c_void_p()
    check(lib().wipes_graph_capture(ctx, C.byref(params), C.byref(batch), C.byref(screen), C.byref(bins), image,
                                    T_final, last, target, dL_dimage, int(bool(backward)), C.byref(g)), ctx)
    return g


def wipes_graph_launch(graph, stream: int = 0) -> None:
    check(lib().wipes_graph_launch(graph, stream))


def wipes_graph_destroy(graph) -> None:
    lib().wipes_graph_destroy(graph)
