"""Signatures of the optional C ABI groups (fitting, graph capture, autotuning,
serving), declared only for the symbols the loaded library exports."""
import ctypes as C


class wipes_serve_config(C.Structure):
    _fields_ = [("max_slots", C.c_int32), ("max_pending", C.c_int32), ("max_batch", C.c_int32),
                ("persistent", C.c_int32), ("hbm_budget_bytes", C.c_int64)]


class wipes_serve_report(C.Structure):
    _fields_ = [("p50_ms", C.c_double), ("p99_ms", C.c_double), ("mean_ms", C.c_double),
                ("frames_per_s", C.c_double), ("completed", C.c_int64), ("admitted", C.c_int64),
                ("deferred", C.c_int64), ("batches", C.c_int64), ("mean_batch", C.c_double),
                ("arena_peak_bytes", C.c_int64)]


class wipes_adam_group(C.Structure):
    _fields_ = [("param", C.c_void_p), ("grad", C.c_void_p), ("m", C.c_void_p), ("v", C.c_void_p),
                ("n", C.c_int64), ("lr", C.c_double)]


WIPES_ADAM_MAX_GROUPS = 8


def declare(L) -> None:
    from .binding import wipes_batch, wipes_buffer, wipes_camera, wipes_params, wipes_prims
    P, PP = C.c_void_p, C.POINTER
    D, I64 = PP(C.c_double), PP(C.c_int64)
    table = {
        "wipes_autotune_candidates": (C.c_int32, [P, P, P, C.c_int32]),
        "wipes_autotune": (C.c_int, [P, PP(wipes_params), PP(wipes_batch), C.c_int32, C.c_int32, PP(wipes_params),
                                     D, P]),
        "wipes_serve_create": (C.c_int, [PP(wipes_serve_config), PP(wipes_params), C.c_int32, PP(C.c_void_p)]),
        "wipes_serve_load_scene": (C.c_int, [P, PP(wipes_prims), PP(C.c_int32)]),
        "wipes_serve_unload_scene": (C.c_int, [P, C.c_int32]),
        "wipes_serve_submit": (C.c_int, [P, C.c_int32, PP(wipes_camera), P, C.c_size_t, P, PP(C.c_uint64)]),
        "wipes_serve_poll": (C.c_int, [P, C.c_uint64, PP(C.c_int32), D]),
        "wipes_serve_drain": (C.c_int, [P]),
        "wipes_serve_stats": (C.c_int, [P, PP(wipes_serve_report)]),
        "wipes_serve_reset_stats": (C.c_int, [P]),
        "wipes_serve_destroy": (None, [P]),
        "wipes_serve_simulate": (C.c_int, [PP(wipes_serve_config), C.c_int64, D, I64, D, D, D, D, I64, I64]),
        "wipes_l2_grad": (C.c_int, [P, PP(wipes_params), PP(wipes_batch), PP(wipes_buffer), P, P, P, P]),
        "wipes_graph_capture": (C.c_int, [P, PP(wipes_params), PP(wipes_batch), PP(wipes_buffer), PP(wipes_buffer),
                                          P, P, P, P, P, C.c_int32, PP(C.c_void_p)]),
        "wipes_graph_launch": (C.c_int, [P, P]),
        "wipes_graph_destroy": (None, [P]),
        "wipes_adam": (C.c_int, [P, C.c_int32, PP(wipes_adam_group), C.c_double, C.c_double, C.c_double, P,
                                 PP(wipes_params), PP(wipes_batch), PP(wipes_buffer), P]),
    }
    for name, (res, args) in table.items():
        if hasattr(L, name):
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
