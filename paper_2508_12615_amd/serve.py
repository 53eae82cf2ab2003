"""Python client of the serving C ABI (wipes_serve_*): resident 3D scenes,
non-blocking render requests, continuous batching inside the library.

Also holds the plain-rasterizer reference loop used to compare against: one
request at a time, B = 1, grid launch, synchronous.
"""
from __future__ import annotations

import ctypes as C
import time

import numpy as np
import torch

from . import binding as B
from .binding_ext import wipes_serve_config, wipes_serve_report
from .raster import Rasterizer, make_camera

SCENE_KEYS = ("mean", "quat", "scale", "freq", "color", "opacity", "velocity", "phase", "sh")


def simulate(cfg: dict, t_arrive, footprint, prep_s, blend_s):
    """Host-only scheduler model (fake executor).  Returns dict of numpy arrays."""
    n = len(t_arrive)
    c = wipes_serve_config(int(cfg["max_slots"]), int(cfg["max_pending"]), int(cfg["max_batch"]),
                           int(cfg.get("persistent", 3)), int(cfg["hbm_budget_bytes"]))
    ta = np.ascontiguousarray(t_arrive, np.float64)
    fp = np.ascontiguousarray(footprint, np.int64)
    ps = np.ascontiguousarray(prep_s, np.float64)
    bs = np.ascontiguousarray(blend_s, np.float64)
    adm = np.zeros(n); done = np.zeros(n); bat = np.zeros(n, np.int64); peak = C.c_int64()
    P = lambda a: a.ctypes.data_as(C.c_void_p)  # noqa: E731
    st = B.lib().wipes_serve_simulate(C.byref(c), n, C.cast(P(ta), C.POINTER(C.c_double)),
                                      C.cast(P(fp), C.POINTER(C.c_int64)), C.cast(P(ps), C.POINTER(C.c_double)),
                                      C.cast(P(bs), C.POINTER(C.c_double)), C.cast(P(adm), C.POINTER(C.c_double)),
                                      C.cast(P(done), C.POINTER(C.c_double)), C.cast(P(bat), C.POINTER(C.c_int64)),
                                      C.byref(peak))
    B.check(st)
    return dict(t_admit=adm, t_done=done, batch=bat, arena_peak=peak.value)


class Server:
    """A wipes_server: load scenes, submit cameras, poll or drain, read stats."""

    def __init__(self, device: int = 0, max_slots: int = 16, max_pending: int = 4096, max_batch: int = 8,
                 persistent: int = 3, hbm_budget_bytes: int = 4 << 30, **overrides):
        self.params = B.wipes_params_default(B.WIPES_3D_ALPHA)
        for k, v in overrides.items():
            if k == "bg":
                for i in range(3):
                    self.params.bg[i] = float(v[i])
            else:
                setattr(self.params, k, v)
        cfg = wipes_serve_config(max_slots, max_pending, max_batch, persistent, int(hbm_budget_bytes))
        h = C.c_void_p()
        B.check(B.lib().wipes_serve_create(C.byref(cfg), C.byref(self.params), device, C.byref(h)))
        self.h = h
        self.device = torch.device("cuda", device)

    def load_scene(self, prims: dict) -> int:
        p = B.wipes_prims()
        p.n = int(prims["opacity"].shape[0])
        for k in SCENE_KEYS:
            t = prims.get(k)
            setattr(p, k, None if t is None else t.data_ptr())
        sid = C.c_int32()
        B.check(B.lib().wipes_serve_load_scene(self.h, C.byref(p), C.byref(sid)))
        return sid.value

    def unload_scene(self, sid: int) -> int:
        return B.check(B.lib().wipes_serve_unload_scene(self.h, sid), allow=(B.WIPES_ERR_BUSY,))

    def submit(self, sid: int, camera: dict, out: torch.Tensor) -> int:
        """Queue a render of scene `sid` from `camera` into `out`, a contiguous
        float32 device tensor of height * width * 3 elements.  The library checks
        the element count and writes `out` only after the work already queued on
        the current stream (e.g. a fill of `out`)."""
        if out.dtype != torch.float32 or not out.is_cuda or not out.is_contiguous():
            raise ValueError("out must be a contiguous float32 CUDA tensor, got %s %s" % (tuple(out.shape), out.dtype))
        rid = C.c_uint64()
        stream = torch.cuda.current_stream(out.device).cuda_stream
        B.check(B.lib().wipes_serve_submit(self.h, sid, C.byref(make_camera(camera)), out.data_ptr(), out.numel(),
                                           stream, C.byref(rid)))
        return rid.value

    def poll(self, rid: int):
        done, lat = C.c_int32(), C.c_double()
        B.check(B.lib().wipes_serve_poll(self.h, rid, C.byref(done), C.byref(lat)))
        return bool(done.value), lat.value

    def drain(self) -> None:
        B.check(B.lib().wipes_serve_drain(self.h))

    def stats(self) -> dict:
        r = wipes_serve_report()
        B.check(B.lib().wipes_serve_stats(self.h, C.byref(r)))
        return {f: getattr(r, f) for f, _ in r._fields_}

    def reset_stats(self) -> None:
        B.check(B.lib().wipes_serve_reset_stats(self.h))

    def close(self) -> None:
        if self.h:
            B.lib().wipes_serve_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def run_plain(rast: Rasterizer, scenes: list, requests: list, outs: list):
    """Plain rasterizer: requests served one at a time in arrival order (B = 1,
    synchronous).  Returns latencies (ms, arrival -> completion) and makespan."""
    t0 = time.perf_counter()
    lat = []
    for req, out in zip(requests, outs):
        now = time.perf_counter() - t0
        if req["t_arrive"] > now:
            time.sleep(req["t_arrive"] - now)
        f = rast.forward([dict(camera=req["camera"], prims=scenes[req["scene"]])])
        out.copy_(f.image.view_as(out))
        torch.cuda.synchronize()
        lat.append((time.perf_counter() - t0 - req["t_arrive"]) * 1e3)
    return np.array(lat), time.perf_counter() - t0


def run_served(server: Server, scene_ids: list, requests: list, outs: list):
    """Submit requests at their arrival times (client thread = caller), then drain.
    Returns latencies (ms, scheduled arrival -> completion, like run_plain: the
    server's submit -> completion time plus the client's delay from the
    scheduled arrival to the submit call) and the makespan."""
    t0 = time.perf_counter()
    ids, late = [], []
    for req, out in zip(requests, outs):
        now = time.perf_counter() - t0
        if req["t_arrive"] > now:
            time.sleep(req["t_arrive"] - now)
        late.append((time.perf_counter() - t0 - req["t_arrive"]) * 1e3)
        ids.append(server.submit(scene_ids[req["scene"]], req["camera"], out))
    server.drain()
    lat = [server.poll(i)[1] + d for i, d in zip(ids, late)]
    return np.array(lat), time.perf_counter() - t0
