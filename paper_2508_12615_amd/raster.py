"""High-level rasterizer on top of the C ABI: workspace management, plain
forward/backward, and torch.autograd integration.

PyTorch provides device memory (workspaces are uint8 tensors from torch's
caching allocator, so steady-state calls do not reach hipMalloc) and the
current HIP stream.  All arithmetic runs in libwipes.so.
"""
from __future__ import annotations

import ctypes as C
from dataclasses import dataclass, field

import numpy as np
import torch

from . import binding as B

_PRIM_KEYS = ("mean", "cov", "quat", "scale", "freq", "color", "opacity", "velocity", "phase", "sh")


def _ptr(t):
    return None if t is None else t.data_ptr()


def _check_tensor(name, t, device):
    if t is None:
        return None
    if not isinstance(t, torch.Tensor):
        raise TypeError("%s must be a torch.Tensor" % name)
    if t.dtype != torch.float32 or not t.is_contiguous() or t.device != device:
        raise ValueError("%s must be a contiguous float32 tensor on %s" % (name, device))
    return t


def make_camera(cam) -> B.wipes_camera:
    """cam: dict(width, height, fx, fy, cx, cy, viewmat (4x4), time) or (width, height) for 2D."""
    c = B.wipes_camera()
    if isinstance(cam, (tuple, list)):
        c.width, c.height = int(cam[0]), int(cam[1])
        for k in range(16):
            c.viewmat[k] = 1.0 if k % 5 == 0 else 0.0
        return c
    c.width, c.height = int(cam["width"]), int(cam["height"])
    c.fx, c.fy, c.cx, c.cy = (float(cam.get(k, 0.0)) for k in ("fx", "fy", "cx", "cy"))
    vm = np.asarray(cam.get("viewmat", np.eye(4)), dtype=np.float32).reshape(16)
    for k in range(16):
        c.viewmat[k] = float(vm[k])
    c.time = float(np.float32(cam.get("time", 0.0)))
    return c


@dataclass
class Frame:
    """Outputs of a forward pass plus the workspaces the backward needs."""
    image: torch.Tensor           # [sum H W, 3]
    T_final: torch.Tensor | None  # [sum H W]
    last: torch.Tensor | None     # [sum H W] int32
    K: int
    screen: torch.Tensor
    bins: torch.Tensor
    cap: int
    with_backward: bool
    sizes: list = field(default_factory=list)

    def images(self):
        out, o = [], 0
        for (w, h) in self.sizes:
            out.append(self.image[o:o + w * h].view(h, w, 3))
            o += w * h
        return out


class Rasterizer:
    """Wavelet rasterizer bound to one device.

    mode: B.WIPES_2D_ADDITIVE or B.WIPES_3D_ALPHA.  Keyword arguments override
    the documented constants (tile_w, tile_h, persistent, alpha_min, ...).
    """

    def __init__(self, mode: int, device=None, **overrides):
        self.device = torch.device(device) if device is not None else torch.device("cuda", torch.cuda.current_device())
        if self.device.type != "cuda":
            raise ValueError("the wavelet rasterizer runs on a HIP device only")
        self.ctx = B.wipes_ctx_create(self.device.index if self.device.index is not None else 0)
        self.params = B.wipes_params_default(mode)
        for k, v in overrides.items():
            if k == "bg":
                for i in range(3):
                    self.params.bg[i] = float(v[i])
            elif hasattr(self.params, k):
                setattr(self.params, k, v)
            else:
                raise KeyError(k)
        self.cap_hint = 0

    @property
    def mode(self) -> int:
        return self.params.mode

    def __del__(self):
        try:
            if getattr(self, "ctx", None):
                B.wipes_ctx_destroy(self.ctx)
                self.ctx = None
        except Exception:
            pass

    # -------------------------------------------------------------- batches
    def make_batch(self, images, grads=None):
        """images: list of dict(camera=..., prims=dict of tensors); grads: list of dicts or None."""
        n = len(images)
        arr = (B.wipes_image * n)()
        keep = []
        sizes = []
        for i, im in enumerate(images):
            cam = make_camera(im["camera"])
            arr[i].cam = cam
            sizes.append((cam.width, cam.height))
            pr = im["prims"]
            cnt = int(pr["opacity"].shape[0])
            arr[i].prims.n = cnt
            for k in _PRIM_KEYS:
                t = _check_tensor(k, pr.get(k), self.device)
                setattr(arr[i].prims, k, _ptr(t))
                keep.append(t)
            if grads is not None and grads[i] is not None:
                for k in _PRIM_KEYS:
                    t = _check_tensor("grad " + k, grads[i].get(k), self.device)
                    setattr(arr[i].grads, k, _ptr(t))
                    keep.append(t)
        batch = B.wipes_batch(n, C.cast(arr, C.POINTER(B.wipes_image)))
        keep.append(arr)
        return batch, keep, sizes

    # -------------------------------------------------------------- passes
    def _stream(self) -> int:
        return torch.cuda.current_stream(self.device).cuda_stream

    def forward(self, images, with_backward: bool = False) -> Frame:
        batch, keep, sizes = self.make_batch(images)
        stream = self._stream()
        sb, _ = B.wipes_workspace_size(self.params, batch, 0, False)
        screen = torch.empty(max(sb, 256), dtype=torch.uint8, device=self.device)
        sbuf = B.wipes_buffer(screen.data_ptr(), screen.numel(), 0, 0, 0)
        B.wipes_project(self.ctx, self.params, batch, sbuf, stream)
        n_total = sum(int(im["prims"]["opacity"].shape[0]) for im in images)
        cap = max(self.cap_hint, 4096, 4 * n_total)
        while True:
            _, bb = B.wipes_workspace_size(self.params, batch, cap, with_backward)
            bins = torch.empty(max(bb, 256), dtype=torch.uint8, device=self.device)
            bbuf = B.wipes_buffer(bins.data_ptr(), bins.numel(), cap, int(with_backward), 0)
            st, K = B.wipes_bin_sort(self.ctx, self.params, batch, sbuf, bbuf, stream)
            if st == B.WIPES_OK:
                break
            cap = int(K * 1.25) + 4096
        self.cap_hint = max(self.cap_hint, int(K * 1.25) + 4096)
        npx = sum(w * h for (w, h) in sizes)
        image = torch.empty((npx, 3), dtype=torch.float32, device=self.device)
        alpha = self.params.mode == B.WIPES_3D_ALPHA
        T = torch.empty(npx, dtype=torch.float32, device=self.device) if alpha else None
        last = torch.empty(npx, dtype=torch.int32, device=self.device) if alpha else None
        B.wipes_render_fwd(self.ctx, self.params, batch, sbuf, bbuf, image.data_ptr(), _ptr(T), _ptr(last), stream)
        return Frame(image, T, last, K, screen, bins, cap, with_backward, sizes)

    def backward(self, images, frame: Frame, dL_dimage: torch.Tensor, grads=None, want_dscreen: bool = False):
        """Parameter gradients (list of dicts, one per image) for dL/dimage [sum H W, 3]."""
        if not frame.with_backward:
            raise ValueError("forward(..., with_backward=True) is required before backward")
        if grads is None:
            grads = []
            for im in images:
                g = {}
                for k in _PRIM_KEYS:
                    t = im["prims"].get(k)
                    if t is not None:
                        g[k] = torch.empty_like(t)
                grads.append(g)
        batch, keep, _ = self.make_batch(images, grads)
        dL = dL_dimage.reshape(-1, 3).contiguous()
        if dL.dtype != torch.float32:
            dL = dL.float()
        sbuf = B.wipes_buffer(frame.screen.data_ptr(), frame.screen.numel(), 0, 0, 0)
        bbuf = B.wipes_buffer(frame.bins.data_ptr(), frame.bins.numel(), frame.cap, 1, 0)
        n_total = sum(int(im["prims"]["opacity"].shape[0]) for im in images)
        dscreen = torch.empty((n_total, 12), dtype=torch.float32, device=self.device) if want_dscreen else None
        B.wipes_render_bwd(self.ctx, self.params, batch, sbuf, bbuf, _ptr(frame.T_final), _ptr(frame.last),
                           dL.data_ptr(), _ptr(dscreen), self._stream())
        return (grads, dscreen) if want_dscreen else grads

    def stats(self, images, frame: Frame):
        """Work counts of a rendered frame (see wipes_render_stats); synchronises."""
        batch, keep, _ = self.make_batch(images)
        sbuf = B.wipes_buffer(frame.screen.data_ptr(), frame.screen.numel(), 0, 0, 0)
        bbuf = B.wipes_buffer(frame.bins.data_ptr(), frame.bins.numel(), frame.cap, int(frame.with_backward), 0)
        return B.wipes_render_stats(self.ctx, self.params, batch, sbuf, bbuf, _ptr(frame.T_final), _ptr(frame.last),
                                    self._stream())

    def bins(self, images, frame: Frame):
        """Sorted tile keys, primitive indices [K] and ranges [n_tiles, 2] as int64 CPU arrays (syncs)."""
        batch, keep, _ = self.make_batch(images)
        sbuf = B.wipes_buffer(frame.screen.data_ptr(), frame.screen.numel(), 0, 0, 0)
        bbuf = B.wipes_buffer(frame.bins.data_ptr(), frame.bins.numel(), frame.cap, int(frame.with_backward), 0)
        kp, vp, rp, nt = B.wipes_bins_view(self.params, batch, sbuf, bbuf)
        base = frame.bins.data_ptr()
        def view(ptr, count):
            off = ptr - base
            return frame.bins[off:off + 4 * count].view(torch.int32).cpu().numpy().view(np.uint32)
        torch.cuda.synchronize(self.device)
        return view(kp, frame.K), view(vp, frame.K), view(rp, 2 * nt).reshape(nt, 2)


# ------------------------------------------------------------------ autotuning

def autotune_candidates():
    n = B.lib().wipes_autotune_candidates(None, None, None, 0)
    tw, th, pe = (C.c_int32 * n)(), (C.c_int32 * n)(), (C.c_int32 * n)()
    B.lib().wipes_autotune_candidates(tw, th, pe, n)
    return [(tw[i], th[i], pe[i]) for i in range(n)]


def workload_signature(rast: Rasterizer, images, with_backward: bool) -> str:
    """Key of the autotune cache: mode, image sizes and primitive counts (rounded to 2 significant digits)."""
    def r2(x):
        return 0 if x == 0 else int(float("%.2g" % x))
    parts = ["m%d" % rast.params.mode, "b%d" % int(with_backward)]
    for im in images:
        cam = make_camera(im["camera"])
        parts.append("%dx%d:%d" % (cam.width, cam.height, r2(int(im["prims"]["opacity"].shape[0]))))
    return "|".join(parts)


def autotune(rast: Rasterizer, images, with_backward: bool = True, reps: int = 3, cache_path: str | None = None):
    """Time every tile shape / launch form on this workload (wipes_autotune), set the fastest
    on `rast` and return {(tw, th, persistent): ms}.  Results are cached as JSON at cache_path."""
    import json
    import os
    key = workload_signature(rast, images, with_backward)
    if cache_path and os.path.exists(cache_path):
        with open(cache_path) as fh:
            cache = json.load(fh)
        if key in cache:
            tw, th, pe = cache[key]["best"]
            rast.params.tile_w, rast.params.tile_h, rast.params.persistent = tw, th, pe
            return {tuple(map(int, k.split(","))): v for k, v in cache[key]["times"].items()}
    cands = autotune_candidates()
    batch, keep, _ = rast.make_batch(images)
    best = B.wipes_params()
    times = (C.c_double * len(cands))()
    B.check(B.lib().wipes_autotune(rast.ctx, C.byref(rast.params), C.byref(batch), int(bool(with_backward)), reps,
                                   C.byref(best), times, rast._stream()), rast.ctx)
    rast.params.tile_w, rast.params.tile_h, rast.params.persistent = best.tile_w, best.tile_h, best.persistent
    out = {c: times[i] for i, c in enumerate(cands)}
    if cache_path:
        cache = {}
        if os.path.exists(cache_path):
            with open(cache_path) as fh:
                cache = json.load(fh)
        cache[key] = dict(best=[best.tile_w, best.tile_h, best.persistent],
                          times={"%d,%d,%d" % c: t for c, t in out.items()})
        with open(cache_path, "w") as fh:
            json.dump(cache, fh, indent=1)
    return out


# ------------------------------------------------------------------ autograd

class _RenderFn(torch.autograd.Function):
    """Differentiable render of one image.  Saves the workspaces (screen
    records, sorted lists, T_final, last); the backward recomputes every
    per-pair quantity, nothing per pair is stored."""

    @staticmethod
    def forward(ctx, rast, camera, keys, *tensors):
        prims = {k: t for k, t in zip(keys, tensors)}
        frame = rast.forward([dict(camera=camera, prims=prims)], with_backward=True)
        ctx.rast, ctx.camera, ctx.keys, ctx.frame = rast, camera, keys, frame
        ctx.save_for_backward(*tensors)
        w, h = frame.sizes[0]
        return frame.image.view(h, w, 3)

    @staticmethod
    def backward(ctx, g):
        tensors = ctx.saved_tensors
        prims = {k: t for k, t in zip(ctx.keys, tensors)}
        grads = ctx.rast.backward([dict(camera=ctx.camera, prims=prims)], ctx.frame, g.contiguous())[0]
        ctx.frame = None
        return (None, None, None) + tuple(grads[k] if ctx.needs_input_grad[3 + i] else None
                                          for i, k in enumerate(ctx.keys))


def render(rast: Rasterizer, camera, **prims) -> torch.Tensor:
    """Differentiable image [H, W, 3] of one set of primitives (torch tensors)."""
    keys = tuple(k for k in _PRIM_KEYS if prims.get(k) is not None)
    return _RenderFn.apply(rast, camera, keys, *[prims[k].contiguous() for k in keys])
