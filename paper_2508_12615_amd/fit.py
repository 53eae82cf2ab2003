"""2D image fitting with wavelet primitives (Sec. 5.1): L2 loss, Adam.

Two drivers over the same rasterizer:

* ``fit_plain``    -- one image, one step = render (autograd) -> L2 loss ->
                      backward -> Adam; the plain per-image rasterizer with one
                      host synchronisation per step (instance count readback).
* ``fit_graph``    -- one image, one step = one hipGraph replay of the whole
                      render step + the library's Adam (a BatchedFit of one
                      image), with no host synchronisation per step.
* ``BatchedFit``   -- many images of uneven size fitted together; one step is a
                      single replay of a hipGraph holding projection, binning,
                      sorting, forward blend, L2 gradient, backward blend and
                      projection backward for every image, followed by one
                      Adam launch (``wipes_adam``) over the concatenated
                      parameters, skipped on the device if the replay
                      overflowed the instance capacity.

Optimiser settings (a reading; the paper keeps GaussianImage's values, which
it does not list): Adam(beta = (0.9, 0.999), eps = 1e-8), learning rate 1e-3
for means, covariance factors, colours and opacities, 2.5e-3 for the
frequencies (the frequency learning rate the paper states for its 3D runs).
"""
from __future__ import annotations

import ctypes as C
import math
import time

import numpy as np
import torch

from . import binding as B
from .raster import Rasterizer, make_camera, render

LR_DEFAULT = 1e-3
LR_FREQ = 2.5e-3
KEYS_2D = ("mean", "cov", "freq", "color", "opacity")


def _adam(params: dict, lr: float = LR_DEFAULT, lr_freq: float = LR_FREQ):
    groups = [dict(params=[params[k]], lr=(lr_freq if k == "freq" else lr)) for k in KEYS_2D if k in params]
    return torch.optim.Adam(groups, betas=(0.9, 0.999), eps=1e-8)


def psnr(img: torch.Tensor, target: torch.Tensor) -> float:
    mse = float(((img - target) ** 2).mean())
    return 10.0 * math.log10(1.0 / max(mse, 1e-20))


def fit_graph(prims: dict, target: torch.Tensor, steps: int, tile=(16, 16), cov: int = B.WIPES_COV_RS,
              log_every: int = 0):
    """Fit one image with one hipGraph replay per step (projection, binning,
    sorting, forward, L2 gradient, backward, projection backward), then Adam.
    The instance count is checked after every replay, before the optimiser
    step; a replay that overflowed the capacity is redone after recapturing
    with more room, so no step uses gradients of a truncated render.
    prims is modified in place.  Returns dict(history, psnr, seconds, steps,
    recaptures)."""
    H, W, _ = target.shape
    fit = BatchedFit([dict(width=W, height=H, target=target.contiguous(), prims=prims)], tile=tile, cov=cov)
    hist = []
    grown = 0
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    it = 0   # steps applied
    while it < steps:
        # launch up to 32 steps without waiting; a replay that overflows makes
        # its Adam step (and every later one, whose inputs are then the same)
        # a no-op on the device, which the step counter shows afterwards
        chunk = min(32, steps - it)
        for j in range(chunk):
            fit.step()
            if log_every and ((it + j) % log_every == 0 or it + j == steps - 1):
                hist.append((it + j, fit.loss()))
        done = fit.steps_applied()
        if done < it + chunk:
            st, K = B.wipes_check_overflow(fit.rast.ctx, fit.rast.params, fit.batch, fit.sbuf,
                                           torch.cuda.current_stream(fit.device).cuda_stream)
            fit.grow(K)
            grown += 1
            hist = [h for h in hist if h[0] < done]   # losses of skipped steps are redone
        it = done
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    with torch.no_grad():
        for k in KEYS_2D:
            prims[k].copy_(fit.params[k])
    fit.render_grads()
    torch.cuda.synchronize()
    final = psnr(fit.image.view(H, W, 3), target)
    fit.close()
    return dict(history=hist, psnr=final, seconds=dt, steps=steps, recaptures=grown)


def fit_plain(prims: dict, target: torch.Tensor, steps: int, rast: Rasterizer | None = None, cov: int = B.WIPES_COV_RS,
              log_every: int = 0):
    """Fit one image.  prims: dict of float32 CUDA tensors (modified in place).
    Returns dict(loss history, final psnr, seconds)."""
    H, W, _ = target.shape
    rast = rast or Rasterizer(B.WIPES_2D_ADDITIVE, device=target.device, cov=cov)
    params = {k: prims[k].detach().clone().requires_grad_(True) for k in KEYS_2D}
    opt = _adam(params)
    hist = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for it in range(steps):
        img = render(rast, (W, H), **params)
        loss = ((img - target) ** 2).mean()
        opt.zero_grad(set_to_none=False)
        loss.backward()
        opt.step()
        if log_every and (it % log_every == 0 or it == steps - 1):
            hist.append((it, float(loss.detach())))
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    with torch.no_grad():
        for k in KEYS_2D:
            prims[k].copy_(params[k])
        final = render(rast, (W, H), **{k: params[k].detach() for k in KEYS_2D})
    return dict(history=hist, psnr=psnr(final, target), seconds=dt, steps=steps)


class BatchedFit:
    """Fit many 2D images of different sizes at once, one graph replay per step.

    images: list of dict(width, height, target [H,W,3] float32 CUDA tensor,
    prims dict of float32 CUDA tensors).  The primitives of all images are
    copied into one tensor per attribute; image b owns rows
    [offset_b, offset_b + n_b).
    """

    def __init__(self, images, device=None, tile=(16, 16), persistent=3, cov: int = B.WIPES_COV_RS,
                 capacity_margin: float = 1.3):
        self.device = torch.device(device) if device is not None else images[0]["target"].device
        self.rast = Rasterizer(B.WIPES_2D_ADDITIVE, device=self.device, cov=cov, tile_w=tile[0], tile_h=tile[1],
                               persistent=persistent)
        self.sizes = [(int(im["width"]), int(im["height"])) for im in images]
        self.counts = [int(im["prims"]["opacity"].shape[0]) for im in images]
        self.offsets = np.concatenate([[0], np.cumsum(self.counts)]).astype(np.int64)
        self.params = {k: torch.cat([im["prims"][k] for im in images]).contiguous().requires_grad_(True)
                       for k in KEYS_2D}
        for k in KEYS_2D:
            self.params[k].grad = torch.zeros_like(self.params[k])
        self.target = torch.cat([im["target"].reshape(-1, 3) for im in images]).contiguous()
        npx = self.target.shape[0]
        self.image = torch.empty((npx, 3), dtype=torch.float32, device=self.device)
        self.dL = torch.empty((npx, 3), dtype=torch.float32, device=self.device)
        # state of the library's Adam (one launch per step for all groups)
        self.adam_m = {k: torch.zeros_like(self.params[k]) for k in KEYS_2D}
        self.adam_v = {k: torch.zeros_like(self.params[k]) for k in KEYS_2D}
        self.adam_lr = {k: (LR_FREQ if k == "freq" else LR_DEFAULT) for k in KEYS_2D}
        self.adam_step = torch.zeros(1, dtype=torch.int32, device=self.device)
        self._views = self._image_views()
        # size the instance capacity from one plain pass
        f = self.rast.forward(self._views)
        self.K0 = f.K
        self.capacity_margin = capacity_margin
        self.batch, self._keep, _ = self.rast.make_batch(self._views, self._grad_views())
        self.graph = None
        self._capture(int(f.K * capacity_margin) + 4096)

    def _capture(self, capacity: int) -> None:
        """(Re)build the workspace for `capacity` instances and capture the step."""
        self.close()
        self.capacity = int(capacity)
        sb, bb = B.wipes_workspace_size(self.rast.params, self.batch, self.capacity, True)
        self.screen = torch.empty(sb, dtype=torch.uint8, device=self.device)
        self.bins = torch.empty(bb, dtype=torch.uint8, device=self.device)
        self.sbuf = B.wipes_buffer(self.screen.data_ptr(), sb, 0, 0, 0)
        self.bbuf = B.wipes_buffer(self.bins.data_ptr(), bb, self.capacity, 1, 0)
        self.graph = B.wipes_graph_capture(self.rast.ctx, self.rast.params, self.batch, self.sbuf, self.bbuf,
                                           self.image.data_ptr(), None, None, self.target.data_ptr(),
                                           self.dL.data_ptr(), True)

    def grow(self, needed: int) -> None:
        """Recapture with room for `needed` instances (parameters and optimiser state are kept)."""
        self._capture(int(needed * self.capacity_margin) + 4096)

    def _image_views(self):
        out = []
        for b, (W, H) in enumerate(self.sizes):
            a, z = int(self.offsets[b]), int(self.offsets[b + 1])
            out.append(dict(camera=(W, H), prims={k: self.params[k].detach()[a:z] for k in KEYS_2D}))
        return out

    def _grad_views(self):
        out = []
        for b in range(len(self.sizes)):
            a, z = int(self.offsets[b]), int(self.offsets[b + 1])
            out.append({k: self.params[k].grad[a:z] for k in KEYS_2D})
        return out

    def render_grads(self) -> None:
        """One replay: image, dL/dimage and parameter gradients (no optimiser step)."""
        B.wipes_graph_launch(self.graph, torch.cuda.current_stream(self.device).cuda_stream)

    def step(self) -> None:
        """One replay and one Adam step (skipped on the device if the replay overflowed)."""
        self.render_grads()
        self.adam()

    def adam(self) -> None:
        groups = [(self.params[k].detach(), self.params[k].grad, self.adam_m[k], self.adam_v[k], self.adam_lr[k])
                  for k in KEYS_2D]
        B.wipes_adam(self.rast.ctx, groups, 0.9, 0.999, 1e-8, self.adam_step.data_ptr(), self.rast.params,
                     self.batch, self.sbuf, torch.cuda.current_stream(self.device).cuda_stream)

    def steps_applied(self) -> int:
        """Adam steps applied so far (synchronises)."""
        return int(self.adam_step.item())

    def check_capacity(self) -> int:
        """Synchronises; raises if the last replay overflowed the instance capacity."""
        st, K = B.wipes_check_overflow(self.rast.ctx, self.rast.params, self.batch, self.sbuf,
                                       torch.cuda.current_stream(self.device).cuda_stream)
        if st != B.WIPES_OK:
            raise B.WipesError(st, "instance capacity %d exceeded (%d needed)" % (self.capacity, K))
        return K

    def loss(self) -> float:
        """Mean over images of each image's L2 loss (from the last replay's image)."""
        tot, o = 0.0, 0
        for (W, H) in self.sizes:
            n = W * H
            tot += float(((self.image[o:o + n] - self.target[o:o + n]) ** 2).mean())
            o += n
        return tot / len(self.sizes)

    def close(self):
        if getattr(self, "graph", None):
            B.wipes_graph_destroy(self.graph)
            self.graph = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
