"""Deformation network of Eq. 8 (Sec. 4.3) on top of the C ABI: the offsets
(dx, df, dq, ds) of every primitive of a dynamic scene at time t, with a
torch.autograd.Function whose backward returns the gradients of the network's
parameters and of the primitives' positions.

PyTorch provides the device memory (the workspace is a uint8 tensor) and the
current stream; the encoding, the layers and their gradients run in
libwipes.so.
"""
from __future__ import annotations

import torch

from . import binding as B

N_OUT = 13


def param_count() -> int:
    return B.wipes_deform_param_count()


_APPLY_KEYS = ("mean", "freq", "quat", "scale")


def apply_offsets(net: "Deformation", prims: dict, offsets: torch.Tensor) -> dict:
    """Deformed primitive set (wipes_deform_apply): mean + dx, freq + df, quat + dq, scale + ds; the other keys
    are passed through.  Differentiable: the gradients of the deformed values flow to the offsets and to the
    original values unchanged."""
    out = dict(prims)
    vals = _ApplyFn.apply(net, offsets, *[prims[k] for k in _APPLY_KEYS])
    for k, v in zip(_APPLY_KEYS, vals):
        out[k] = v
    return out


class _ApplyFn(torch.autograd.Function):
    @staticmethod
    def forward(ctx, net, offsets, mean, freq, quat, scale):
        ins = [t.detach().to(torch.float32).contiguous() for t in (offsets, mean, freq, quat, scale)]
        n = ins[1].shape[0]
        if ins[0].shape != (n, N_OUT):
            raise ValueError("offsets must be [n, 13]")
        outs = [torch.empty_like(t) for t in ins[1:]]
        B.wipes_deform_apply(net.ctx, n, *[t.data_ptr() for t in ins], *[t.data_ptr() for t in outs],
                             torch.cuda.current_stream(net.device).cuda_stream)
        return tuple(outs)

    @staticmethod
    def backward(ctx, gm, gf, gq, gs):
        # the identity: the offsets' gradient is the four gradients side by side
        parts = [g if g is not None else torch.zeros(0) for g in (gm, gf, gq, gs)]
        n = next(g.shape[0] for g in parts if g.numel())
        widths = (3, 3, 4, 3)
        dev = next(g.device for g in parts if g.numel())
        cols = [g if g.numel() else torch.zeros((n, w), device=dev) for g, w in zip(parts, widths)]
        return (None, torch.cat(cols, dim=1), gm, gf, gq, gs)


class Deformation:
    """Holds one context and a workspace sized for the largest primitive count seen."""

    def __init__(self, device=None, precision: int = B.WIPES_DEFORM_BF16X3):
        self.device = torch.device("cuda", torch.cuda.current_device()) if device is None else torch.device(device)
        self.precision = precision
        self.ctx = B.wipes_ctx_create(self.device.index or 0)
        self._ws = None

    def close(self):
        if self.ctx is not None:
            B.wipes_ctx_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _workspace(self, n: int, with_backward: bool) -> torch.Tensor:
        need = B.wipes_deform_workspace_size(n, with_backward)
        if self._ws is None or self._ws.numel() < need:
            self._ws = torch.empty(need, dtype=torch.uint8, device=self.device)
        return self._ws

    def new_workspace(self, n: int) -> torch.Tensor:
        """A workspace of its own for one forward/backward pair."""
        return torch.empty(B.wipes_deform_workspace_size(n, True), dtype=torch.uint8, device=self.device)

    def _check(self, params, mean):
        for name, t in (("params", params), ("mean", mean)):
            if t.dtype != torch.float32 or not t.is_contiguous() or t.device != self.device:
                raise ValueError("%s must be a contiguous float32 tensor on %s" % (name, self.device))
        if params.numel() != param_count():
            raise ValueError("params must hold %d values" % param_count())
        if mean.dim() != 2 or mean.shape[1] != 3:
            raise ValueError("mean must be [n, 3]")

    def forward(self, params: torch.Tensor, mean: torch.Tensor, time: float, keep_for_backward: bool = False,
                workspace: torch.Tensor | None = None):
        """Offsets [n, 13].  With keep_for_backward the workspace (the shared one unless given) holds the
        layer inputs until the matching backward call."""
        self._check(params, mean)
        n = mean.shape[0]
        out = torch.empty((n, N_OUT), dtype=torch.float32, device=self.device)
        ws = self._workspace(n, keep_for_backward) if workspace is None else workspace
        B.wipes_deform_fwd(self.ctx, self.precision, params.data_ptr(), n, mean.data_ptr(), float(time),
                           out.data_ptr(), ws.data_ptr(), ws.numel(), keep_for_backward,
                           torch.cuda.current_stream(self.device).cuda_stream)
        return out

    def backward(self, params: torch.Tensor, mean: torch.Tensor, time: float, d_offsets: torch.Tensor,
                 workspace: torch.Tensor | None = None):
        """Gradients after a forward(..., keep_for_backward=True) on the same inputs and workspace:
        (d_params, d_mean)."""
        self._check(params, mean)
        n = mean.shape[0]
        d_offsets = d_offsets.to(torch.float32).contiguous()
        if d_offsets.shape != (n, N_OUT):
            raise ValueError("d_offsets must be [n, 13]")
        ws = self._workspace(n, True) if workspace is None else workspace
        dp = torch.empty_like(params)
        dm = torch.empty_like(mean)
        B.wipes_deform_bwd(self.ctx, self.precision, params.data_ptr(), n, mean.data_ptr(), float(time),
                           d_offsets.data_ptr(), ws.data_ptr(), ws.numel(), dp.data_ptr(), dm.data_ptr(),
                           torch.cuda.current_stream(self.device).cuda_stream)
        return dp, dm

    def __call__(self, params: torch.Tensor, mean: torch.Tensor, time: float) -> torch.Tensor:
        """Differentiable offsets [n, 13] (gradients reach params and mean)."""
        return _DeformFn.apply(self, params, mean, float(time))


class _DeformFn(torch.autograd.Function):
    @staticmethod
    def forward(ctx, net: Deformation, params, mean, time):
        ctx.net, ctx.time = net, time
        ctx.ws = net.new_workspace(mean.shape[0])
        ctx.save_for_backward(params, mean)
        return net.forward(params.detach().contiguous(), mean.detach().contiguous(), time, keep_for_backward=True,
                           workspace=ctx.ws)

    @staticmethod
    def backward(ctx, d_off):
        params, mean = ctx.saved_tensors
        dp, dm = ctx.net.backward(params.detach().contiguous(), mean.detach().contiguous(), ctx.time, d_off,
                                  workspace=ctx.ws)
        ctx.ws = None
        return None, dp, dm, None
