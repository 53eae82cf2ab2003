"""The allocation-free forward frame (wipes_render_fwd_noalloc, for callers
that cannot allocate device memory) against the caller-buffer path
(wipes_project + wipes_bin_sort + wipes_render_fwd) through the C ABI: the
same kernels on the same inputs, so the images, final transmittance and
`last` must agree bit for bit.  Two calls in a row, the second smaller (the
static workspace keeps the first call's contents), in both blend modes, plus
the host-side rejection of a batch too large for the workspace."""
import numpy as np
import pytest

from helpers import small_scene_2d, small_scene_3d, to_torch

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_2508_12615_amd import binding as B  # noqa: E402
from paper_2508_12615_amd.raster import Rasterizer  # noqa: E402


def _say(msg):
    print(msg, flush=True)


def _noalloc(r, images):
    batch, keep, sizes = r.make_batch(images)
    npx = sum(w * h for (w, h) in sizes)
    dev = r.device
    image = torch.full((npx, 3), float("nan"), device=dev)
    alpha = r.params.mode == B.WIPES_3D_ALPHA
    T = torch.full((npx,), float("nan"), device=dev) if alpha else None
    last = torch.full((npx,), -7, dtype=torch.int32, device=dev) if alpha else None
    st, K = B.wipes_render_fwd_noalloc(r.ctx, r.params, batch, image.data_ptr(),
                                       T.data_ptr() if alpha else None, last.data_ptr() if alpha else None,
                                       r._stream())
    torch.cuda.synchronize()
    return st, K, image, T, last


def _same(a, b):
    return a is None and b is None or torch.equal(a, b)


@pytest.mark.parametrize("mode", ["alpha", "additive"])
def test_noalloc_equals_caller_buffers_twice(mode):
    cases = [(30000, 320, 200), (4000, 96, 72)]   # second call smaller
    for i, (n, W, H) in enumerate(cases):
        _say("no-alloc %s call %d: n=%d %dx%d" % (mode, i, n, W, H))
        if mode == "alpha":
            prims, cam = small_scene_3d(n, W, H, 700 + i, 710 + i)
            r = Rasterizer(B.WIPES_3D_ALPHA)
            images = [dict(camera=cam, prims=to_torch(prims))]
        else:
            prims = small_scene_2d(n, W, H, 720 + i)
            r = Rasterizer(B.WIPES_2D_ADDITIVE)
            images = [dict(camera=(W, H), prims=to_torch(prims))]
        ref = r.forward(images)
        torch.cuda.synchronize()
        st, K, image, T, last = _noalloc(r, images)
        assert st == B.WIPES_OK and K == ref.K, (st, K, ref.K)
        assert torch.equal(image, ref.image)
        assert _same(T, ref.T_final) and _same(last, ref.last)


def test_noalloc_two_images_then_one():
    """A two-image batch, then a single smaller image on the same context."""
    r = Rasterizer(B.WIPES_3D_ALPHA)
    p0, c0 = small_scene_3d(20000, 256, 160, 731, 732)
    p1, c1 = small_scene_3d(12000, 200, 120, 733, 734)
    big = [dict(camera=c0, prims=to_torch(p0)), dict(camera=c1, prims=to_torch(p1))]
    small = [dict(camera=c1, prims=to_torch(p1))]
    for images in (big, small):
        _say("no-alloc batch of %d" % len(images))
        ref = r.forward(images)
        st, K, image, T, last = _noalloc(r, images)
        assert st == B.WIPES_OK and K == ref.K
        assert torch.equal(image, ref.image) and torch.equal(T, ref.T_final) and torch.equal(last, ref.last)


def test_noalloc_rejects_oversized_batch():
    """About 200 bytes of projection workspace per primitive: 2M primitives cannot fit in the
    static workspace; the call fails on the host before any work is queued."""
    r = Rasterizer(B.WIPES_3D_ALPHA)
    n = 2_000_000
    dev = r.device
    z = torch.zeros((n, 4), device=dev)
    prims = dict(mean=z[:, :3].contiguous(), quat=z.clone(), scale=z[:, :3].contiguous(),
                 freq=z[:, :3].contiguous(), color=z[:, :3].contiguous(), opacity=z[:, 0].contiguous())
    cam = dict(width=64, height=48, fx=50.0, fy=50.0, cx=32.0, cy=24.0, viewmat=np.eye(4))
    batch, keep, _ = r.make_batch([dict(camera=cam, prims=prims)])
    out = torch.zeros((64 * 48, 3), device=dev)
    T = torch.zeros(64 * 48, device=dev)
    last = torch.zeros(64 * 48, dtype=torch.int32, device=dev)
    st = B.lib().wipes_render_fwd_noalloc(r.ctx, B.C.byref(r.params), B.C.byref(batch), out.data_ptr(),
                                          T.data_ptr(), last.data_ptr(), None, r._stream())
    assert st == B.WIPES_ERR_CAPACITY
    assert "static workspace" in B.last_error(r.ctx)
    torch.cuda.synchronize()
    assert torch.count_nonzero(out) == 0
