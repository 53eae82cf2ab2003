"""Parity of the HIP path with the FP64 oracle, stage by stage, on seeded
inputs; every call goes through the C ABI (via the ctypes binding).

Bars: integer work (pixel boxes, keys, sorted order, tile ranges) bit-exact;
images within 1e-4 max-abs on non-tie pixels; gradients within 1e-3
relative per tensor (max|g - g*| / max|g*|), with the upstream gradient
zeroed on tie pixels.
"""
import math

import numpy as np
import pytest

import oracle as O
from helpers import (compare_image, oracle_camera, oracle_params, rel_err, sanitize_dLdC, small_scene_3d,
                     to_torch)

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_2508_12615_amd import binding as B  # noqa: E402
from paper_2508_12615_amd import synth  # noqa: E402
from paper_2508_12615_amd.raster import Rasterizer, render  # noqa: E402

COV = {"rs": (B.WIPES_COV_RS, O.COV_RS), "cholesky": (B.WIPES_COV_CHOLESKY, O.COV_CHOLESKY)}

# Gradients across tile shapes: FP32 reordering of the same per-pixel sums (derivation and measured
# values in test_tile_shape_and_launch_form_do_not_change_results).
XSHAPE_GRAD_TOL = 1e-4


def rast2d(cov="rs", **kw):
    return Rasterizer(B.WIPES_2D_ADDITIVE, cov=COV[cov][0], **kw)


def records(frame, n):
    recs = frame.screen[: n * 64].view(torch.float32).view(n, 16).cpu().numpy()
    off = (n * 64 + 255) // 256 * 256
    aux = frame.screen[off: off + n * 16].view(torch.float32).view(n, 4).cpu().numpy()
    return recs, aux


# ----------------------------------------------------------------------------- projection

@pytest.mark.parametrize("cov", ["rs", "cholesky"])
def test_project_2d(cov):
    W, H, n = 200, 150, 3000
    prims = synth.prims_2d(n, W, H, 11, cov=cov)
    prims["cov"][:5] = 0.0                        # degenerate covariances are culled
    r = rast2d(cov)
    f = r.forward([dict(camera=(W, H), prims=to_torch(prims))])
    recs, aux = records(f, n)
    scr = O.project(oracle_params(O.MODE_ADD2D, COV[cov][1]), prims)
    valid = scr[:, 15] != 0
    assert np.array_equal(aux[:, 0] >= 0, valid) and not valid[:5].any()
    v = valid
    assert np.array_equal(recs[v, 0].astype(np.float64) + recs[v, 11], scr[v, 0])
    assert np.array_equal(recs[v, 1].astype(np.float64) + recs[v, 12], scr[v, 1])
    for c in (2, 3, 4):
        assert np.all(np.abs(recs[v, c] - scr[v, c]) <= 2e-7 * np.abs(scr[v, c]) + 1e-30)
    assert np.array_equal(recs[v, 5:11], scr[v, 5:11].astype(np.float32))
    assert np.all(aux[v, 0] >= scr[v, 12]) and np.all(aux[v, 0] <= scr[v, 12] * 1.0002 + 2e-3)


def test_project_3d():
    prims, cam = small_scene_3d(20000, 320, 180, 3001, 3002, velocity=True, time=0.37)
    r = Rasterizer(B.WIPES_3D_ALPHA)
    f = r.forward([dict(camera=cam, prims=to_torch(prims))])
    recs, aux = records(f, 20000)
    ocam = oracle_camera(cam)
    scr = O.project(oracle_params(O.MODE_ALPHA3D, O.COV_QUAT_SCALE), prims, ocam)
    keys = O.depth_keys(prims, ocam)
    valid = scr[:, 15] != 0
    assert np.array_equal(aux[:, 0] >= 0, valid)
    assert np.array_equal(aux[valid, 2].view(np.uint32), keys[valid])
    v = valid
    mx = recs[v, 0].astype(np.float64) + recs[v, 11]
    my = recs[v, 1].astype(np.float64) + recs[v, 12]
    assert np.max(np.abs(mx - scr[v, 0])) < 1e-9 * max(1.0, np.abs(scr[v, 0]).max())
    assert np.max(np.abs(my - scr[v, 1])) < 1e-9 * max(1.0, np.abs(scr[v, 1]).max())
    for c in (2, 3, 4, 5, 6):
        assert np.all(np.abs(recs[v, c] - scr[v, c]) <= 2e-7 * np.abs(scr[v, c]) + 1e-30), c
    assert np.all(aux[v, 0] >= scr[v, 12] * 0.9999999) and np.all(aux[v, 1] >= scr[v, 13] * 0.9999999)


# ----------------------------------------------------------------------------- binning and sort

@pytest.mark.parametrize("mode,tw,th,n,seed", [
    (B.WIPES_3D_ALPHA, 16, 16, 5000, 1),
    (B.WIPES_3D_ALPHA, 8, 8, 3000, 2),
    (B.WIPES_2D_ADDITIVE, 16, 16, 5000, 3),
    (B.WIPES_2D_ADDITIVE, 32, 16, 7000, 4),
    (B.WIPES_3D_ALPHA, 16, 8, 1, 5),
    (B.WIPES_2D_ADDITIVE, 8, 16, 0, 6),
    # more than 2^21 primitives: the depth sort switches to 4096-key workgroups
    (B.WIPES_3D_ALPHA, 16, 16, 2_200_000, 7),
])
@pytest.mark.parametrize("W,H", [(333, 257)])
def test_bin_sort_bit_exact(mode, tw, th, n, seed, W, H):
    """Given the same FP32 records, boxes, instance keys, sorted order and ranges match O-bin."""
    _bin_sort_case(mode, tw, th, n, seed, W, H)


@pytest.mark.parametrize("mode", [B.WIPES_3D_ALPHA, B.WIPES_2D_ADDITIVE])
def test_bin_sort_more_than_65536_tiles(mode):
    """2200 x 2048 pixels in 8 x 8 tiles (70400 tiles, 17-bit tile keys): the tile sort
    takes three passes and stages 32-bit keys; the result still matches O-bin bit for bit."""
    _bin_sort_case(mode, 8, 8, 20000, 8, 2200, 2048)


def _bin_sort_case(mode, tw, th, n, seed, W, H):
    rec = synth.screen_records(max(n, 1), W, H, seed)
    rec = {k: v[:n] for k, v in rec.items()}
    p = B.wipes_params_default(mode)
    p.tile_w, p.tile_h = tw, th
    dev = torch.device("cuda")
    dummy = torch.zeros((max(n, 1), 4), dtype=torch.float32, device=dev)
    img = B.wipes_image()
    img.cam.width, img.cam.height, img.cam.fx, img.cam.fy = W, H, 1.0, 1.0
    img.prims.n = n
    for k in ("mean", "cov", "quat", "scale", "freq", "color", "opacity"):
        setattr(img.prims, k, dummy.data_ptr())
    arr = (B.wipes_image * 1)(img)
    batch = B.wipes_batch(1, arr)
    sb, _ = B.wipes_workspace_size(p, batch, 0, False)
    screen = torch.zeros(sb, dtype=torch.uint8, device=dev)
    if n:
        recs = np.zeros((n, 16), np.float32)
        recs[:, 0], recs[:, 1] = rec["mx"], rec["my"]
        recs[:, 2], recs[:, 3], recs[:, 4] = rec["ca"], rec["cb"], rec["cc"]
        aux = np.zeros((n, 4), np.float32)
        aux[:, 0], aux[:, 1], aux[:, 2], aux[:, 3] = rec["rx"], rec["ry"], rec["depth"], rec["Qs"]
        off = (n * 64 + 255) // 256 * 256
        screen[: n * 64] = torch.from_numpy(recs.view(np.uint8).reshape(-1)).to(dev)
        screen[off: off + n * 16] = torch.from_numpy(aux.view(np.uint8).reshape(-1)).to(dev)
    omode = O.MODE_ALPHA3D if mode == B.WIPES_3D_ALPHA else O.MODE_ADD2D
    ob = O.bin_tiles(W, H, tw, th, omode, rec["mx"], rec["my"], rec["rx"], rec["ry"], rec["depth"], rec["ca"],
                     rec["cb"], rec["cc"], rec["Qs"])
    cap = ob["K"] + 17
    _, bb = B.wipes_workspace_size(p, batch, cap, True)
    bins = torch.zeros(bb, dtype=torch.uint8, device=dev)
    sbuf = B.wipes_buffer(screen.data_ptr(), sb, 0, 0, 0)
    bbuf = B.wipes_buffer(bins.data_ptr(), bb, cap, 1, 0)
    ctx = B.wipes_ctx_create(0)
    try:
        st, K = B.wipes_bin_sort(ctx, p, batch, sbuf, bbuf)
        assert st == B.WIPES_OK and K == ob["K"]
        kp, vp, rp, nt = B.wipes_bins_view(p, batch, sbuf, bbuf)
        torch.cuda.synchronize()
        base = bins.data_ptr()
        get = lambda ptr, cnt: bins[ptr - base: ptr - base + 4 * cnt].view(torch.int32).cpu().numpy().view(np.uint32)
        tiles_ref = (ob["keys"] >> np.uint64(32)) if omode == O.MODE_ALPHA3D else ob["keys"]
        assert np.array_equal(get(kp, K), tiles_ref.astype(np.uint32))
        assert np.array_equal(get(vp, K), ob["vals"])
        assert np.array_equal(get(rp, 2 * nt).reshape(nt, 2), ob["ranges"])
        if n:
            boxes = screen[: n * 64].view(torch.int32).view(n, 16)[:, 14:16].cpu().numpy().view(np.uint32)
            bx = ob["box"]
            nonempty = (bx[:, 0] <= bx[:, 2]) & (bx[:, 1] <= bx[:, 3])
            assert np.array_equal(boxes[nonempty, 0], (bx[nonempty, 0] | (bx[nonempty, 1] << 16)).astype(np.uint32))
            assert np.array_equal(boxes[nonempty, 1], (bx[nonempty, 2] | (bx[nonempty, 3] << 16)).astype(np.uint32))
        # capacity: one instance short is reported, with the required count
        if K > 0:
            bbuf2 = B.wipes_buffer(bins.data_ptr(), bb, K - 1, 1, 0)
            st2, K2 = B.wipes_bin_sort(ctx, p, batch, sbuf, bbuf2)
            assert st2 == B.WIPES_ERR_CAPACITY and K2 == K
    finally:
        B.wipes_ctx_destroy(ctx)


# ----------------------------------------------------------------------------- forward

@pytest.mark.parametrize("cov", ["rs", "cholesky"])
@pytest.mark.parametrize("tile", [(16, 16), (8, 8), (32, 16)])
def test_render_2d(cov, tile):
    W, H, n = 150, 118, 1200
    prims = synth.prims_2d(n, W, H, 21, cov=cov)
    r = rast2d(cov, tile_w=tile[0], tile_h=tile[1])
    f = r.forward([dict(camera=(W, H), prims=to_torch(prims))])
    P = oracle_params(O.MODE_ADD2D, COV[cov][1])
    ref, _, _, tie, jb = O.render_o1(P, W, H, O.project(P, prims), jump=True)
    compare_image(f.image.cpu().numpy(), ref, tie, jb)


def test_render_3d():
    prims, cam = small_scene_3d(8000, 240, 136, 3001, 3002)
    r = Rasterizer(B.WIPES_3D_ALPHA)
    f = r.forward([dict(camera=cam, prims=to_torch(prims))])
    P = oracle_params(O.MODE_ALPHA3D, O.COV_QUAT_SCALE)
    ocam = oracle_camera(cam)
    ref, T, nc, tie, jb = O.render_o1(P, cam["width"], cam["height"], O.project(P, prims, ocam),
                                      O.depth_keys(prims, ocam), jump=True)
    assert nc.max() > 20 and (T < 1e-4).mean() > 0.01      # the scene exercises compositing and termination
    compare_image(f.image.cpu().numpy(), ref, tie, jb, T_gpu=f.T_final.cpu().numpy(), T_ref=T)


def test_render_3d_background_and_velocity():
    prims, cam = small_scene_3d(3000, 160, 100, 3101, 3102, velocity=True, time=0.6)
    bg = (0.25, 0.5, 0.75)
    r = Rasterizer(B.WIPES_3D_ALPHA, bg=bg)
    f = r.forward([dict(camera=cam, prims=to_torch(prims))])
    P = oracle_params(O.MODE_ALPHA3D, O.COV_QUAT_SCALE, bg=bg)
    ocam = oracle_camera(cam)
    ref, _, _, tie, jb = O.render_o1(P, cam["width"], cam["height"], O.project(P, prims, ocam),
                                     O.depth_keys(prims, ocam), jump=True)
    compare_image(f.image.cpu().numpy(), ref, tie, jb)


def test_empty_and_offscreen():
    """No primitives, and primitives entirely off screen: background only."""
    r = Rasterizer(B.WIPES_3D_ALPHA, bg=(0.1, 0.2, 0.3))
    prims, cam = small_scene_3d(64, 40, 24, 1, 2)
    prims["opacity"][:] = np.float32(0.001)                  # below alpha_min: every primitive is culled
    f = r.forward([dict(camera=cam, prims=to_torch(prims))])
    img = f.image.cpu().numpy()
    assert f.K == 0 and np.allclose(img, np.float32([0.1, 0.2, 0.3]))
    r2 = rast2d()
    empty = {k: v[:0] for k, v in synth.prims_2d(1, 20, 20, 1).items()}
    f2 = r2.forward([dict(camera=(20, 20), prims=to_torch(empty))])
    assert f2.K == 0 and np.all(f2.image.cpu().numpy() == 0)


# ----------------------------------------------------------------------------- backward

@pytest.mark.parametrize("cov", ["rs", "cholesky"])
def test_backward_2d(cov):
    W, H, n = 96, 80, 400
    prims = synth.prims_2d(n, W, H, 31, cov=cov)
    tp = to_torch(prims)
    r = rast2d(cov)
    f = r.forward([dict(camera=(W, H), prims=tp)], with_backward=True)
    P = oracle_params(O.MODE_ADD2D, COV[cov][1])
    scr = O.project(P, prims)
    ref, _, _, tie, jb = O.render_o1(P, W, H, scr, jump=True)
    compare_image(f.image.cpu().numpy(), ref, tie, jb)
    g = sanitize_dLdC(np.random.default_rng(5).normal(0, 1, (H * W, 3)).astype(np.float32), tie)
    grads, ds = r.backward([dict(camera=(W, H), prims=tp)], f, torch.from_numpy(g.astype(np.float32)).cuda(),
                           want_dscreen=True)
    ds_ref = O.render_bwd_o1(P, W, H, scr, g)
    for c in range(11):
        assert rel_err(ds.cpu().numpy()[:, c], ds_ref[:, c]) < 1e-3, c
    pg = O.project_bwd(P, prims, scr, ds_ref)
    for k in ("mean", "cov", "freq", "color", "opacity"):
        assert rel_err(grads[0][k].cpu().numpy(), pg[k]) < 1e-3, k


@pytest.mark.parametrize("velocity", [False, True])
def test_backward_3d(velocity):
    prims, cam = small_scene_3d(3000, 128, 96, 3201, 3202, velocity=velocity, time=0.45)
    tp = to_torch(prims)
    r = Rasterizer(B.WIPES_3D_ALPHA, bg=(0.3, 0.2, 0.1))
    f = r.forward([dict(camera=cam, prims=tp)], with_backward=True)
    P = oracle_params(O.MODE_ALPHA3D, O.COV_QUAT_SCALE, bg=(0.3, 0.2, 0.1))
    ocam = oracle_camera(cam)
    scr = O.project(P, prims, ocam)
    keys = O.depth_keys(prims, ocam)
    W, H = cam["width"], cam["height"]
    ref, T, nc, tie, jb = O.render_o1(P, W, H, scr, keys, jump=True)
    compare_image(f.image.cpu().numpy(), ref, tie, jb, T_gpu=f.T_final.cpu().numpy(), T_ref=T)
    g = sanitize_dLdC(np.random.default_rng(6).normal(0, 1, (H * W, 3)).astype(np.float32), tie)
    grads, ds = r.backward([dict(camera=cam, prims=tp)], f, torch.from_numpy(g.astype(np.float32)).cuda(),
                           want_dscreen=True)
    ds_ref = O.render_bwd_o1(P, W, H, scr, g, keys)
    dsg = ds.cpu().numpy()
    for c in range(11):
        assert rel_err(dsg[:, c], ds_ref[:, c]) < 1e-3, c
    pg = O.project_bwd(P, prims, scr, ds_ref, ocam)
    names = ["mean", "quat", "scale", "freq", "color", "opacity"] + (["velocity"] if velocity else [])
    for k in names:
        assert rel_err(grads[0][k].cpu().numpy(), pg[k]) < 1e-3, k


def test_autograd_matches_direct_backward():
    W, H, n = 64, 48, 300
    prims = synth.prims_2d(n, W, H, 41)
    tp = {k: v.clone().requires_grad_(True) for k, v in to_torch(prims).items()}
    r = rast2d()
    img = render(r, (W, H), **tp)
    target = torch.rand((H, W, 3), device="cuda", generator=torch.Generator("cuda").manual_seed(0))
    loss = ((img - target) ** 2).mean()
    loss.backward()
    f = r.forward([dict(camera=(W, H), prims=to_torch(prims))], with_backward=True)
    g = (2.0 * (f.image.view(H, W, 3) - target) / (H * W * 3)).reshape(-1, 3)
    gd = r.backward([dict(camera=(W, H), prims=to_torch(prims))], f, g)[0]
    for k in ("mean", "cov", "freq", "color", "opacity"):
        assert torch.allclose(tp[k].grad, gd[k], rtol=1e-5, atol=1e-9), k


# ----------------------------------------------------------------------------- invariances

@pytest.mark.parametrize("mode", [B.WIPES_2D_ADDITIVE, B.WIPES_3D_ALPHA])
def test_tile_shape_and_launch_form_do_not_change_results(mode):
    """The per-pixel rule is tile-independent.  Grid, queue and longest-first queue launches of one
    tile shape give bit-identical images and gradients.  Across tile shapes the images are
    bit-identical too (every 8x8 block sees the same primitives in the same order, in block-relative
    coordinates).  Gradients sum the same per-pixel terms grouped differently (block, tile and slot
    sums), so they differ by FP32 reordering: about sqrt(n) u of the terms' magnitude for n terms
    (u = 2^-24; n up to ~8e3 pixels per primitive here gives ~5e-6), more where a gradient's terms
    cancel.  Measured per tensor: 6.1e-6 (2D) and 7.1e-6 (3D) here, 2.3e-5 over the autotuner's 2D
    batch (primitives of up to ~1e4 pixels).  The bar, 1e-4 relative per tensor, keeps a 4x margin
    over the largest and sits far inside the oracle bar (1e-3)."""
    if mode == B.WIPES_2D_ADDITIVE:
        W, H = 131, 77
        prims = synth.prims_2d(900, W, H, 51)
        cam = (W, H)
    else:
        prims, cam = small_scene_3d(4000, 131, 77, 3301, 3302)
        W, H = cam["width"], cam["height"]
    tp = to_torch(prims)
    g = torch.from_numpy(np.random.default_rng(7).normal(0, 1, (W * H, 3)).astype(np.float32)).cuda()
    base = None
    worst = 0.0
    for tile in [(16, 16), (8, 8), (16, 8), (8, 16), (32, 8), (32, 16)]:
        same_tile = None
        for persistent in (0, 1, 2, 3):
            r = Rasterizer(mode, tile_w=tile[0], tile_h=tile[1], persistent=persistent)
            f = r.forward([dict(camera=cam, prims=tp)], with_backward=True)
            gr = r.backward([dict(camera=cam, prims=tp)], f, g)[0]
            out = (f.image.cpu().numpy(), {k: v.cpu().numpy() for k, v in gr.items()})
            if same_tile is None:
                same_tile = out
            else:
                assert np.array_equal(out[0], same_tile[0]), tile
                for k in out[1]:
                    assert np.array_equal(out[1][k], same_tile[1][k]), (tile, k)
            if base is None:
                base = out
                continue
            assert np.array_equal(out[0], base[0]), (tile, persistent)
            for k in base[1]:
                e = rel_err(out[1][k], base[1][k])
                worst = max(worst, e)
                assert e < XSHAPE_GRAD_TOL, (tile, persistent, k)
    print("worst cross-shape gradient rel err %.2e" % worst, flush=True)


@pytest.mark.parametrize("launch", [(16, 16, 0), (32, 16, 2), (8, 8, 1), (8, 16, 3)])
@pytest.mark.parametrize("mode", [B.WIPES_2D_ADDITIVE, B.WIPES_3D_ALPHA])
def test_batched_equals_single(mode, launch):
    """Several images of different sizes rendered in one call give, bit for bit, the images and
    gradients of rendering each alone."""
    imgs = []
    for i, (W, H, n) in enumerate([(97, 61, 700), (64, 64, 300), (150, 33, 500)]):
        if mode == B.WIPES_2D_ADDITIVE:
            imgs.append(dict(camera=(W, H), prims=to_torch(synth.prims_2d(n, W, H, 70 + i))))
        else:
            prims, cam = small_scene_3d(n * 3, W, H, 3500 + i, 3600 + i, velocity=(i == 1), time=0.3)
            imgs.append(dict(camera=cam, prims=to_torch(prims)))
    npx = [97 * 61, 64 * 64, 150 * 33]
    g = torch.from_numpy(np.random.default_rng(9).normal(0, 1, (sum(npx), 3)).astype(np.float32)).cuda()
    r = Rasterizer(mode, tile_w=launch[0], tile_h=launch[1], persistent=launch[2])
    fb = r.forward(imgs, with_backward=True)
    gb = r.backward(imgs, fb, g)
    o = 0
    for i, im in enumerate(imgs):
        f1 = r.forward([im], with_backward=True)
        g1 = r.backward([im], f1, g[o:o + npx[i]].contiguous())[0]
        assert torch.equal(f1.image, fb.image[o:o + npx[i]]), i
        if mode == B.WIPES_3D_ALPHA:
            assert torch.equal(f1.T_final, fb.T_final[o:o + npx[i]]), i
        for k in g1:
            assert torch.equal(g1[k], gb[i][k]), (i, k)
        o += npx[i]


def test_longest_first_order_over_many_tiles():
    """30000 tiles (the two-pass longest-first ordering, two slices of workgroups): the
    longest-first queue gives the grid launch's images and gradients bit for bit."""
    W, H = 1600, 1200
    prims = to_torch(synth.prims_2d(30000, W, H, 81))
    g = torch.from_numpy(np.random.default_rng(11).normal(0, 1, (W * H, 3)).astype(np.float32)).cuda()
    outs = []
    for persistent in (0, 2):
        r = Rasterizer(B.WIPES_2D_ADDITIVE, tile_w=8, tile_h=8, persistent=persistent)
        f = r.forward([dict(camera=(W, H), prims=prims)], with_backward=True)
        gr = r.backward([dict(camera=(W, H), prims=prims)], f, g)[0]
        outs.append((f.image.cpu(), {k: v.cpu() for k, v in gr.items()}))
    assert torch.equal(outs[0][0], outs[1][0])
    for k in outs[0][1]:
        assert torch.equal(outs[0][1][k], outs[1][1][k]), k


def test_batched_more_than_eight_images():
    """Ten images in one call (the descriptor table then goes through the pinned staging ring,
    not a kernel argument) give, bit for bit, the images and gradients of each alone."""
    imgs, npx = [], []
    for i in range(10):
        W, H = 40 + 7 * i, 30 + 5 * i
        imgs.append(dict(camera=(W, H), prims=to_torch(synth.prims_2d(150 + 20 * i, W, H, 90 + i))))
        npx.append(W * H)
    g = torch.from_numpy(np.random.default_rng(12).normal(0, 1, (sum(npx), 3)).astype(np.float32)).cuda()
    r = Rasterizer(B.WIPES_2D_ADDITIVE, persistent=2)
    fb = r.forward(imgs, with_backward=True)
    gb = r.backward(imgs, fb, g)
    o = 0
    for i, im in enumerate(imgs):
        f1 = r.forward([im], with_backward=True)
        g1 = r.backward([im], f1, g[o:o + npx[i]].contiguous())[0]
        assert torch.equal(f1.image, fb.image[o:o + npx[i]]), i
        for k in g1:
            assert torch.equal(g1[k], gb[i][k]), (i, k)
        o += npx[i]


@pytest.mark.parametrize("mode", [B.WIPES_2D_ADDITIVE, B.WIPES_3D_ALPHA])
def test_deterministic(mode):
    if mode == B.WIPES_2D_ADDITIVE:
        prims, cam = synth.prims_2d(2000, 200, 160, 61), (200, 160)
        W, H = cam
    else:
        prims, cam = small_scene_3d(6000, 200, 160, 3401, 3402)
        W, H = cam["width"], cam["height"]
    tp = to_torch(prims)
    g = torch.from_numpy(np.random.default_rng(8).normal(0, 1, (W * H, 3)).astype(np.float32)).cuda()
    outs = []
    for _ in range(2):
        r = Rasterizer(mode)
        f = r.forward([dict(camera=cam, prims=tp)], with_backward=True)
        gr = r.backward([dict(camera=cam, prims=tp)], f, g)[0]
        outs.append((f.image.cpu().numpy(), {k: v.cpu().numpy() for k, v in gr.items()}))
    assert np.array_equal(outs[0][0], outs[1][0])
    for k in outs[0][1]:
        assert np.array_equal(outs[0][1][k], outs[1][1][k]), k


@pytest.mark.parametrize("mode", [B.WIPES_2D_ADDITIVE, B.WIPES_3D_ALPHA])
def test_repeated_renders_of_one_bin_sort(mode):
    """The first forward and backward render after a bin_sort skip the clears that bin_sort
    already did; a second forward render and a second backward on the same bins clear again
    and must give the same image, T, last and gradients bit for bit."""
    if mode == B.WIPES_2D_ADDITIVE:
        prims, cam = synth.prims_2d(2500, 208, 152, 71), (208, 152)
        W, H = cam
    else:
        prims, cam = small_scene_3d(5000, 208, 152, 3501, 3502)
        W, H = cam["width"], cam["height"]
    tp = to_torch(prims)
    ims = [dict(camera=cam, prims=tp)]
    g = torch.from_numpy(np.random.default_rng(9).normal(0, 1, (W * H, 3)).astype(np.float32)).cuda()
    r = Rasterizer(mode, persistent=2)
    f = r.forward(ims, with_backward=True)
    g1 = r.backward(ims, f, g)[0]
    g2 = r.backward(ims, f, g)[0]   # slot marks and queue counters are stale now: cleared again
    for k in g1:
        assert torch.equal(g1[k], g2[k]), k
    # a second forward render into fresh outputs from the same bins
    batch, keep, _ = r.make_batch(ims)
    sbuf = B.wipes_buffer(f.screen.data_ptr(), f.screen.numel(), 0, 0, 0)
    bbuf = B.wipes_buffer(f.bins.data_ptr(), f.bins.numel(), f.cap, 1, 0)
    img2 = torch.full_like(f.image, 7.0)
    T2 = torch.full_like(f.T_final, 7.0) if f.T_final is not None else None
    last2 = torch.full_like(f.last, 7) if f.last is not None else None
    B.wipes_render_fwd(r.ctx, r.params, batch, sbuf, bbuf, img2.data_ptr(), None if T2 is None else T2.data_ptr(),
                       None if last2 is None else last2.data_ptr(), r._stream())
    torch.cuda.synchronize()
    assert torch.equal(img2, f.image)
    if T2 is not None:
        assert torch.equal(T2, f.T_final) and torch.equal(last2, f.last)
    g3 = r.backward(ims, f, g)[0]   # its contribution mask was rebuilt by the second forward
    for k in g1:
        assert torch.equal(g1[k], g3[k]), k


# ----------------------------------------------------------------------------- full-size workloads

def test_config1_full_size():
    """2D fit, 512x512, 10k primitives: full-image forward and backward against O1."""
    c = synth.config1()
    W, H = c["width"], c["height"]
    tp = to_torch(c["prims"])
    r = rast2d()
    f = r.forward([dict(camera=(W, H), prims=tp)], with_backward=True)
    P = oracle_params(O.MODE_ADD2D, O.COV_RS)
    scr = O.project(P, c["prims"])
    ref, _, _, tie, jb = O.render_o1(P, W, H, scr, jump=True)
    compare_image(f.image.cpu().numpy(), ref, tie, jb)
    # L2 loss gradient against the 1/f target, tie pixels masked
    g = (2.0 * (f.image.cpu().numpy() - c["target"].reshape(-1, 3)) / (W * H * 3)).astype(np.float32)
    g = sanitize_dLdC(g, tie).astype(np.float32)
    grads = r.backward([dict(camera=(W, H), prims=tp)], f, torch.from_numpy(g).cuda())[0]
    ds_ref = O.render_bwd_o1(P, W, H, scr, g)
    pg = O.project_bwd(P, c["prims"], scr, ds_ref)
    for k in ("mean", "cov", "freq", "color", "opacity"):
        assert rel_err(grads[k].cpu().numpy(), pg[k]) < 1e-3, k


def test_config3_full_size_sampled():
    """3D, 1M primitives, 1920x1080: sampled pixels against O1 (brute force over all primitives),
    and the full backward under an upstream gradient supported on those pixels."""
    c = synth.config3()
    cam = c["camera"]
    W, H = cam["width"], cam["height"]
    tp = to_torch(c["prims"])
    r = Rasterizer(B.WIPES_3D_ALPHA)
    f = r.forward([dict(camera=cam, prims=tp)], with_backward=True)
    img = f.image.cpu().numpy()
    P = oracle_params(O.MODE_ALPHA3D, O.COV_QUAT_SCALE)
    ocam = oracle_camera(cam)
    scr = O.project(P, c["prims"], ocam)
    keys = O.depth_keys(c["prims"], ocam)
    gsel = np.random.default_rng(9)
    # sample covered pixels (where the image is not background) and a few random ones
    covered = np.flatnonzero(img.max(axis=1) > 0.05)
    pix = np.unique(np.concatenate([gsel.choice(covered, 200, replace=False), gsel.integers(0, W * H, 56)]))
    ref, T, nc, tie, jb = O.render_o1(P, W, H, scr, keys, pix=pix, jump=True)
    assert nc.max() > 20
    compare_image(img[pix], ref, tie, jb, min_tie_allow=2, T_gpu=f.T_final.cpu().numpy()[pix], T_ref=T)
    # backward with dL/dC supported on the sampled non-tie pixels
    gpix = pix[tie == 0][:96]
    gv = gsel.normal(0, 1, (gpix.size, 3)).astype(np.float32)
    g = np.zeros((W * H, 3), np.float32)
    g[gpix] = gv
    grads, ds = r.backward([dict(camera=cam, prims=tp)], f, torch.from_numpy(g).cuda(), want_dscreen=True)
    ds_ref = O.render_bwd_o1(P, W, H, scr, gv, keys, pix=gpix)
    dsg = ds.cpu().numpy()
    touched = np.flatnonzero(np.abs(ds_ref).sum(axis=1) > 0)
    assert touched.size > 100
    for col in range(11):
        assert rel_err(dsg[touched, col], ds_ref[touched, col]) < 1e-3, col
    others = np.setdiff1d(np.arange(dsg.shape[0]), touched)
    assert np.all(dsg[others] == 0.0)


@pytest.mark.parametrize("mode", [B.WIPES_2D_ADDITIVE, B.WIPES_3D_ALPHA])
def test_work_counts_match_oracle(mode):
    """The support-pair counts used as the roofline numerator equal the oracle's (up to support ties)."""
    if mode == B.WIPES_2D_ADDITIVE:
        W, H = 120, 90
        prims = synth.prims_2d(800, W, H, 81)
        cam = (W, H)
        P = oracle_params(O.MODE_ADD2D, O.COV_RS)
        scr = O.project(P, prims)
        keys = None
    else:
        prims, cam = small_scene_3d(5000, 120, 90, 3701, 3702)
        W, H = cam["width"], cam["height"]
        P = oracle_params(O.MODE_ALPHA3D, O.COV_QUAT_SCALE)
        ocam = oracle_camera(cam)
        scr = O.project(P, prims, ocam)
        keys = O.depth_keys(prims, ocam)
    r = Rasterizer(mode)
    im = [dict(camera=cam, prims=to_torch(prims))]
    f = r.forward(im, with_backward=True)
    st = r.stats(im, f)
    cf, cb = O.support_counts(P, W, H, scr, keys)
    assert abs(st["support_fwd"] - cf.sum()) <= 1e-4 * cf.sum() + 4
    assert abs(st["support_bwd"] - cb.sum()) <= 1e-4 * cb.sum() + 4
    assert st["tile_pairs"] >= st["subblock_pairs"] >= st["support_fwd"] >= st["support_bwd"] > 0
