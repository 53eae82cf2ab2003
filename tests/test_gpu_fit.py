"""Graph capture, L2 gradient and the fitting drivers (GPU)."""
import numpy as np
import pytest

from helpers import to_torch

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_2508_12615_amd import binding as B  # noqa: E402
from paper_2508_12615_amd import synth  # noqa: E402
from paper_2508_12615_amd.fit import BatchedFit, fit_plain  # noqa: E402
from paper_2508_12615_amd.raster import Rasterizer  # noqa: E402


def uneven_images(n=5, seed=0):
    g = np.random.default_rng(seed)
    out = []
    for i in range(n):
        W, H = int(g.integers(40, 140)), int(g.integers(40, 140))
        N = int(g.integers(200, 1500))
        out.append(dict(width=W, height=H, target=torch.from_numpy(synth.texture_1f(H, W, 900 + i)).cuda(),
                        prims=to_torch(synth.prims_2d(N, W, H, 950 + i))))
    return out


def test_l2_grad_kernel():
    ims = uneven_images(3, 1)
    r = Rasterizer(B.WIPES_2D_ADDITIVE)
    views = [dict(camera=(im["width"], im["height"]), prims=im["prims"]) for im in ims]
    f = r.forward(views)
    target = torch.cat([im["target"].reshape(-1, 3) for im in ims])
    batch, keep, _ = r.make_batch(views)
    sb, _ = B.wipes_workspace_size(r.params, batch, 0, False)
    screen = torch.empty(sb, dtype=torch.uint8, device="cuda")
    grad = torch.empty_like(f.image)
    B.wipes_l2_grad(r.ctx, r.params, batch, B.wipes_buffer(screen.data_ptr(), sb, 0, 0, 0), f.image.data_ptr(),
                    target.data_ptr(), grad.data_ptr(), torch.cuda.current_stream().cuda_stream)
    o = 0
    for im in ims:
        n = im["width"] * im["height"]
        ref = 2.0 * (f.image[o:o + n] - target[o:o + n]) / (3 * n)
        assert torch.allclose(grad[o:o + n], ref, rtol=1e-6, atol=1e-12)
        o += n


def test_graph_replays_match_eager():
    """Every replay (with eager work and synchronisation in between) equals an eager render of the
    same parameters: image, dL/dimage and gradients, bit for bit."""
    ims = uneven_images(4, 2)
    fit = BatchedFit(ims)
    r = fit.rast
    for rep in range(3):
        with torch.no_grad():
            fit.params["mean"].add_(0.05)            # eager work between replays changes the inputs
        torch.cuda.synchronize()
        fit.render_grads()
        torch.cuda.synchronize()
        assert fit.check_capacity() > 0
        views = fit._image_views()
        f = r.forward(views, with_backward=True)
        assert torch.equal(f.image, fit.image), rep
        target = fit.target
        o, dL = 0, torch.empty_like(f.image)
        for (W, H) in fit.sizes:
            n = W * H
            dL[o:o + n] = 2.0 * (f.image[o:o + n] - target[o:o + n]) / (3 * n)
            o += n
        assert torch.allclose(dL, fit.dL, rtol=1e-6, atol=0)
        grads = r.backward(views, f, fit.dL.clone())
        for b, g in enumerate(grads):
            a, z = int(fit.offsets[b]), int(fit.offsets[b + 1])
            for k in g:
                assert torch.equal(g[k], fit.params[k].grad[a:z]), (rep, b, k)
    fit.close()


def test_graph_overflow_is_reported():
    ims = uneven_images(2, 3)
    fit = BatchedFit(ims, capacity_margin=1.0)
    torch.cuda.synchronize()
    fit.render_grads()
    fit.check_capacity()                                       # fits exactly
    with torch.no_grad():
        fit.params["cov"].mul_(3.0)                            # larger footprints: more instances
    before = fit.image.clone()
    fit.render_grads()
    with pytest.raises(B.WipesError):
        fit.check_capacity()
    assert torch.equal(before, fit.image)                      # outputs untouched on overflow
    fit.close()


def test_plain_fit_reduces_loss():
    W, H = 96, 64
    target = torch.from_numpy(synth.texture_1f(H, W, 7)).cuda()
    prims = to_torch(synth.prims_2d(1500, W, H, 8))
    with torch.no_grad():
        prims["color"].mul_(0.1)
    out = fit_plain(prims, target, 60, log_every=10)
    losses = [l for _, l in out["history"]]
    assert losses[-1] < 0.5 * losses[0]


def test_batched_step_equals_plain_steps():
    """One batched (graph) step updates every image's parameters exactly as a plain step per image."""
    ims = uneven_images(3, 4)
    fit = BatchedFit(ims)
    plain = []
    for im in ims:
        prims = {k: v.clone() for k, v in im["prims"].items()}
        fit_plain(prims, im["target"], 1)
        plain.append(prims)
    fit.step()
    torch.cuda.synchronize()
    for b, pr in enumerate(plain):
        a, z = int(fit.offsets[b]), int(fit.offsets[b + 1])
        for k in pr:
            assert torch.allclose(fit.params[k].detach()[a:z], pr[k], rtol=1e-6, atol=1e-7), (b, k)
    fit.close()


def test_library_adam_matches_torch():
    """wipes_adam over several groups (two learning rates) follows torch.optim.Adam step for step
    (same update, constants formed the same way) and counts its steps on the device."""
    g = torch.Generator(device="cuda").manual_seed(5)
    sizes, lrs = [1000, 37, 4096], [1e-3, 2.5e-3, 1e-3]
    ps = [torch.randn(n, device="cuda", generator=g) for n in sizes]
    ref = [p.clone().requires_grad_(True) for p in ps]
    opt = torch.optim.Adam([dict(params=[r], lr=lr) for r, lr in zip(ref, lrs)], betas=(0.9, 0.999), eps=1e-8)
    ms = [torch.zeros_like(p) for p in ps]
    vs = [torch.zeros_like(p) for p in ps]
    step = torch.zeros(1, dtype=torch.int32, device="cuda")
    ctx = B.wipes_ctx_create(0)
    try:
        for it in range(6):
            grads = [torch.randn(n, device="cuda", generator=g) * (0.1 + it) for n in sizes]
            for r, gr in zip(ref, grads):
                r.grad = gr.clone()
            opt.step()
            B.wipes_adam(ctx, [(p, gr, m, v, lr) for p, gr, m, v, lr in zip(ps, grads, ms, vs, lrs)], 0.9, 0.999,
                         1e-8, step.data_ptr(), stream=torch.cuda.current_stream().cuda_stream)
            for p, r in zip(ps, ref):
                assert torch.allclose(p, r.detach(), rtol=1e-6, atol=1e-7), it
        assert int(step.item()) == 6
    finally:
        B.wipes_ctx_destroy(ctx)


def test_adam_skipped_after_overflow():
    """A replay that overflows the instance capacity leaves parameters, optimiser state and the step
    count unchanged; after growing the capacity the next step applies."""
    ims = uneven_images(2, 4)
    fit = BatchedFit(ims, capacity_margin=1.0)
    fit.step()
    assert fit.steps_applied() == 1
    with torch.no_grad():
        fit.params["cov"].mul_(3.0)                            # larger footprints: more instances
    before = {k: v.detach().clone() for k, v in fit.params.items()}
    m_before = {k: v.clone() for k, v in fit.adam_m.items()}
    fit.step()
    assert fit.steps_applied() == 1
    for k in before:
        assert torch.equal(before[k], fit.params[k].detach()), k
        assert torch.equal(m_before[k], fit.adam_m[k]), k
    with pytest.raises(B.WipesError):
        fit.check_capacity()
    st, K = B.wipes_check_overflow(fit.rast.ctx, fit.rast.params, fit.batch, fit.sbuf,
                                   torch.cuda.current_stream().cuda_stream)
    fit.grow(K)
    fit.step()
    assert fit.steps_applied() == 2
    fit.check_capacity()
    assert not torch.equal(before["mean"], fit.params["mean"].detach())
    fit.close()
