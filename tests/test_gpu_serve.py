"""The serving library on the GPU: results alone == in the mix, scene lifetime, stats."""
import ctypes as C

import numpy as np
import pytest

from helpers import to_torch

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_2508_12615_amd import binding as B  # noqa: E402
from paper_2508_12615_amd import synth  # noqa: E402
from paper_2508_12615_amd.raster import Rasterizer, make_camera  # noqa: E402
from paper_2508_12615_amd.serve import Server  # noqa: E402

RES = [(320, 180), (480, 270), (400, 224), (640, 360)]


def scenes():
    return [to_torch(synth.scene_3d(n, 7000 + i, velocity=True)) for i, n in enumerate((20_000, 50_000, 35_000))]


def requests(k, seed):
    g = np.random.default_rng(seed)
    out = []
    for i in range(k):
        W, H = RES[int(g.integers(0, len(RES)))]
        out.append(dict(scene=int(g.integers(0, 3)),
                        camera=synth.orbit_camera(int(g.integers(0, 1 << 30)), W, H, time=float(g.uniform(0, 1)))))
    return out


def test_served_images_equal_alone():
    """Every request rendered in a mixed, continuously batched stream equals, bit for bit, the same
    camera rendered alone by the plain rasterizer."""
    sc = scenes()
    reqs = requests(24, 1)
    srv = Server(max_slots=8, max_batch=4, hbm_budget_bytes=1 << 30)
    ids = [srv.load_scene(s) for s in sc]
    outs = [torch.full((r["camera"]["height"], r["camera"]["width"], 3), -1.0, device="cuda") for r in reqs]
    rid = [srv.submit(ids[r["scene"]], r["camera"], o) for r, o in zip(reqs, outs)]
    srv.drain()
    for i in rid:
        done, lat = srv.poll(i)
        assert done and lat >= 0
    st = srv.stats()
    assert st["completed"] == len(reqs) and st["batches"] >= 1 and st["mean_batch"] >= 1
    rast = Rasterizer(B.WIPES_3D_ALPHA)
    for r, o in zip(reqs, outs):
        f = rast.forward([dict(camera=r["camera"], prims=sc[r["scene"]])])
        assert torch.equal(f.image.view_as(o), o)
    srv.close()


def test_scene_lifetime_and_queue_limits():
    sc = scenes()
    srv = Server(max_slots=2, max_batch=1, max_pending=3, hbm_budget_bytes=1 << 30)
    a = srv.load_scene(sc[1])
    cam = synth.orbit_camera(5, 640, 360)
    outs = [torch.empty((360, 640, 3), device="cuda") for _ in range(8)]
    busy = 0
    ids = []
    for o in outs:
        try:
            ids.append(srv.submit(a, cam, o))
        except B.WipesError as e:
            assert e.status == B.WIPES_ERR_BUSY
            busy += 1
    # requests are pending or in flight: the scene cannot go away
    assert srv.unload_scene(a) in (B.WIPES_ERR_BUSY, B.WIPES_OK)
    srv.drain()
    assert srv.unload_scene(a) == B.WIPES_OK
    with pytest.raises(B.WipesError):
        srv.submit(a, cam, outs[0])
    srv.close()


def test_submit_rejects_mis_sized_output():
    """The library writes through the raw output pointer: wipes_serve_submit itself rejects a
    buffer smaller than the camera's image (WIPES_ERR_NOMEM), and the client rejects layouts it
    cannot pass as one contiguous float32 array, before anything is queued."""
    sc = scenes()
    srv = Server(max_slots=2, max_batch=1, hbm_budget_bytes=1 << 30)
    a = srv.load_scene(sc[0])
    cam = synth.orbit_camera(5, 640, 360)
    with pytest.raises(B.WipesError) as ei:
        srv.submit(a, cam, torch.empty((180, 320, 3), device="cuda"))
    assert ei.value.status == B.WIPES_ERR_NOMEM
    small = torch.empty(640 * 360 * 3 - 1, device="cuda")
    rid = C.c_uint64()
    st = B.lib().wipes_serve_submit(srv.h, a, C.byref(make_camera(cam)), small.data_ptr(), small.numel(), None,
                                    C.byref(rid))
    assert st == B.WIPES_ERR_NOMEM
    for bad in (torch.empty((640, 360, 3), device="cuda").transpose(0, 1),
                torch.empty((360, 640, 3), dtype=torch.float64, device="cuda")):
        with pytest.raises(ValueError):
            srv.submit(a, cam, bad)
    assert srv.stats()["admitted"] == 0
    srv.close()


def test_submit_waits_for_the_callers_stream():
    """A fill of the output queued on the caller's stream before submit -- here behind a long
    sleep kernel -- lands before the served image, never over it."""
    sc = scenes()
    srv = Server(max_slots=4, max_batch=2, hbm_budget_bytes=1 << 30)
    a = srv.load_scene(sc[0])
    cam = synth.orbit_camera(7, 320, 180)
    ref = torch.empty((180, 320, 3), device="cuda")
    srv.submit(a, cam, ref)
    srv.drain()
    s = torch.cuda.Stream()
    out = torch.empty((180, 320, 3), device="cuda")
    with torch.cuda.stream(s):
        torch.cuda._sleep(20_000_000)   # keeps the caller's stream busy well past the render
        out.fill_(-1.0)
        srv.submit(a, cam, out)
    srv.drain()
    torch.cuda.synchronize()
    assert torch.equal(out, ref)
    srv.close()


def test_small_budget_defers_but_completes():
    """With an arena that holds about one request's workspace, requests wait for memory and still
    all complete."""
    sc = scenes()
    srv = Server(max_slots=8, max_batch=4, hbm_budget_bytes=96 << 20)
    ids = [srv.load_scene(s) for s in sc]
    reqs = requests(10, 2)
    outs = [torch.empty((r["camera"]["height"], r["camera"]["width"], 3), device="cuda") for r in reqs]
    for r, o in zip(reqs, outs):
        srv.submit(ids[r["scene"]], r["camera"], o)
    srv.drain()
    st = srv.stats()
    assert st["completed"] == 10 and st["arena_peak_bytes"] <= 96 << 20
    srv.close()
