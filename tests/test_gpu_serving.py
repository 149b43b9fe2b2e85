"""GPU tests of novel-view serving: plx_render_views against the FP64 oracle
(camera rays from the same pinhole definition, rendered by the oracle) on
small scenes and, on sampled pixels, at 1920x1080 on 512^3 and 256^3 FP16
scenes; a view rendered alone versus inside mixed batches (bitwise equal: a
pixel's colour depends only on its own ray and scene); a scene table of
another storage type (nothing rendered, status raised); launches on two
streams overlapping on the device; and the continuous-batching server
(every result equal to its stand-alone render, admission within the HBM
budget)."""
import math

import numpy as np
import pytest
import torch

import synth
from oracle import oracle as O
from paper_2112_05131_amd import binding as B
from paper_2112_05131_amd.serve import Request, Server, random_requests, run_load
from tests.gpu_util import RGB_ATOL, make_pair, say

pytestmark = pytest.mark.gpu


def _scenes(sh_dtype=B.PLX_F32):
    a = synth.blob_scene((48, 48, 48), n_blobs=6, occupancy=0.1, seed=3)
    b = synth.blob_scene((40, 56, 36), n_blobs=5, occupancy=0.08, seed=4)
    pa = make_pair(a, sh_dtype=sh_dtype)
    pb = make_pair(b, sh_dtype=sh_dtype)
    return [pa[0], pb[0]], [pa[1], pb[1]]


def _view(req, off=0):
    v = B.PlxView()
    v.c2w[:] = [float(x) for x in np.asarray(req.c2w, np.float64).reshape(12)]
    v.focal = float(req.focal)
    v.width, v.height, v.scene, v.reserved = req.width, req.height, req.scene, 0
    v.out_offset = off
    return v


def _render(grids, reqs):
    views, off = [], 0
    for r in reqs:
        views.append(_view(r, off))
        off += r.n_pixels
    out = torch.full((off * 3,), -1.0, device="cuda")
    q = B.views_queue()
    B.plx_render_views(B.SceneTable(grids), views, out, q)
    B.plx_render_views_status(q)
    assert torch.count_nonzero(q[:12]).item() == 0  # left at zero for the next launch
    res, off = [], 0
    for r in reqs:
        res.append(out[3 * off:3 * (off + r.n_pixels)].view(r.height, r.width, 3).clone())
        off += r.n_pixels
    return res


@pytest.mark.parametrize("sh_dtype", [B.PLX_F32, B.PLX_F16])
def test_views_match_oracle(sh_dtype):
    say("views vs oracle", sh_dtype)
    ogs, grids = _scenes(sh_dtype)
    reqs = random_requests(3, 2, seed=5, resolutions=((37, 23), (64, 48), (50, 50)))
    outs = _render(grids, reqs)
    for r, img in zip(reqs, outs):
        o, d = O.camera_rays(r.c2w, r.focal, r.width, r.height)
        ref = O.render_fwd(ogs[r.scene], o, d)[0].reshape(r.height, r.width, 3)
        err = np.abs(img.cpu().double().numpy() - ref).max()
        assert err <= RGB_ATOL, err


def test_view_alone_equals_view_in_mixed_batches():
    say("views alone vs mixed")
    _, grids = _scenes()
    reqs = random_requests(7, 2, seed=6, resolutions=((31, 17), (80, 60), (120, 90), (16, 16)))
    alone = [_render(grids, [r])[0] for r in reqs]
    mixed = _render(grids, reqs)
    rev = _render(grids, reqs[::-1])[::-1]
    for a, m, v in zip(alone, mixed, rev):
        assert torch.equal(a, m) and torch.equal(a, v)


def test_server_continuous_batching_results_and_budget():
    say("server")
    _, grids = _scenes()
    reqs = random_requests(40, 2, seed=7, resolutions=((64, 64), (128, 96), (200, 200), (48, 32)))
    refs = [_render(grids, [r])[0] for r in reqs]
    budget = 3 * 200 * 200 * 12  # room for about three large requests
    srv = Server(grids, hbm_budget=budget, n_streams=3, max_batch=8)
    # arrivals spread in time: some requests join while others run
    lat, wall = run_load(srv, reqs, rate_hz=4000.0, seed=8)
    assert 0 < srv.peak_in_use <= budget
    for r, ref in zip(reqs, refs):
        assert r.done and torch.equal(r.rgb, ref)
        assert r.t_done >= r.t_launch >= r.t_arrival
    assert len(lat) == len(reqs) and np.all(lat > 0)
    # FIFO admission: launch order follows arrival order
    t_launch = np.array([r.t_launch for r in reqs])
    assert np.all(np.diff(t_launch) >= 0)
    assert srv.in_use == 0 and not srv.inflight and not srv.queue
    with pytest.raises(ValueError):
        srv.submit(Request(0, reqs[0].c2w, 100.0, 1000, 1000))  # beyond the budget


def test_views_c5_size_sampled_against_oracle():
    """One launch with a 1920x1080 view of a 512^3 (5%) and of a 256^3 (10%)
    FP16 scene (the serving configuration's largest requests); 1500 sampled
    pixels of each against the oracle fed the stored FP16 coefficients."""
    say("views at 1920x1080, sampled")
    svs = [synth.blob_scene((512,) * 3, 32, 0.05, 3), synth.blob_scene((256,) * 3, 32, 0.10, 4)]
    pairs = [make_pair(sv, sh_dtype=B.PLX_F16) for sv in svs]
    ogs, grids = [p[0] for p in pairs], [p[1] for p in pairs]
    reqs = random_requests(2, 2, seed=31, resolutions=((1920, 1080),))
    reqs[0].scene, reqs[1].scene = 0, 1
    outs = _render(grids, reqs)
    rng = np.random.default_rng(32)
    for r, img in zip(reqs, outs):
        o, d = O.camera_rays(r.c2w, r.focal, r.width, r.height)
        sel = np.sort(rng.choice(r.n_pixels, 1500, replace=False))
        ref = O.render_fwd(ogs[r.scene], o[sel], d[sel])[0]
        got = img.reshape(-1, 3)[torch.from_numpy(sel).cuda()].cpu().double().numpy()
        err = np.abs(got - ref).max()
        say(f"  scene {r.scene}: max |gpu - oracle| over 1500 pixels = {err:.2e}")
        assert err <= RGB_ATOL, err
        assert torch.all(img >= 0)  # every pixel written


def test_scene_table_of_another_storage_type_renders_nothing():
    say("views: table / dtype mismatch")
    _, grids = _scenes(B.PLX_F32)
    table = B.SceneTable(grids)
    reqs = random_requests(2, 2, seed=9, resolutions=((40, 30),))
    views = [_view(reqs[0], 0), _view(reqs[1], reqs[0].n_pixels)]
    out = torch.full((3 * sum(r.n_pixels for r in reqs),), -1.0, device="cuda")
    q = B.views_queue()
    table.sh_dtype = B.PLX_F16  # claims FP16 over an FP32 table
    B.plx_render_views(table, views, out, q)
    with pytest.raises(B.PlxError, match="not rendered"):
        B.plx_render_views_status(q)
    assert torch.all(out == -1.0)
    table.sh_dtype = B.PLX_F32
    q = B.views_queue()
    B.plx_render_views(table, views, out, q)
    B.plx_render_views_status(q)
    assert torch.all(out >= 0.0)


def test_launches_on_two_streams_overlap():
    """Two launches issued on two streams run at the same time: their
    common span is well below the sum of their stand-alone durations (each
    launch holds fewer tiles than the device has workgroup slots)."""
    say("views: two streams overlap")
    grids = [make_pair(synth.blob_scene((192,) * 3, 16, 0.2, s))[1] for s in (41, 42)]
    table = B.SceneTable(grids)
    reqs = random_requests(2, 2, seed=43, resolutions=((288, 288),))
    reqs[0].scene, reqs[1].scene = 0, 1
    streams = [torch.cuda.Stream(), torch.cuda.Stream()]
    outs = [torch.empty(3 * r.n_pixels, device="cuda") for r in reqs]
    qs = [B.views_queue() for _ in reqs]
    for st in streams:
        st.wait_stream(torch.cuda.current_stream())
    ev = lambda: torch.cuda.Event(enable_timing=True)  # noqa: E731

    def alone(i):
        best = float("inf")
        for _ in range(5):
            a, b = ev(), ev()
            a.record(streams[i])
            B.plx_render_views(table, [_view(reqs[i])], outs[i], qs[i], stream=streams[i])
            b.record(streams[i])
            b.synchronize()
            best = min(best, a.elapsed_time(b))
        return best

    d0, d1 = alone(0), alone(1)
    spans = []
    for _ in range(5):
        torch.cuda.synchronize()
        start, e0, e1 = ev(), ev(), ev()
        main = torch.cuda.current_stream()
        start.record(main)
        for i, st in enumerate(streams):
            st.wait_event(start)
            B.plx_render_views(table, [_view(reqs[i])], outs[i], qs[i], stream=st)
        e0.record(streams[0])
        e1.record(streams[1])
        torch.cuda.synchronize()
        spans.append(max(start.elapsed_time(e0), start.elapsed_time(e1)))
    span = min(spans)
    say(f"  alone {d0:.3f} + {d1:.3f} ms, together {span:.3f} ms")
    assert span < 0.8 * (d0 + d1), (span, d0, d1)


def test_long_view_lists_span_launches():
    """More views than one launch takes (24 as kernel arguments): the list is
    split over launches, and every view equals its stand-alone render."""
    say("views: 30 views in one call")
    _, grids = _scenes()
    reqs = random_requests(30, 2, seed=51, resolutions=((24, 20), (40, 32), (17, 9)))
    alone = [_render(grids, [r])[0] for r in reqs]
    together = _render(grids, reqs)
    for a, t in zip(alone, together):
        assert torch.equal(a, t)


def test_scene_table_of_many_scenes():
    """A table of more scenes than one set-up launch writes (24): views of the
    last scenes equal their renders from a table of that scene alone."""
    say("views: 30-scene table")
    grids = [make_pair(synth.blob_scene((20, 18, 22), n_blobs=2, occupancy=0.2, seed=60 + i))[1]
             for i in range(30)]
    table = B.SceneTable(grids)
    reqs = random_requests(6, 30, seed=61, resolutions=((24, 16),))
    for k, r in enumerate(reqs):
        r.scene = 24 + k  # scenes written by the second set-up launch
    together = _render(grids, reqs)
    for r, img in zip(reqs, together):
        alone = _render([grids[r.scene]], [Request(0, r.c2w, r.focal, r.width, r.height)])[0]
        assert torch.equal(img, alone)
