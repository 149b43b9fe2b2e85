"""GPU tests of novel-view serving: plx_render_views against the FP64 oracle
(camera rays from the same pinhole definition, rendered by the oracle), a
view rendered alone versus inside mixed batches (bitwise equal: a pixel's
colour depends only on its own ray and scene), and the continuous-batching
server (every result equal to its stand-alone render, admission within the
HBM budget)."""
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
    ws = torch.empty(B.plx_render_views_workspace(len(grids), len(views)), dtype=torch.uint8,
                     device="cuda")
    B.plx_render_views([g.desc() for g in grids], views, out, ws)
    torch.cuda.synchronize()
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
