"""Host-side driver logic on the CPU: the epoch-permutation ray sampler
(every ray once per epoch, seeded, coherent batches are the same rays in
storage order), the coherent order of the synthetic batch generator, and the
Morton key."""
import numpy as np
import pytest
import torch

import synth
from paper_2112_05131_amd.train import RaySampler


def _rays(n):
    ids = torch.arange(n, dtype=torch.float32)
    o = torch.stack([ids, ids + 0.5, ids + 0.25], dim=1)
    return o, o * 2.0, o * 3.0


@pytest.mark.parametrize("coherent", [False, True])
def test_sampler_epoch_visits_every_ray_once(coherent):
    n, batch = 1000, 100
    o, d, t = _rays(n)
    s = RaySampler(o, d, t, batch, seed=3, coherent=coherent)
    seen = []
    for _ in range(n // batch):
        bo, bd, bt = s.next_batch()
        assert bo.shape == (batch, 3)
        ids = bo[:, 0].long()
        # the three arrays stay aligned
        assert torch.equal(bd, o[ids] * 2.0) and torch.equal(bt, o[ids] * 3.0)
        if coherent:
            assert torch.all(ids[1:] > ids[:-1])
        seen.append(ids)
    seen = torch.cat(seen)
    assert s.epoch == 0
    assert torch.equal(torch.sort(seen).values, torch.arange(n))
    s.next_batch()
    assert s.epoch == 1


def test_sampler_is_seeded_and_coherent_order_keeps_the_rays():
    n, batch = 777, 64
    o, d, t = _rays(n)
    a = RaySampler(o, d, t, batch, seed=9, coherent=False)
    b = RaySampler(o, d, t, batch, seed=9, coherent=True)
    c = RaySampler(o, d, t, batch, seed=10, coherent=False)
    for _ in range(30):  # crosses epoch boundaries (tails dropped)
        ra, rb, rc = a.next_batch()[0], b.next_batch()[0], c.next_batch()[0]
        assert torch.equal(torch.sort(ra[:, 0]).values, rb[:, 0])
    assert not torch.equal(ra, rc)


def test_sampler_rejects_bad_shapes():
    o, d, t = _rays(10)
    with pytest.raises(ValueError):
        RaySampler(o, d[:5], t, 4)
    with pytest.raises(ValueError):
        RaySampler(o, d, t, 0)


def test_morton_key_interleaves_bits():
    x = torch.tensor([0, 1, 0, 1, 2, 3, 65535])
    y = torch.tensor([0, 0, 1, 1, 0, 3, 65535])
    k = synth.morton2(x, y)
    assert k.tolist() == [0, 1, 2, 3, 4, 15, (1 << 32) - 1]


def test_coherent_batches_hold_the_same_rays():
    poses = synth.sphere_poses(3, seed=4)
    o1, d1, i1 = synth.sampled_camera_rays(poses, 32, 24, 500, seed=5)
    o2, d2, i2 = synth.sampled_camera_rays(poses, 32, 24, 500, seed=5, coherent=True)
    assert torch.equal(torch.sort(i1).values, torch.sort(i2).values)
    cam = i2 // (32 * 24)
    assert torch.all(cam[1:] >= cam[:-1])
    # rays follow their ids
    p1 = torch.argsort(i1, stable=True)
    p2 = torch.argsort(i2, stable=True)
    assert torch.equal(d1[p1], d2[p2]) and torch.equal(o1[p1], o2[p2])


def test_psnr_and_camera_set_order():
    from paper_2112_05131_amd.runs import _camera_set, psnr
    a = torch.zeros(10, 3)
    b = torch.full((10, 3), 0.1)
    assert abs(psnr(a, b) - 20.0) < 1e-6  # 0.1 rounded to float32
    assert psnr(a, a) == float("inf")
    # every pixel of every camera once, each camera's pixels in Morton order
    o, d = _camera_set(2, 8, 4, seed=1, device="cpu")
    o1, d1 = synth.all_camera_rays(synth.sphere_poses(2, seed=1), 8, 4)
    assert o.shape == o1.shape == (64, 3)
    pix = torch.arange(32)
    order = torch.argsort(synth.morton2(pix % 8, pix // 8))
    assert torch.equal(d[:32], d1[order]) and torch.equal(d[32:], d1[32 + order])
