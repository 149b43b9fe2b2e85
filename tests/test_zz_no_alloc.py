"""The training call for callers that cannot allocate
(plx_render_train_static, fixed per-device scratch) against the call with
caller-owned segment lists (plx_render_train) and the FP64 oracle, through
the C ABI: two calls in a row on one device, the second with a smaller batch
on another grid (the scratch keeps the first call's contents, which must not
leak into the second)."""
import numpy as np
import pytest
import torch

import synth
from oracle import oracle as O
from paper_2112_05131_amd import binding as B
from tests.gpu_util import (RGB_ATOL, assert_grads_close, assert_touched_equal, grad_mass, make_pair,
                            say, split_records)

pytestmark = pytest.mark.gpu


def _case(reso, occ, seed, n):
    sv = synth.dense_random(reso, seed=seed, occupancy=occ, ho_scale=0.2)
    og, gg = make_pair(sv)
    o, d = synth.random_rays(n, seed=seed + 1)
    tgt = synth.targets_uniform(n, seed=seed + 2)
    return og, gg, o, d, tgt


def _train(fn, gg, o, d, tgt):
    n, m = o.shape[0], gg.n_vox
    grad = torch.zeros(m, 32, device="cuda")
    touched = torch.zeros(m, dtype=torch.uint8, device="cuda")
    loss = torch.zeros(1, dtype=torch.float64, device="cuda")
    rgb = torch.empty(n, 3, device="cuda")
    fn(gg.desc(), o.cuda(), d.cuda(), tgt.cuda(), 1.0 / n, grad, touched, loss, rgb)
    torch.cuda.synchronize()
    return grad, touched, loss.item(), rgb


def test_static_training_call_matches_binned_call_twice():
    for reso, occ, seed, n in (((64, 56, 72), 0.3, 501, 5000), ((24, 20, 28), 0.6, 511, 700)):
        say("static training call", reso, n)
        og, gg, o, d, tgt = _case(reso, occ, seed, n)
        g1, t1, l1, rgb1 = _train(B.plx_render_train_static, gg, o, d, tgt)
        g2, t2, l2, rgb2 = _train(B.plx_render_train, gg, o, d, tgt)
        # same kernels, same segment order: colours and loss agree; touched
        # sets bit for bit; gradients up to the order of FP32 atomics
        assert (rgb1 - rgb2).abs().max().item() <= 1e-6
        assert abs(l1 - l2) <= 1e-6 * abs(l2)
        assert torch.equal(t1, t2)
        on, dn = o.numpy(), d.numpy()
        rgb_ref = O.render_fwd(og, on, dn)[0]
        assert np.abs(rgb1.cpu().double().numpy() - rgb_ref).max() <= RGB_ATOL
        g_rgb, loss_ref = O.mse_grad(rgb_ref, tgt.double().numpy())
        assert abs(l1 - loss_ref) <= 1e-5 * loss_ref
        gd, gs, t_ref = O.render_bwd(og, on, dn, g_rgb)
        assert_touched_equal(t1, t_ref, "static")
        mass = grad_mass(og, on, dn, g_rgb, chain_rays=n)
        assert_grads_close(g1, gd, gs, "static", mass)
        d1, s1 = split_records(g1)
        d2, s2 = split_records(g2)
        assert_grads_close(g2, d1, s1, "binned vs static", mass)


def test_static_training_call_refuses_oversized_batch():
    og, gg, o, d, tgt = _case((64, 56, 72), 0.3, 521, 10)
    big = torch.zeros(200000, 3)
    with pytest.raises(B.PlxError) as e:
        _train(B.plx_render_train_static, gg, big, big, big)
    assert e.value.code == B.PLX_ENOMEM
