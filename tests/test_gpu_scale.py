"""GPU parity at the sizes the benchmark and the configurations run, through
the C ABI, against the FP64 oracle.

- The fused training call on the benchmark's own launch: the whole 1M-ray
  batch on the 512^3 grid at 5% occupancy (Sec. 3.1-3.3, Eq. (1); MSE of
  Sec. 3.5), every ray's colour and every voxel's gradient compared, the
  touched set bit for bit.
- A 5000-ray training step (fused render + MSE + backward, TV on a 1%
  segment, RMSProp) on the 256^3 grid that 64^3 -> prune (sigma < 5) ->
  upsample produces (coarse-to-fine, Sec. 3.4).
- BF16 and FP16 SH storage on the 512^3 scene: sampled rays of the full
  batch against the oracle fed the same rounded coefficients (kernel
  parity) and against the FP32 originals (storage precision, stated per
  pixel), and a training call's gradient on a sampled sub-batch.
- The caller-owned segment lists and the trainer that bins the next batch
  on a second stream.

Tolerances as in tests/gpu_util.py; inputs from the seeded generators in
synth/, expected values from the oracle."""
import math

import numpy as np
import pytest
import torch

import synth
from oracle import oracle as O
from paper_2112_05131_amd import binding as B
from paper_2112_05131_amd.grid import Grid
from paper_2112_05131_amd.train import RaySampler, TrainConfig, Trainer
from tests.gpu_util import (RGB_ATOL, assert_grads_close, assert_touched_equal, grad_mass, make_pair,
                            rounded_sh, say, split_records)

pytestmark = pytest.mark.gpu

# per-pixel budget of 16-bit SH storage against the FP32 coefficients
STORAGE_ATOL = 2e-3


def _np(t):
    return t.detach().cpu().numpy()


@pytest.mark.timeout(900)
def test_c3_full_batch_train_matches_oracle(c3_scene):
    """plx_render_train on the whole 1M-ray batch of the benchmark's
    workload: a grid part-way through training (the ground-truth occupancy,
    perturbed values) against oracle renders of the ground truth."""
    sv, _, og_gt, o, d = c3_scene
    n = o.shape[0]
    on, dn = _np(o), _np(d)
    say("c3 full batch: oracle targets")
    target = O.render_fwd(og_gt, on, dn)[0].astype(np.float32)
    pert = synth.perturbed(sv, seed=1002, device="cuda")
    og, gg = make_pair(pert)
    m = gg.n_vox
    grad = torch.zeros(m, 32, device="cuda")
    touched = torch.zeros(m, dtype=torch.uint8, device="cuda")
    loss = torch.zeros(1, dtype=torch.float64, device="cuda")
    rgb = torch.empty(n, 3, device="cuda")
    desc = gg.desc()
    bins = B.make_bins(desc, o, d)
    say(f"c3 full batch: {n} rays, {bins.n_seg} segments")
    B.plx_render_train(desc, o, d, torch.from_numpy(target).cuda(), 1.0 / n, grad, touched, loss, rgb,
                       bins=bins)
    torch.cuda.synchronize()
    B.plx_bins_verify(desc, bins)
    say("c3 full batch: oracle forward")
    rgb_ref = O.render_fwd(og, on, dn)[0]
    err = float(np.abs(_np(rgb).astype(np.float64) - rgb_ref).max())
    say(f"  max |rgb - oracle| over {n} rays = {err:.2e}")
    assert err <= RGB_ATOL
    g_rgb, loss_ref = O.mse_grad(rgb_ref, target.astype(np.float64))
    assert abs(loss.item() - loss_ref) <= 1e-5 * loss_ref
    say("c3 full batch: oracle backward")
    gd, gs, t_ref = O.render_bwd(og, on, dn, g_rgb)
    assert_touched_equal(touched, t_ref, "c3 full batch")
    say("c3 full batch: oracle gradient mass")
    mass = grad_mass(og, on, dn, g_rgb, chain_rays=n)
    assert_grads_close(grad, gd, gs, "c3 full batch", mass)
    # each voxel of the grid is crossed by many rays of the batch, the
    # contention regime the benchmark times
    assert int(t_ref.sum()) > 0.9 * m


def _c2_grids():
    """Ground truth (256^3 at 10%, 32 blobs, seed 1) and the training grid
    of the coarse-to-fine schedule: a 64^3 grid of the same blobs, pruned at
    sigma < 5 and upsampled to 256^3, on both sides."""
    gt = synth.blob_scene((256,) * 3, n_blobs=32, occupancy=0.10, seed=1, device="cuda")
    coarse = synth.blob_scene((64,) * 3, n_blobs=32, occupancy=1.0, seed=1)
    og64, gg64 = make_pair(coarse)
    gg_pruned, kept, pruned = gg64.prune(5.0)
    og_pruned, kept_ref, pruned_ref = O.prune(og64, 5.0)
    assert (kept, pruned) == (kept_ref, pruned_ref)
    gg = gg_pruned.upsample((256,) * 3)
    og = O.upsample(og_pruned, (256,) * 3)
    assert gg.n_vox == og.n_vox == kept * 64
    assert np.array_equal(_np(gg.index), og.index)
    # the grid stores FP32 values: the oracle's resampled values, rounded
    og.density = og.density.astype(np.float32).astype(np.float64)
    og.sh = og.sh.astype(np.float32).astype(np.float64)
    return gt, og, gg


def test_c2_step_after_prune_and_upsample():
    """One 5000-ray training step on the upsampled 256^3 grid: fused render
    + MSE + backward, TV (lambda 1e-5 / 1e-3) on a 1% segment, RMSProp at
    the schedule's first learning rates."""
    say("c2 step")
    gt, og, gg = _c2_grids()
    d64, s64 = gg.unpack()
    np.testing.assert_allclose(_np(d64).astype(np.float64), og.density, rtol=2e-7, atol=1e-30)
    og_gt = O.make_grid(np.array(gt.reso, np.int32), _np(gt.mask), _np(gt.density).astype(np.float64),
                        _np(gt.sh).astype(np.float64))
    poses = synth.sphere_poses(100, seed=1)
    o, d, _ = synth.sampled_camera_rays(poses, 800, 800, 5000, seed=11, coherent=True)
    on, dn = o.numpy(), d.numpy()
    target = O.render_fwd(og_gt, on, dn)[0].astype(np.float32)
    n, m = o.shape[0], gg.n_vox
    ncell = 256 ** 3
    start, count = 123457, int(math.ceil(0.01 * ncell))
    lam_s, lam_h, eps_tv = 1e-5, 1e-3, 1e-9
    grad = torch.zeros(m, 32, device="cuda")
    touched = torch.zeros(m, dtype=torch.uint8, device="cuda")
    loss = torch.zeros(1, dtype=torch.float64, device="cuda")
    tvl = torch.zeros(1, dtype=torch.float64, device="cuda")
    rgb = torch.empty(n, 3, device="cuda")
    B.plx_render_train(gg.desc(), o.cuda(), d.cuda(), torch.from_numpy(target).cuda(), 1.0 / n, grad,
                       touched, loss, rgb)
    B.plx_tv_grad(gg.desc(), start, count, lam_s, lam_h, eps_tv, grad, touched, tvl)
    torch.cuda.synchronize()
    rgb_ref = O.render_fwd(og, on, dn)[0]
    assert np.abs(_np(rgb).astype(np.float64) - rgb_ref).max() <= RGB_ATOL
    g_rgb, loss_ref = O.mse_grad(rgb_ref, target.astype(np.float64))
    assert abs(loss.item() - loss_ref) <= 1e-5 * loss_ref
    gd, gs, t1 = O.render_bwd(og, on, dn, g_rgb)
    tvl_ref, td, ts, t2 = O.tv(og, start, count, lam_s, lam_h, eps_tv)
    assert abs(tvl.item() - tvl_ref) <= 1e-5 * tvl_ref
    gd, gs, act = gd + td, gs + ts, (t1 | t2)
    assert_touched_equal(touched, act, "c2 step")
    say(f"  active {int(act.sum())} of {m} voxels")
    md, ms = grad_mass(og, on, dn, g_rgb, chain_rays=n)
    # TV's terms, in FP32 against FP64, enter with the same per-term factor
    # as the rendering terms: their size bounds the accumulation error
    mass = (md + 4e-6 * np.abs(td), ms + 4e-6 * np.abs(ts))
    assert_grads_close(grad, gd, gs, "c2 step", mass)
    beta, eps = 0.95, 1e-8
    lr_s = B.plx_lr_schedule(0, 30, 0.05, 250000, 15000, 0.01)
    lr_h = B.plx_lr_schedule(0, 0.01, 5e-6, 250000)
    vstate = torch.zeros(m, 32, device="cuda")
    B.plx_rmsprop_step(gg.desc(), None, vstate, grad, touched, lr_s, lr_h, beta, eps)
    torch.cuda.synchronize()
    dens, sh = og.density.copy(), og.sh.copy()
    O.rmsprop(act, dens, sh, np.zeros(m), np.zeros((m, 27)), gd.copy(), gs.copy(), lr_s, lr_h, beta, eps)
    pd, ps = split_records(gg.data)
    for name, got, ref, p0, g, lr, mm in (("sigma", pd, dens, og.density, gd, lr_s, mass[0]),
                                          ("sh", ps, sh, og.sh, gs, lr_h, mass[1])):
        gtol = 1e-4 * np.abs(g) + mm
        sens = lr * eps / (math.sqrt(1 - beta) * np.abs(g) + eps) ** 2
        tol = sens * gtol + 4e-7 * np.abs(p0) + 1e-6 * lr
        bad = np.abs(got - ref) > tol
        assert not bad.any(), f"c2 step {name}: {int(bad.sum())} parameters outside tolerance"
    assert torch.all(grad == 0) and torch.all(touched == 0)


@pytest.mark.parametrize("sh_dtype", [B.PLX_BF16, B.PLX_F16])
def test_16bit_storage_at_c4_size(c3_scene, sh_dtype):
    """16-bit SH on the 512^3 scene: the forward over the whole 1M-ray batch
    checked on 1500 sampled rays, and a training call on a 20000-ray
    sub-batch checked in full."""
    sv, _, og32, o, d = c3_scene
    name = "bf16" if sh_dtype == B.PLX_BF16 else "f16"
    say(f"16-bit at c4 size: {name}")
    g16 = Grid.from_mask(sv.mask, sv.reso, sv.density, sv.sh, sh_dtype=sh_dtype)
    og16 = O.make_grid(np.array(sv.reso, np.int32), _np(sv.mask), _np(sv.density).astype(np.float64),
                       rounded_sh(sv.sh, sh_dtype).numpy())
    n = o.shape[0]
    rgb = torch.empty(n, 3, device="cuda")
    B.plx_render_fwd(g16.desc(), o, d, rgb)
    torch.cuda.synchronize()
    sel = np.random.default_rng(84).choice(n, 1500, replace=False)
    so, sd = _np(o)[sel], _np(d)[sel]
    got = _np(rgb)[sel].astype(np.float64)
    ref16 = O.render_fwd(og16, so, sd)[0]
    ref32 = O.render_fwd(og32, so, sd)[0]
    kern = float(np.abs(got - ref16).max())
    store = float(np.abs(got - ref32).max())
    say(f"  {name}: max |rgb - oracle(rounded)| = {kern:.2e}, max |rgb - oracle(FP32)| = {store:.2e}")
    assert kern <= RGB_ATOL
    assert store <= STORAGE_ATOL
    # a training call on a sub-batch, gradient against the oracle fed the
    # rounded coefficients
    sub = torch.from_numpy(np.sort(np.random.default_rng(85).choice(n, 20000, replace=False))).cuda()
    to, td_ = o[sub].contiguous(), d[sub].contiguous()
    ns = to.shape[0]
    tgt = synth.targets_uniform(ns, seed=86)
    grad = torch.zeros(g16.n_vox, 32, device="cuda")
    touched = torch.zeros(g16.n_vox, dtype=torch.uint8, device="cuda")
    loss = torch.zeros(1, dtype=torch.float64, device="cuda")
    rgb_s = torch.empty(ns, 3, device="cuda")
    B.plx_render_train(g16.desc(), to, td_, tgt.cuda(), 1.0 / ns, grad, touched, loss, rgb_s)
    torch.cuda.synchronize()
    ton, tdn = _np(to), _np(td_)
    rgb_ref = O.render_fwd(og16, ton, tdn)[0]
    assert np.abs(_np(rgb_s).astype(np.float64) - rgb_ref).max() <= RGB_ATOL
    g_rgb, loss_ref = O.mse_grad(rgb_ref, tgt.double().numpy())
    assert abs(loss.item() - loss_ref) <= 1e-5 * loss_ref
    gd, gs, t_ref = O.render_bwd(og16, ton, tdn, g_rgb)
    assert_touched_equal(touched, t_ref, f"{name} sub-batch")
    tb = t_ref.astype(bool)
    on_ = torch.from_numpy(tb).cuda()
    md, ms = grad_mass(og16, ton, tdn, g_rgb, chain_rays=ns)
    assert_grads_close(grad[on_], gd[tb], gs[tb], f"{name} sub-batch", (md[tb], ms[tb]))
    assert torch.all(grad[~on_] == 0)


@pytest.mark.parametrize("samples", [True, False])
def test_bins_serve_every_call_and_verify(samples):
    """One set of segment lists serves forward, backward and the fused call
    (the same results as lists made afresh), plx_bins_verify finds every
    segment where the count reserved it, and buffers larger than needed are
    accepted; with and without a sample buffer (recorded backward or the
    replay's own scatter)."""
    say("bins reuse, samples", samples)
    sv = synth.dense_random((37, 29, 41), seed=301, occupancy=0.3, ho_scale=0.2)
    og, gg = make_pair(sv)
    o, d = synth.random_rays(3001, seed=302)
    o, d = o.cuda(), d.cuda()
    n, m = o.shape[0], gg.n_vox
    desc = gg.desc()
    big_r = B.workspace(B.plx_bins_ray_bytes(gg.reso, n) + 4096)
    bins = B.make_bins(desc, o, d, ray_buf=big_r, samples=samples)
    assert bins.ray_buf.data_ptr() == big_r.data_ptr()
    assert (bins.samp_buf is not None) == samples and bins.n_brick > 0 and bins.n_samp >= bins.n_seg
    B.plx_bins_verify(desc, bins)
    rgb1, tau1 = torch.empty(n, 3, device="cuda"), torch.empty(n, device="cuda")
    rgb2, tau2 = torch.empty(n, 3, device="cuda"), torch.empty(n, device="cuda")
    B.plx_render_fwd(desc, o, d, rgb1, tau1, bins=bins)
    B.plx_render_fwd(desc, o, d, rgb2, tau2)
    G = torch.from_numpy(np.random.default_rng(303).normal(size=(n, 3))).float().cuda()
    g1 = torch.zeros(m, 32, device="cuda")
    t1 = torch.zeros(m, dtype=torch.uint8, device="cuda")
    B.plx_render_bwd(desc, o, d, G, tau1, g1, t1, bins=bins)
    tgt = synth.targets_uniform(n, seed=304).cuda()
    g2 = torch.zeros_like(g1)
    t2 = torch.zeros_like(t1)
    loss = torch.zeros(1, dtype=torch.float64, device="cuda")
    B.plx_render_train(desc, o, d, tgt, 1.0 / n, g2, t2, loss, bins=bins)
    torch.cuda.synchronize()
    assert torch.equal(rgb1, rgb2) and torch.equal(tau1, tau2)
    rgb_ref = O.render_fwd(og, _np(o), _np(d))[0]
    assert np.abs(_np(rgb1).astype(np.float64) - rgb_ref).max() <= RGB_ATOL
    gd, gs, t_ref = O.render_bwd(og, _np(o), _np(d), _np(G).astype(np.float64))
    assert_touched_equal(t1, t_ref, "bins bwd")
    assert_grads_close(g1, gd, gs, "bins bwd", grad_mass(og, _np(o), _np(d), _np(G).astype(np.float64)))
    assert_touched_equal(t2, t_ref, "bins train")
    # lists made for other rays are refused
    with pytest.raises(B.PlxError, match="made for"):
        B.plx_render_fwd(desc, o[:100].contiguous(), d[:100].contiguous(), rgb1[:100], bins=bins)


def test_trainer_overlapped_binning_matches_sequential():
    """Trainer.run bins batch t+1 on a second stream while step t runs; the
    losses of every step equal those of the plain loop over the same
    batches (up to the order of FP32 atomics).  Repeated run() calls reuse
    the trainer's two sets of segment-list buffers."""
    say("overlapped trainer")
    gt = synth.blob_scene((48, 48, 48), n_blobs=6, occupancy=0.2, seed=311)
    poses = synth.sphere_poses(8, seed=311)
    o, d = synth.all_camera_rays(poses, 64, 64)
    o, d = o.cuda(), d.cuda()
    g_gt = Grid.from_mask(gt.mask.cuda(), gt.reso, gt.density.cuda(), gt.sh.cuda())
    tgt = torch.empty(o.shape[0], 3, device="cuda")
    B.plx_render_fwd(g_gt.desc(), o, d, tgt)
    init = synth.perturbed(gt, seed=312, device="cuda")
    losses = {}
    for overlap in (False, True):
        g = Grid.from_mask(init.mask, init.reso, init.density, init.sh)
        tr = Trainer(g, TrainConfig(), seed=5)
        sampler = RaySampler(o, d, tgt, 5000, seed=7)
        per_step = []
        for _ in range(6):
            tr.loss_sum.zero_()
            tr.run(sampler, 1, overlap=overlap)
            torch.cuda.synchronize()
            per_step.append(tr.loss_sum.item())
        # the single-step runs all used the first set (ray and segment buffers)
        ptr0 = [x.data_ptr() if x is not None else None for x in tr._run_bufs[0]]
        assert ptr0[0] is not None and ptr0[1] is not None
        tr.loss_sum.zero_()
        tr.run(sampler, 5, overlap=overlap)
        torch.cuda.synchronize()
        per_step.append(tr.loss_sum.item())
        losses[overlap] = per_step
        # batches of one scene differ by a few segments; the buffers' slack holds them
        assert ptr0 == [x.data_ptr() if x is not None else None for x in tr._run_bufs[0]]
        assert tr._run_bufs[1][1] is not None
    say(f"  losses {losses[True]}")
    np.testing.assert_allclose(losses[True], losses[False], rtol=1e-4)
    assert all(x > 0 for x in losses[True])


@pytest.mark.parametrize("sh_dtype", [B.PLX_F32, B.PLX_BF16, B.PLX_F16])
def test_crowded_bricks_recorded_backward(sh_dtype):
    """The recorded backward where one brick holds many segments and long
    ones: 30000 rays through a 13^3 grid (8 bricks) with a step of 0.1 voxel,
    so a brick holds thousands of segments (several groups of 256) and tens
    of thousands of samples (many LDS passes, segments across pass
    boundaries, walked last pass first); with that many segments per brick
    the forward is the sample-parallel one (groups of 512 segments walked
    by one, two or four lanes each, FP32 corners staged in two halves, more
    samples than one chunk).  plx_render_bwd with and without a sample
    buffer against the oracle, and the touched set bit-exact."""
    say("crowded bricks", sh_dtype)
    sv = synth.dense_random((13, 13, 13), seed=331, occupancy=0.6, sigma_lo=0.5, sigma_hi=6.0, ho_scale=0.2)
    og, gg = make_pair(sv, sh_dtype=sh_dtype, step_voxels=0.1)
    o, d = synth.random_rays(30000, seed=332)
    n = o.shape[0]
    oc, dc = o.cuda(), d.cuda()
    G = np.random.default_rng(333).normal(size=(n, 3))
    Gc = torch.from_numpy(G).float().cuda()
    rgb, tau = torch.empty(n, 3, device="cuda"), torch.empty(n, device="cuda")
    desc = gg.desc()
    B.plx_render_fwd(desc, oc, dc, rgb, tau)
    rgb_ref = O.render_fwd(og, o.numpy(), d.numpy())[0]
    assert np.abs(rgb.cpu().double().numpy() - rgb_ref).max() <= RGB_ATOL
    gd, gs, t_ref = O.render_bwd(og, o.numpy(), d.numpy(), G)
    mass = grad_mass(og, o.numpy(), d.numpy(), G)
    for samples in (True, False):
        bins = B.make_bins(desc, oc, dc, samples=samples)
        if samples:
            say(f"  {bins.n_seg} segments in {bins.n_brick} bricks, {bins.n_samp} sample slots")
            assert bins.n_seg > 8 * 256 and bins.n_samp > 8 * 1536
        grad = torch.zeros(gg.n_vox, 32, device="cuda")
        touched = torch.zeros(gg.n_vox, dtype=torch.uint8, device="cuda")
        B.plx_render_bwd(desc, oc, dc, Gc, tau, grad, touched, bins=bins)
        torch.cuda.synchronize()
        assert_touched_equal(touched, t_ref, f"crowded, samples={samples}")
        assert_grads_close(grad, gd, gs, f"crowded, samples={samples}", mass)
