"""GPU parity of the MSI background of 360-degree scenes (Sec. 3.6) against
the FP64 oracle, through the C ABI: the background colour of each ray and
its gradient, the foreground calls with per-ray background colours and the
background gradient they hand back, and a full training step of both
models.  Tolerances: colours 1e-5 absolute per channel (the RGB bound);
gradients the mass rule of tests/gpu_util.py for both models (for the
background from orc_bg_render_bwd's absolute-term mode), plus, in the chained
step, the terms of the error bounds of the quantities passed between the
two models (the background colours and their gradient); touched sets bit
for bit.  Inputs come from the seeded generators in synth/, expected values
from the oracle."""
import numpy as np
import pytest
import torch

import synth
from oracle import oracle as O
from paper_2112_05131_amd import binding as B
from paper_2112_05131_amd.grid import Grid
from tests.gpu_util import (GATE_REL, GRAD_MASS, RGB_ATOL, assert_grads_close, assert_touched_equal, grad_mass,
                            make_pair, say)

pytestmark = pytest.mark.gpu


def bg_pair(reso, seed, occupancy=0.7, sigma_hi=4.0):
    """(oracle background grid, GPU grid) with random opacities and
    degree-0 colour coefficients (some negative)."""
    n = int(np.prod(reso))
    g = torch.Generator().manual_seed(seed)
    mask = (torch.rand(n, generator=g, dtype=torch.float64) < occupancy).to(torch.uint8)
    m = int(mask.sum())
    dens = (torch.rand(m, generator=g, dtype=torch.float64) * sigma_hi).float()
    coef = (torch.rand(m, 3, generator=g, dtype=torch.float64) * 4.0 - 1.0).float()
    sh = torch.zeros(m, 27)
    sh[:, 24:27] = coef
    og = O.bg_grid(reso, mask.numpy(), dens.double().numpy(), coef.double().numpy())
    gg = Grid.from_mask(mask.cuda(), reso, dens.cuda(), sh.cuda())
    return og, gg


def test_background_empty_inputs():
    """Zero rays write nothing (background passes, NDC warp); a zero-cell
    background TV adds nothing; a background with no stored voxel renders
    the constant colour with transmittance 1 and writes no gradient (NULL
    gradient buffers)."""
    say("bg empty")
    reso = (6, 8, 10)
    _, gg = bg_pair(reso, 131)
    bgc = (0.1, 0.2, 0.3)
    z = torch.zeros(0, 3, device="cuda")
    out = torch.full((1, 3), 7.0, device="cuda")
    grad = torch.zeros(gg.n_vox, 32, device="cuda")
    touched = torch.zeros(gg.n_vox, dtype=torch.uint8, device="cuda")
    loss = torch.zeros(1, dtype=torch.float64, device="cuda")
    B.plx_bg_render_fwd(gg.desc(), z, z, out[:0], None, bgc)
    B.plx_bg_render_bwd(gg.desc(), z, z, z, grad, touched, bgc)
    B.plx_rays_to_ndc(z, z, 64, 48, 50.0, 1.0, z, z)
    B.plx_bg_tv_grad(gg.desc(), 0, 0, 1e-3, 1e-3, 1e-9, grad, touched, loss)
    torch.cuda.synchronize()
    assert torch.all(out == 7.0) and loss.item() == 0.0
    assert not torch.any(grad != 0) and not torch.any(touched != 0)
    empty = Grid.from_mask(torch.zeros(int(np.prod(reso)), dtype=torch.uint8, device="cuda"), reso)
    assert empty.n_vox == 0
    o, d = bg_rays(200, 132)
    n = o.shape[0]
    rgb = torch.empty(n, 3, device="cuda")
    t = torch.empty(n, device="cuda")
    B.plx_bg_render_fwd(empty.desc(), o.cuda(), d.cuda(), rgb, t, bgc)
    B.plx_bg_render_bwd(empty.desc(), o.cuda(), d.cuda(), torch.ones(n, 3, device="cuda"),
                        torch.zeros(0, 32, device="cuda"), torch.zeros(0, dtype=torch.uint8, device="cuda"), bgc)
    torch.cuda.synchronize()
    assert torch.all(rgb.cpu() == torch.tensor([bgc] * n)) and torch.all(t == 1.0)


def bg_mass(og, o, d, gabs, bg, extra_gabs=None):
    """Tolerance mass of the background gradient, by the rule of grad_mass:
    GRAD_MASS times the absolute-term sums for |dL/dC_bg|, terms at
    ambiguous gates in full, plus (extra_gabs) the full terms of a bound on
    the error of dL/dC_bg itself."""
    pd, ps = O.bg_render_bwd_mass(og, o, d, gabs, bg)
    ad, as_ = O.bg_render_bwd_mass(og, o, d, gabs, bg, gate_rel=GATE_REL)
    md, ms = GRAD_MASS * pd + (ad - pd), GRAD_MASS * ps + (as_ - ps)
    if extra_gabs is not None:
        ed, es = O.bg_render_bwd_mass(og, o, d, extra_gabs, bg, gate_rel=GATE_REL)
        md, ms = md + ed, ms + es
    return md, ms


def bg_rays(n, seed):
    """Rays from inside the unit sphere, a few from outside it, and the axis
    and pole directions from the centre."""
    o, d = synth.random_rays(n, seed=seed, radius=0.7, target_half=0.4)
    o2, d2 = synth.random_rays(16, seed=seed + 1, radius=1.4, target_half=0.3)
    ax = torch.tensor([[1.0, 0, 0], [0, 1.0, 0], [-1.0, 0, 0], [0, -1.0, 0], [0, 0, 1.0], [0, 0, -1.0]])
    return torch.cat([o, o2, torch.zeros(6, 3)]), torch.cat([d, d2, ax])


@pytest.mark.parametrize("reso,seed", [((8, 16, 32), 121), ((5, 7, 9), 122), ((80, 6, 10), 123)])
def test_bg_forward_backward_match_oracle(reso, seed):
    """(80, 6, 10): 158 samples per ray, more than one 128-sample round of
    the wave-per-ray kernels."""
    say("bg fwd/bwd", reso)
    og, gg = bg_pair(reso, seed)
    o, d = bg_rays(1500, seed + 10)
    n = o.shape[0]
    bgc = (0.2, 0.6, 0.9)
    rgb = torch.empty(n, 3, device="cuda")
    t = torch.empty(n, device="cuda")
    B.plx_bg_render_fwd(gg.desc(), o.cuda(), d.cuda(), rgb, t, bgc)
    G = torch.from_numpy(np.random.default_rng(seed).normal(size=(n, 3))).float()
    grad = torch.zeros(gg.n_vox, 32, device="cuda")
    touched = torch.zeros(gg.n_vox, dtype=torch.uint8, device="cuda")
    B.plx_bg_render_bwd(gg.desc(), o.cuda(), d.cuda(), G.cuda(), grad, touched, bgc)
    torch.cuda.synchronize()
    rgb_ref, t_ref = O.bg_render_fwd(og, o.numpy(), d.numpy(), bgc)
    assert np.abs(rgb.cpu().double().numpy() - rgb_ref).max() <= RGB_ATOL
    assert np.abs(t.cpu().double().numpy() - t_ref).max() <= RGB_ATOL
    gd, gs, t_touch = O.bg_render_bwd(og, o.numpy(), d.numpy(), G.double().numpy(), bgc)
    assert_touched_equal(touched, t_touch, "bg bwd")
    assert_grads_close(grad, gd, gs, "bg bwd", bg_mass(og, o.numpy(), d.numpy(), G.double().numpy(), bgc))
    # only the density and the three colour slots are written
    used = [24, 25, 26, 28]
    rest = [q for q in range(32) if q not in used]
    assert torch.all(grad[:, rest] == 0)


def test_foreground_with_per_ray_background_matches_oracle():
    say("fg + per-ray background")
    sv = synth.dense_random((21, 19, 23), seed=123, occupancy=0.5, sigma_lo=0.0, sigma_hi=20.0, ho_scale=0.3)
    og, gg = make_pair(sv)
    o, d = synth.random_rays(2500, seed=124)
    n = o.shape[0]
    bg = np.random.default_rng(125).uniform(0.0, 1.0, (n, 3)).astype(np.float32)
    bgt = torch.from_numpy(bg).cuda()
    rgb = torch.empty(n, 3, device="cuda")
    tau = torch.empty(n, device="cuda")
    B.plx_render_fwd(gg.desc(), o.cuda(), d.cuda(), rgb, tau, bgt)
    G = torch.from_numpy(np.random.default_rng(126).normal(size=(n, 3))).float()
    grad = torch.zeros(gg.n_vox, 32, device="cuda")
    touched = torch.zeros(gg.n_vox, dtype=torch.uint8, device="cuda")
    gbg = torch.full((n, 3), 7.0, device="cuda")
    B.plx_render_bwd(gg.desc(), o.cuda(), d.cuda(), G.cuda(), tau, grad, touched, bgt, grad_bg=gbg)
    torch.cuda.synchronize()
    bgd = bg.astype(np.float64)
    rgb_ref, _, tf, _ = O.render_fwd(og, o.numpy(), d.numpy(), bgd)
    assert np.abs(rgb.cpu().double().numpy() - rgb_ref).max() <= RGB_ATOL
    Gd = G.double().numpy()
    gd, gs, t_ref = O.render_bwd(og, o.numpy(), d.numpy(), Gd, bgd)
    assert_touched_equal(touched, t_ref, "fg per-ray bg")
    assert_grads_close(grad, gd, gs, "fg per-ray bg", grad_mass(og, o.numpy(), d.numpy(), Gd, bgd))
    # dL/d(background) = T_final dL/dC
    np.testing.assert_allclose(gbg.cpu().double().numpy(), tf[:, None] * Gd, rtol=2e-5, atol=1e-7)
    # the stored-state backward hands back the same
    state = torch.empty(B.plx_render_state_bytes(n, 64), dtype=torch.uint8, device="cuda")
    B.plx_render_fwd_state(gg.desc(), o.cuda(), d.cuda(), rgb, tau, state, 64, bgt)
    gbg2 = torch.zeros(n, 3, device="cuda")
    grad2 = torch.zeros_like(grad)
    B.plx_render_bwd_state(gg.desc(), o.cuda(), d.cuda(), G.cuda(), tau, state, 64, grad2, touched, bgt,
                           grad_bg=gbg2)
    torch.cuda.synchronize()
    assert np.abs(rgb.cpu().double().numpy() - rgb_ref).max() <= RGB_ATOL
    np.testing.assert_allclose(gbg2.cpu().double().numpy(), tf[:, None] * Gd, rtol=2e-5, atol=1e-7)
    assert_grads_close(grad2, gd, gs, "fg per-ray bg, stored state", grad_mass(og, o.numpy(), d.numpy(), Gd, bgd))


def test_training_step_foreground_and_background_matches_oracle():
    say("360 step")
    sv = synth.dense_random((17, 17, 17), seed=127, occupancy=0.4, sigma_lo=0.0, sigma_hi=15.0, ho_scale=0.3)
    og, gg = make_pair(sv)
    obg, gbgrid = bg_pair((6, 12, 24), 128)
    o, d = synth.random_rays(3000, seed=129, radius=0.9, target_half=0.45)
    n = o.shape[0]
    target = np.random.default_rng(130).uniform(0.0, 1.0, (n, 3)).astype(np.float32)
    bgc = (0.0, 0.0, 0.0)
    # device: background colours, fused foreground step, background gradient
    cbg = torch.empty(n, 3, device="cuda")
    B.plx_bg_render_fwd(gbgrid.desc(), o.cuda(), d.cuda(), cbg, None, bgc)
    grad = torch.zeros(gg.n_vox, 32, device="cuda")
    touched = torch.zeros(gg.n_vox, dtype=torch.uint8, device="cuda")
    loss = torch.zeros(1, dtype=torch.float64, device="cuda")
    rgb = torch.empty(n, 3, device="cuda")
    gbg = torch.empty(n, 3, device="cuda")
    B.plx_render_train(gg.desc(), o.cuda(), d.cuda(), torch.from_numpy(target).cuda(), 1.0 / n, grad, touched,
                       loss, rgb, cbg, grad_bg=gbg)
    bgrad = torch.zeros(gbgrid.n_vox, 32, device="cuda")
    btouched = torch.zeros(gbgrid.n_vox, dtype=torch.uint8, device="cuda")
    B.plx_bg_render_bwd(gbgrid.desc(), o.cuda(), d.cuda(), gbg, bgrad, btouched, bgc)
    torch.cuda.synchronize()
    # oracle: the same chain
    on, dn = o.numpy(), d.numpy()
    cbg_ref, _ = O.bg_render_fwd(obg, on, dn, bgc)
    assert np.abs(cbg.cpu().double().numpy() - cbg_ref).max() <= RGB_ATOL
    rgb_ref, _, tf, _ = O.render_fwd(og, on, dn, cbg_ref)
    # the foreground kernel against the oracle fed the device's background
    # colours: within the RGB tolerance; end to end, the two stages' bounds add
    rgb_dev_bg = O.render_fwd(og, on, dn, cbg.cpu().double().numpy())[0]
    assert np.abs(rgb.cpu().double().numpy() - rgb_dev_bg).max() <= RGB_ATOL
    assert np.abs(rgb.cpu().double().numpy() - rgb_ref).max() <= 2 * RGB_ATOL
    g_rgb, loss_ref = O.mse_grad(rgb_ref, target)
    assert abs(loss.item() - loss_ref) <= 1e-5 * loss_ref
    gd, gs, t_ref = O.render_bwd(og, on, dn, g_rgb, cbg_ref)
    assert_touched_equal(touched, t_ref, "360 fg")
    md, ms = grad_mass(og, on, dn, g_rgb, cbg_ref, chain_rays=n)
    # the device's background colours (within RGB_ATOL of the oracle's) enter
    # every density term through R_k: add the terms' mass for |bg| = RGB_ATOL
    # (the same walk with all colours 0 and a unit background)
    black = O.Grid(og.reso, og.scale, og.offset, og.step, og.index, og.density, np.zeros_like(og.sh))
    bd, _ = O.render_bwd_mass(black, on, dn, np.abs(g_rgb), (1.0, 1.0, 1.0), gate_rel=GATE_REL)
    assert_grads_close(grad, gd, gs, "360 fg", (md + RGB_ATOL * bd, ms))
    gbg_ref = tf[:, None] * g_rgb
    # dL/dC carries the colours' FP32 error (<= 2 RGB_ATOL per channel) times 2/R
    gerr = 4 * RGB_ATOL / n + 1e-5 * np.abs(gbg_ref)
    assert np.all(np.abs(gbg.cpu().double().numpy() - gbg_ref) <= gerr)
    bgd, bgs, bt_ref = O.bg_render_bwd(obg, on, dn, gbg_ref, bgc)
    assert_touched_equal(btouched, bt_ref, "360 bg")
    assert_grads_close(bgrad, bgd, bgs, "360 bg", bg_mass(obg, on, dn, gbg_ref, bgc, extra_gabs=gerr))
    assert bt_ref.sum() > 100 and t_ref.sum() > 100


@pytest.mark.parametrize("start,count", [(0, 6 * 12 * 24), (1500, 900)])
def test_bg_tv_matches_oracle(start, count):
    say("bg tv", start, count)
    og, gg = bg_pair((6, 12, 24), 134, occupancy=0.8)
    grad = torch.zeros(gg.n_vox, 32, device="cuda")
    touched = torch.zeros(gg.n_vox, dtype=torch.uint8, device="cuda")
    loss = torch.zeros(1, dtype=torch.float64, device="cuda")
    B.plx_bg_tv_grad(gg.desc(), start, count, 0.9, 1.3, 1e-9, grad, touched, loss)
    torch.cuda.synchronize()
    l_ref, gd, gs, t_ref = O.bg_tv(og, start, count, 0.9, 1.3, 1e-9)
    assert abs(loss.item() - l_ref) <= 1e-5 * abs(l_ref)
    assert_touched_equal(touched, t_ref, "bg tv")
    assert_grads_close(grad, gd, gs, "bg tv")
    assert torch.all(grad[:, :24] == 0) and torch.all(grad[:, 29:] == 0)


def test_bg_full_size_sampled():
    """The paper's background size, 64 spheres of 1024 x 2048 (10% of the
    voxels stored), 1M rays from inside the unit sphere; 1000 of them
    checked against the oracle."""
    say("bg full size")
    reso = (64, 1024, 2048)
    og, gg = bg_pair(reso, 131, occupancy=0.1)
    o, d = synth.random_rays(1 << 20, seed=132, radius=0.8, target_half=0.45)
    n = o.shape[0]
    rgb = torch.empty(n, 3, device="cuda")
    B.plx_bg_render_fwd(gg.desc(), o.cuda(), d.cuda(), rgb, None, (1.0, 1.0, 1.0))
    torch.cuda.synchronize()
    sel = np.random.default_rng(133).choice(n, 1000, replace=False)
    ref, _ = O.bg_render_fwd(og, o[sel].numpy(), d[sel].numpy(), (1.0, 1.0, 1.0))
    assert np.abs(rgb[sel].cpu().double().numpy() - ref).max() <= RGB_ATOL
