"""GPU parity of the sparsity (Cauchy) and beta priors of Sec. 3.7 against
the FP64 oracle, through the C ABI: plx_render_train, plx_render_bwd and
plx_render_bwd_state with the priors switched on.

Tolerances: the density gradient is the colour gradient plus the priors'
terms, so the per-element bound is the colour-gradient bound of
tests/gpu_util.py plus the same conditioning rule applied to the priors'
terms (4e-6 times their absolute sum, from orc_regularisers, with terms at an
ambiguous density gate counted in full).  SH gradients and the touched set do
not change.  The prior losses: L_s within 1e-4 relative (per-lane FP32 sums
of up to a few hundred log terms), L_b within 1e-6 relative (FP64 per ray
from the FP32 optical depth).  Inputs come from the seeded generators in
synth/, expected values from the oracle."""
import numpy as np
import pytest
import torch

import synth
from oracle import oracle as O
from paper_2112_05131_amd import binding as B
from tests.gpu_util import (GATE_REL, GRAD_MASS, assert_grads_close, assert_touched_equal, grad_mass, make_pair,
                            say)

pytestmark = pytest.mark.gpu

LS, LB, EPS = 0.02, 0.05, 1e-3


def prior_mass(og, o, d, lam_s, lam_b, eps):
    _, _, _, plain = O.regularisers(og, o, d, lam_s, lam_b, eps, gate_rel=0.0)
    _, _, _, amb = O.regularisers(og, o, d, lam_s, lam_b, eps, gate_rel=GATE_REL)
    return GRAD_MASS * plain + (amb - plain)


def scene(seed, reso=(27, 22, 30), occ=0.45):
    sv = synth.dense_random(reso, seed=seed, occupancy=occ, sigma_lo=-5.0, sigma_hi=40.0, ho_scale=0.3)
    return make_pair(sv)


def check_losses(loss, ls_ref, lb_ref):
    got = loss.cpu().numpy()
    say("  prior losses", got.tolist(), "ref", ls_ref, lb_ref)
    assert abs(got[0] - ls_ref) <= 1e-4 * abs(ls_ref) + 1e-12
    assert abs(got[1] - lb_ref) <= 1e-6 * abs(lb_ref) + 1e-9


@pytest.mark.parametrize("samples", [True, False])
@pytest.mark.parametrize("sh_dtype", [B.PLX_F32, B.PLX_F16])
def test_train_with_priors_matches_oracle(sh_dtype, samples):
    say("train + priors", sh_dtype, "samples", samples)
    og, gg = make_pair(synth.dense_random((27, 22, 30), seed=81, occupancy=0.45, sigma_lo=-5.0, sigma_hi=40.0,
                                          ho_scale=0.3), sh_dtype)
    o, d = synth.random_rays(3001, seed=82)
    n = o.shape[0]
    on, dn = o.numpy(), d.numpy()
    target = np.random.default_rng(83).uniform(0.0, 1.0, (n, 3)).astype(np.float32)
    grad = torch.zeros(gg.n_vox, 32, device="cuda")
    touched = torch.zeros(gg.n_vox, dtype=torch.uint8, device="cuda")
    loss = torch.zeros(1, dtype=torch.float64, device="cuda")
    pl = torch.zeros(2, dtype=torch.float64, device="cuda")
    bins = B.make_bins(gg.desc(), o.cuda(), d.cuda(), samples=samples)
    B.plx_render_train(gg.desc(), o.cuda(), d.cuda(), torch.from_numpy(target).cuda(), 1.0 / n, grad, touched,
                       loss, priors=B.Priors(LS, LB, EPS, pl), bins=bins)
    torch.cuda.synchronize()
    rgb_ref = O.render_fwd(og, on, dn)[0]
    g_rgb, loss_ref = O.mse_grad(rgb_ref, target)
    gd, gs, t_ref = O.render_bwd(og, on, dn, g_rgb)
    ls_ref, lb_ref, gd_p, _ = O.regularisers(og, on, dn, LS, LB, EPS)
    assert abs(loss.item() - loss_ref) <= 1e-5 * loss_ref
    check_losses(pl, ls_ref, lb_ref)
    assert_touched_equal(touched, t_ref, "train + priors")
    md, ms = grad_mass(og, on, dn, g_rgb, chain_rays=n)
    assert_grads_close(grad, gd + gd_p, gs, "train + priors", (md + prior_mass(og, on, dn, LS, LB, EPS), ms))
    # the priors change the density gradient noticeably here
    assert np.abs(gd_p).max() > 0.1 * np.abs(gd).max()


@pytest.mark.parametrize("lam_s,lam_b", [(LS, 0.0), (0.0, LB), (LS, LB)])
def test_bwd_with_priors_matches_oracle(lam_s, lam_b):
    say("bwd + priors", lam_s, lam_b)
    og, gg = scene(84)
    o, d = synth.random_rays(2500, seed=85)
    n = o.shape[0]
    on, dn = o.numpy(), d.numpy()
    bg = (0.2, 0.7, 0.4)
    G = torch.from_numpy(np.random.default_rng(86).normal(size=(n, 3)) * 1e-3).float()
    rgb = torch.empty(n, 3, device="cuda")
    tau = torch.empty(n, device="cuda")
    B.plx_render_fwd(gg.desc(), o.cuda(), d.cuda(), rgb, tau, bg)
    grad = torch.zeros(gg.n_vox, 32, device="cuda")
    touched = torch.zeros(gg.n_vox, dtype=torch.uint8, device="cuda")
    pl = torch.zeros(2, dtype=torch.float64, device="cuda")
    B.plx_render_bwd(gg.desc(), o.cuda(), d.cuda(), G.cuda(), tau, grad, touched, bg,
                     priors=B.Priors(lam_s, lam_b, EPS, pl))
    torch.cuda.synchronize()
    Gd = G.double().numpy()
    gd, gs, t_ref = O.render_bwd(og, on, dn, Gd, bg)
    ls_ref, lb_ref, gd_p, _ = O.regularisers(og, on, dn, lam_s, lam_b, EPS)
    check_losses(pl, ls_ref, lb_ref)
    assert_touched_equal(touched, t_ref, "bwd + priors")
    md, ms = grad_mass(og, on, dn, Gd, bg)
    assert_grads_close(grad, gd + gd_p, gs, "bwd + priors", (md + prior_mass(og, on, dn, lam_s, lam_b, EPS), ms))


@pytest.mark.parametrize("cap", [4096, 0])
def test_bwd_state_with_priors_matches_oracle(cap):
    say("bwd state + priors", cap)
    og, gg = scene(87)
    o, d = synth.random_rays(2000, seed=88)
    n = o.shape[0]
    on, dn = o.numpy(), d.numpy()
    G = torch.from_numpy(np.random.default_rng(89).normal(size=(n, 3)) * 1e-3).float()
    rgb = torch.empty(n, 3, device="cuda")
    tau = torch.empty(n, device="cuda")
    state = torch.empty(B.plx_render_state_bytes(n, cap), dtype=torch.uint8, device="cuda")
    B.plx_render_fwd_state(gg.desc(), o.cuda(), d.cuda(), rgb, tau, state, cap)
    grad = torch.zeros(gg.n_vox, 32, device="cuda")
    touched = torch.zeros(gg.n_vox, dtype=torch.uint8, device="cuda")
    pl = torch.zeros(2, dtype=torch.float64, device="cuda")
    B.plx_render_bwd_state(gg.desc(), o.cuda(), d.cuda(), G.cuda(), tau, state, cap, grad, touched,
                           priors=B.Priors(LS, LB, EPS, pl))
    torch.cuda.synchronize()
    Gd = G.double().numpy()
    gd, gs, t_ref = O.render_bwd(og, on, dn, Gd)
    ls_ref, lb_ref, gd_p, _ = O.regularisers(og, on, dn, LS, LB, EPS)
    check_losses(pl, ls_ref, lb_ref)
    assert_touched_equal(touched, t_ref, "bwd state + priors")
    md, ms = grad_mass(og, on, dn, Gd)
    assert_grads_close(grad, gd + gd_p, gs, "bwd state + priors", (md + prior_mass(og, on, dn, LS, LB, EPS), ms))


def test_priors_validation_and_zero_weights():
    say("priors validation")
    og, gg = scene(90, reso=(9, 8, 10))
    o, d = synth.random_rays(300, seed=91)
    n = o.shape[0]
    G = torch.zeros(n, 3, device="cuda")
    tau = torch.zeros(n, device="cuda")
    grad = torch.zeros(gg.n_vox, 32, device="cuda")
    touched = torch.zeros(gg.n_vox, dtype=torch.uint8, device="cuda")
    for bad in (B.Priors(0.0, 1.0, 0.0), B.Priors(0.0, 1.0, -1.0), B.Priors(float("nan"), 0.0, 1e-3),
                B.Priors(0.0, float("inf"), 1e-3)):
        with pytest.raises(B.PlxError):
            B.plx_render_bwd(gg.desc(), o.cuda(), d.cuda(), G, tau, grad, touched, priors=bad)
    # zero weights: no prior gradient and no loss; with dL/dC = 0 nothing at all
    pl = torch.zeros(2, dtype=torch.float64, device="cuda")
    B.plx_render_fwd(gg.desc(), o.cuda(), d.cuda(), torch.empty(n, 3, device="cuda"), tau)
    B.plx_render_bwd(gg.desc(), o.cuda(), d.cuda(), G, tau, grad, touched, priors=B.Priors(0.0, 0.0, 0.0, pl))
    torch.cuda.synchronize()
    assert torch.all(grad == 0) and torch.all(pl == 0) and int(touched.sum()) > 0
