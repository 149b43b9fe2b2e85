"""Multi-step training runs on the seeded synthetic scenes.

coarse_to_fine: the coarse-to-fine schedule of Sec. 3.6 / supplement B.1 at
  the 256^3 sparse-scene size: a dense 64^3 grid with the uniform init is
  trained on 5000-ray batches drawn from all pixels of 100 cameras, pruned
  (with dilation) by density or by the maximum sample weight over all the
  training rays (Sec. 3.4), upsampled to 256^3 and trained further.  Reports
  the time per step of each stage, the prune/upsample times (and the weight
  pass's time and ray rate) and voxel counts, and the held-out PSNR after
  each stage.

precision_drift: the same training (same init, same batch sequence) with the
  SH coefficients stored as FP32, BF16 and FP16 (FP32 density, master
  records, optimiser state and accumulation in all three) on the 512^3 / 5%
  scene with 1M-ray batches; reports, after the given number of steps, the
  held-out PSNR of each grid against the ground truth and the per-pixel
  difference of the 16-bit runs from the FP32 run.

forward_facing: forward-facing capture in NDC space (Sec. 3.6; the
  forward-facing experiments of supplement B.1): a blob scene over the NDC
  cube at 512x512x128 seen by 20 forward-facing cameras at 1008x756, their
  rays warped to NDC on the device; a dense 256x256x128 grid with the uniform
  init is trained with TV throughout (5e-4 / 5e-3) and the sparsity prior
  (1e-12), pruned at density 1 (densities here are per NDC unit; the
  paper's threshold of 5 belongs to its units and removes the visible blob
  fringes of these scenes), upsampled to 512x512x128, trained further,
  and finally upsampled to the experiments' 1408x1156x128 grid, where 5000-
  and 1M-ray steps are timed.  Reports times, voxel counts and held-out PSNR.

unbounded_360: a 360-degree scene (Sec. 3.6): a 256^3 blob scene inside the
  unit sphere in front of a procedural sky on a 64 x 256 x 512 MSI
  background, seen by 64 inward-looking cameras at radius 0.8 (640x360); a
  dense 128^3 foreground and a dense background are trained jointly (the
  paper's 360-degree TV, sparsity and beta weights), the foreground pruned
  by weight over all training rays and upsampled to 256^3 and trained
  further; then 1M-ray steps are timed
  with the background at the paper's 64 x 1024 x 2048.  Reports times,
  voxel counts and held-out PSNR.

Host code only chooses the schedule; every step is the library's fused
render/MSE/backward, TV and sparse RMSProp.

    python -m paper_2112_05131_amd.runs coarse_to_fine [--prune weight --prune-thresh 0.256]
    python -m paper_2112_05131_amd.runs drift --steps 2000
    python -m paper_2112_05131_amd.runs forward_facing --steps 300 [--prune-thresh 1]
    python -m paper_2112_05131_amd.runs unbounded_360 --steps 300
"""
from __future__ import annotations

import argparse
import json
import math
import sys
import time

import numpy as np
import torch

import synth

from . import binding as B
from .grid import Grid
from .train import RaySampler, TrainConfig, Trainer


def render_rays(grid: Grid, o: torch.Tensor, d: torch.Tensor, bg=(1.0, 1.0, 1.0),
                chunk: int = 1 << 22) -> torch.Tensor:
    out = torch.empty(o.shape[0], 3, dtype=torch.float32, device=o.device)
    for s in range(0, o.shape[0], chunk):
        B.plx_render_fwd(grid.desc(), o[s:s + chunk], d[s:s + chunk], out[s:s + chunk], None, bg)
    return out


def psnr(a: torch.Tensor, b: torch.Tensor) -> float:
    mse = torch.mean((a.double() - b.double()) ** 2).item()
    return float("inf") if mse == 0 else -10.0 * math.log10(mse)


def _camera_set(n_cams: int, width: int, height: int, seed: int, device):
    """All rays of n_cams cameras, each camera's pixels in Morton order (so
    that a sorted batch is spatially coherent)."""
    poses = synth.sphere_poses(n_cams, seed=seed)
    o, d = synth.all_camera_rays(poses, width, height, device=device)
    npix = width * height
    pix = torch.arange(npix, device=device)
    order = torch.argsort(synth.scenes.morton2(pix % width, pix // width))
    idx = (torch.arange(n_cams, device=device)[:, None] * npix + order[None, :]).reshape(-1)
    return o[idx].contiguous(), d[idx].contiguous()


def _timed_steps(trainer: Trainer, sampler: RaySampler, steps: int) -> float:
    """Runs `steps` training steps; returns the mean ms per step (device
    events around the steps; batch gathers and segment lists included, the
    next batch's made on a second stream during each step)."""
    if steps <= 0:
        return 0.0
    torch.cuda.synchronize()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record()
    trainer.run(sampler, steps)
    b.record()
    torch.cuda.synchronize()
    return a.elapsed_time(b) / steps


def coarse_to_fine(steps_coarse: int = 300, steps_fine: int = 300, batch: int = 5000,
                   gt_reso=(256, 256, 256), occupancy: float = 0.10, n_blobs: int = 32,
                   coarse=(64, 64, 64), prune: str = "density", prune_thresh: float | None = None,
                   n_cams: int = 100, width: int = 800, height: int = 800, seed: int = 1,
                   log=print) -> dict:
    """prune: "density" (threshold on the stored density, default 5) or
    "weight" (threshold on the per-voxel maximum sample weight over all
    training rays, default 0.256, the synthetic-scene value of supplement
    B.1)."""
    if prune not in ("density", "weight"):
        raise ValueError("prune must be 'density' or 'weight'")
    if prune_thresh is None:
        prune_thresh = 5.0 if prune == "density" else 0.256
    dev = torch.device("cuda")
    t0 = time.time()
    gt = synth.blob_scene(gt_reso, n_blobs, occupancy, seed, device=dev)
    gt_grid = Grid.from_mask(gt.mask, gt_reso, gt.density, gt.sh)
    del gt
    o, d = _camera_set(n_cams, width, height, seed, dev)
    tgt = render_rays(gt_grid, o, d)
    ho, hd = _camera_set(2, 200, 200, seed + 500, dev)  # held-out views
    htgt = render_rays(gt_grid, ho, hd)
    del gt_grid
    torch.cuda.synchronize()
    log(f"c2 data: {o.shape[0]} training rays, {ho.shape[0]} held-out, {time.time() - t0:.1f}s")

    n = coarse[0] * coarse[1] * coarse[2]
    mask = torch.ones(n, dtype=torch.uint8, device=dev)
    grid = Grid.from_mask(mask, coarse, sigma0=0.1, dc=math.sqrt(math.pi))
    trainer = Trainer(grid, TrainConfig(), seed=seed)
    sampler = RaySampler(o, d, tgt, batch, seed=seed)
    _timed_steps(trainer, sampler, 5)  # warm-up
    ms_coarse = _timed_steps(trainer, sampler, steps_coarse)
    p_coarse = psnr(render_rays(trainer.grid, ho, hd), htgt)
    log(f"c2 coarse {coarse}: M={grid.n_vox}, {ms_coarse:.3f} ms/step, held-out PSNR {p_coarse:.2f}")

    torch.cuda.synchronize()
    t0w = time.perf_counter()
    weight_pass = None
    if prune == "weight":
        wmax = trainer.grid.max_weight(o, d, batch=1 << 22)
        torch.cuda.synchronize()
        tw = time.perf_counter() - t0w
        q = torch.quantile(wmax[wmax > 0][::7].double(), torch.tensor([0.5, 0.9, 0.99], dtype=torch.float64,
                                                                       device=dev)).tolist()
        weight_pass = {"rays": o.shape[0], "ms": round(tw * 1e3, 3),
                       "mrays_per_s": round(o.shape[0] / tw / 1e6, 2),
                       "voxels_seen": int((wmax > 0).sum()), "max_weight": float(wmax.max()),
                       "weight_p50_p90_p99_of_seen": [round(v, 6) for v in q]}
        log(f"c2 weight pass: {o.shape[0]} rays in {tw * 1e3:.1f} ms, {weight_pass}")
    t1 = time.perf_counter()
    if prune == "weight":
        pruned_grid, kept, pruned = trainer.grid.prune_by_weight(wmax, prune_thresh)
        del wmax
    else:
        pruned_grid, kept, pruned = trainer.grid.prune(prune_thresh)
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    if kept == 0:
        raise RuntimeError(f"a {prune} threshold of {prune_thresh} prunes every voxel")
    fine = pruned_grid.upsample(gt_reso)
    torch.cuda.synchronize()
    t3 = time.perf_counter()
    trainer.set_grid(fine)
    del grid, pruned_grid
    p_up = psnr(render_rays(fine, ho, hd), htgt)
    ms_fine = _timed_steps(trainer, sampler, steps_fine)
    p_fine = psnr(render_rays(trainer.grid, ho, hd), htgt)
    log(f"c2 fine {tuple(gt_reso)}: M={fine.n_vox}, {ms_fine:.3f} ms/step, PSNR after upsample "
        f"{p_up:.2f}, after training {p_fine:.2f}")
    return {
        "scene": f"{gt_reso[0]}^3 blobs at {occupancy:.0%} occupancy, {n_cams} cameras {width}x{height}",
        "batch_rays": batch,
        "coarse": {"reso": list(coarse), "n_vox": n, "steps": steps_coarse,
                   "ms_per_step": round(ms_coarse, 4), "psnr_heldout": round(p_coarse, 3)},
        "prune": {"by": prune, "thresh": prune_thresh, "kept": kept, "pruned": pruned,
                  "ms": round((t2 - t1) * 1e3, 3), "weight_pass": weight_pass},
        "upsample": {"reso": list(gt_reso), "n_vox": fine.n_vox, "ms": round((t3 - t2) * 1e3, 3),
                     "psnr_heldout": round(p_up, 3)},
        "fine": {"steps": steps_fine, "ms_per_step": round(ms_fine, 4),
                 "psnr_heldout": round(p_fine, 3)},
    }


NDC_LO, NDC_HI = (-1.0, -1.0, -1.0), (1.0, 1.0, 1.0)


def ndc_step_voxels(reso) -> float:
    """Sample step of half a voxel of the depth axis for a grid over the NDC
    cube (NDC rays of a forward-facing capture run nearly along z), in the
    finest-axis voxels Grid takes."""
    return 0.5 * max(reso) / reso[2]


def _ndc_camera_set(poses, width: int, height: int, device, near: float = 1.0):
    """All rays of the cameras (each camera's pixels in Morton order), warped
    to NDC with the reference camera's intrinsics."""
    o, d = synth.all_camera_rays(poses, width, height, device=device)
    npix = width * height
    pix = torch.arange(npix, device=device)
    order = torch.argsort(synth.scenes.morton2(pix % width, pix // width))
    idx = (torch.arange(poses.shape[0], device=device)[:, None] * npix + order[None, :]).reshape(-1)
    o, d = o[idx].contiguous(), d[idx].contiguous()
    B.plx_rays_to_ndc(o, d, width, height, synth.focal_length(width), near, o, d)
    return o, d


def forward_facing(steps_coarse: int = 300, steps_fine: int = 300, batch: int = 5000,
                   gt_reso=(512, 512, 128), occupancy: float = 0.10, n_blobs: int = 24,
                   coarse=(256, 256, 128), final=(1408, 1156, 128), prune_sigma: float = 1.0,
                   n_cams: int = 20, width: int = 1008, height: int = 756, seed: int = 3,
                   log=print) -> dict:
    dev = torch.device("cuda")
    t0 = time.time()
    gt = synth.blob_scene(gt_reso, n_blobs, occupancy, seed, device=dev)
    gt_grid = Grid.from_mask(gt.mask, gt_reso, gt.density, gt.sh, lo=NDC_LO, hi=NDC_HI,
                             step_voxels=ndc_step_voxels(gt_reso))
    del gt
    o, d = _ndc_camera_set(synth.forward_facing_poses(n_cams, seed=seed), width, height, dev)
    tgt = render_rays(gt_grid, o, d)
    ho, hd = _ndc_camera_set(synth.forward_facing_poses(2, seed=seed + 500), width // 2, height // 2, dev)
    htgt = render_rays(gt_grid, ho, hd)
    del gt_grid
    torch.cuda.synchronize()
    log(f"ff data: {o.shape[0]} training rays, {ho.shape[0]} held-out, {time.time() - t0:.1f}s")

    cfg = TrainConfig(lambda_tv_sigma=5e-4, lambda_tv_sh=5e-3, lambda_sparsity=1e-12)
    n = coarse[0] * coarse[1] * coarse[2]
    grid = Grid.from_mask(torch.ones(n, dtype=torch.uint8, device=dev), coarse, sigma0=0.1,
                          dc=math.sqrt(math.pi), lo=NDC_LO, hi=NDC_HI, step_voxels=ndc_step_voxels(coarse))
    trainer = Trainer(grid, cfg, seed=seed)
    sampler = RaySampler(o, d, tgt, batch, seed=seed)
    _timed_steps(trainer, sampler, 5)
    ms_coarse = _timed_steps(trainer, sampler, steps_coarse)
    p_coarse = psnr(render_rays(trainer.grid, ho, hd), htgt)
    log(f"ff coarse {coarse}: {ms_coarse:.3f} ms/step, held-out PSNR {p_coarse:.2f}")

    pruned_grid, kept, pruned = trainer.grid.prune(prune_sigma)
    if kept == 0:
        raise RuntimeError("the density threshold prunes every voxel")
    fine = pruned_grid.upsample(gt_reso, ndc_step_voxels(gt_reso))
    trainer.set_grid(fine)
    del grid, pruned_grid
    ms_fine = _timed_steps(trainer, sampler, steps_fine)
    p_fine = psnr(render_rays(trainer.grid, ho, hd), htgt)
    log(f"ff fine {tuple(gt_reso)}: M={fine.n_vox}, {ms_fine:.3f} ms/step, held-out PSNR {p_fine:.2f}")

    big = trainer.grid.upsample(final, ndc_step_voxels(final))
    trainer.set_grid(big)
    p_big = psnr(render_rays(big, ho, hd), htgt)
    ms_big = _timed_steps(trainer, sampler, 20)
    big_sampler = RaySampler(o, d, tgt, 1 << 20, seed=seed + 1)
    _timed_steps(trainer, big_sampler, 2)
    ms_big_1m = _timed_steps(trainer, big_sampler, 5)
    log(f"ff final {tuple(final)}: M={big.n_vox}, {ms_big:.3f} ms per 5000-ray step, "
        f"{ms_big_1m:.3f} ms per 1M-ray step, PSNR after upsample {p_big:.2f}")
    return {
        "scene": f"{gt_reso[0]}x{gt_reso[1]}x{gt_reso[2]} blobs over the NDC cube at {occupancy:.0%} "
                 f"occupancy, {n_cams} forward-facing cameras {width}x{height}",
        "batch_rays": batch,
        "coarse": {"reso": list(coarse), "n_vox": n, "steps": steps_coarse, "ms_per_step": round(ms_coarse, 4),
                   "psnr_heldout": round(p_coarse, 3)},
        "prune": {"sigma_thresh": prune_sigma, "kept": kept, "pruned": pruned},
        "fine": {"reso": list(gt_reso), "n_vox": fine.n_vox, "steps": steps_fine,
                 "ms_per_step": round(ms_fine, 4), "psnr_heldout": round(p_fine, 3)},
        "final": {"reso": list(final), "n_vox": big.n_vox, "psnr_after_upsample": round(p_big, 3),
                  "ms_per_step_5000": round(ms_big, 4), "ms_per_step_1m": round(ms_big_1m, 4),
                  "mrays_s_1m": round((1 << 20) / ms_big_1m / 1e3, 2)},
    }


def render_rays_360(fg: Grid, bg: Grid, o: torch.Tensor, d: torch.Tensor, bg_colour=(0.0, 0.0, 0.0),
                    chunk: int = 1 << 22) -> torch.Tensor:
    """Colours of rays through a foreground grid in front of an MSI
    background."""
    out = torch.empty(o.shape[0], 3, dtype=torch.float32, device=o.device)
    cbg = torch.empty(min(chunk, o.shape[0]), 3, dtype=torch.float32, device=o.device)
    for s in range(0, o.shape[0], chunk):
        e = min(s + chunk, o.shape[0])
        B.plx_bg_render_fwd(bg.desc(), o[s:e], d[s:e], cbg[:e - s], None, bg_colour)
        B.plx_render_fwd(fg.desc(), o[s:e], d[s:e], out[s:e], None, cbg[:e - s])
    return out


def _bg_grid(reso, density, coef, device) -> Grid:
    sh = torch.zeros(density.shape[0], 27, dtype=torch.float32, device=device)
    sh[:, 24:27] = coef
    n = reso[0] * reso[1] * reso[2]
    return Grid.from_mask(torch.ones(n, dtype=torch.uint8, device=device), reso, density, sh)


def unbounded_360(steps_coarse: int = 300, steps_fine: int = 300, batch: int = 5000,
                  gt_reso=(256, 256, 256), occupancy: float = 0.08, n_blobs: int = 24,
                  coarse=(128, 128, 128), bg_reso=(64, 256, 512), bg_full=(64, 1024, 2048),
                  prune_weight: float = 0.001, n_cams: int = 64, width: int = 640, height: int = 360,
                  lambda_beta: float = 1e-5, seed: int = 4, log=print) -> dict:
    dev = torch.device("cuda")
    t0 = time.time()
    gt = synth.blob_scene(gt_reso, n_blobs, occupancy, seed, device=dev)
    gt_fg = Grid.from_mask(gt.mask, gt_reso, gt.density, gt.sh)
    del gt
    _, bd, bc = synth.sky_background(bg_reso, seed)
    gt_bg = _bg_grid(bg_reso, bd.to(dev), bc.to(dev), dev)
    poses = synth.sphere_poses(n_cams, seed=seed, radius=0.8)
    o, d = synth.all_camera_rays(poses, width, height, fov_deg=70.0, device=dev)
    tgt = render_rays_360(gt_fg, gt_bg, o, d)
    hp = synth.sphere_poses(2, seed=seed + 500, radius=0.8)
    ho, hd = synth.all_camera_rays(hp, width // 2, height // 2, fov_deg=70.0, device=dev)
    htgt = render_rays_360(gt_fg, gt_bg, ho, hd)
    del gt_fg, gt_bg
    torch.cuda.synchronize()
    log(f"360 data: {o.shape[0]} training rays, {ho.shape[0]} held-out, {time.time() - t0:.1f}s")

    cfg = TrainConfig(lambda_tv_sigma=5e-5, lambda_tv_sh=5e-3, lambda_sparsity=1e-11, lambda_beta=lambda_beta)
    n = coarse[0] * coarse[1] * coarse[2]
    fg = Grid.from_mask(torch.ones(n, dtype=torch.uint8, device=dev), coarse, sigma0=0.1, dc=math.sqrt(math.pi))
    nb = bg_reso[0] * bg_reso[1] * bg_reso[2]
    bg = _bg_grid(bg_reso, torch.full((nb,), 0.1, device=dev),
                  torch.full((nb, 3), math.sqrt(math.pi), device=dev), dev)
    trainer = Trainer(fg, cfg, seed=seed, background=bg)
    sampler = RaySampler(o, d, tgt, batch, seed=seed)
    _timed_steps(trainer, sampler, 5)
    ms_coarse = _timed_steps(trainer, sampler, steps_coarse)
    p_coarse = psnr(render_rays_360(trainer.grid, trainer.bg, ho, hd), htgt)
    log(f"360 coarse {coarse} + bg {bg_reso}: {ms_coarse:.3f} ms/step, held-out PSNR {p_coarse:.2f}")

    # pruning by weight, the paper's choice for 360-degree scenes
    wmax = trainer.grid.max_weight(o, d, batch=1 << 22)
    pruned, kept, npruned = trainer.grid.prune_by_weight(wmax, prune_weight)
    del wmax
    if kept == 0:
        raise RuntimeError("the weight threshold prunes every voxel")
    fine = pruned.upsample(gt_reso)
    trainer.set_grid(fine)
    del fg, pruned
    ms_fine = _timed_steps(trainer, sampler, steps_fine)
    p_fine = psnr(render_rays_360(trainer.grid, trainer.bg, ho, hd), htgt)
    log(f"360 fine {gt_reso}: M={fine.n_vox}, {ms_fine:.3f} ms/step, held-out PSNR {p_fine:.2f}")

    # 1M-ray steps with the background at the paper's size (dense)
    nf = bg_full[0] * bg_full[1] * bg_full[2]
    big_bg = _bg_grid(bg_full, torch.full((nf,), 0.1, device=dev), torch.full((nf, 3), math.sqrt(math.pi), device=dev),
                      dev)
    trainer.set_background(big_bg)
    del bg
    torch.cuda.empty_cache()
    big = RaySampler(o, d, tgt, 1 << 20, seed=seed + 1)
    _timed_steps(trainer, big, 2)
    ms_1m = _timed_steps(trainer, big, 5)
    # the two background kernels on one 1M-ray batch
    bo, bdd, _ = big.next_batch()
    cb = torch.empty(bo.shape[0], 3, device=dev)
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
    ev[0].record()
    B.plx_bg_render_fwd(trainer.bg.desc(), bo, bdd, cb, None, cfg.bg_background)
    ev[1].record()
    B.plx_bg_render_bwd(trainer.bg.desc(), bo, bdd, cb, trainer.bg_grad, trainer.bg_touched, cfg.bg_background)
    ev[2].record()
    torch.cuda.synchronize()
    ms_bgf, ms_bgb = ev[0].elapsed_time(ev[1]), ev[1].elapsed_time(ev[2])
    log(f"360 1M-ray step, fg {gt_reso} M={fine.n_vox}, bg {bg_full}: {ms_1m:.3f} ms "
        f"(bg fwd {ms_bgf:.3f} ms, bg bwd {ms_bgb:.3f} ms)")
    return {
        "scene": f"{gt_reso[0]}^3 blobs at {occupancy:.0%} occupancy inside the unit sphere, procedural sky on "
                 f"{bg_reso[0]}x{bg_reso[1]}x{bg_reso[2]} MSI, {n_cams} inward cameras {width}x{height} at radius 0.8",
        "batch_rays": batch,
        "lambda_beta": lambda_beta,
        "coarse": {"fg_reso": list(coarse), "bg_reso": list(bg_reso), "steps": steps_coarse,
                   "ms_per_step": round(ms_coarse, 4), "psnr_heldout": round(p_coarse, 3)},
        "prune": {"weight_thresh": prune_weight, "kept": kept, "pruned": npruned},
        "fine": {"fg_reso": list(gt_reso), "n_vox": fine.n_vox, "steps": steps_fine,
                 "ms_per_step": round(ms_fine, 4), "psnr_heldout": round(p_fine, 3)},
        "step_1m": {"bg_reso": list(bg_full), "bg_voxels": nf, "ms_per_step": round(ms_1m, 4),
                    "mrays_s": round((1 << 20) / ms_1m / 1e3, 2), "bg_fwd_ms": round(ms_bgf, 4),
                    "bg_bwd_ms": round(ms_bgb, 4)},
    }


def precision_drift(steps: int = 2000, batch: int = 1 << 20, reso=(512, 512, 512),
                    occupancy: float = 0.05, n_blobs: int = 32, n_cams: int = 100,
                    width: int = 800, height: int = 800, seed: int = 2, log=print,
                    on_final=None) -> dict:
    """on_final(name, grid, heldout_rays): called with each trained grid
    before it is released (the held-out rays are (o, d) of 10 poses at
    200x200)."""
    dev = torch.device("cuda")
    gt = synth.blob_scene(reso, n_blobs, occupancy, seed, device=dev)
    gt_grid = Grid.from_mask(gt.mask, reso, gt.density, gt.sh)
    o, d = _camera_set(n_cams, width, height, seed, dev)
    tgt = render_rays(gt_grid, o, d)
    ho, hd = _camera_set(10, 200, 200, seed + 500, dev)  # 10 held-out poses
    htgt = render_rays(gt_grid, ho, hd)
    del gt_grid
    # the trained grids start from the ground-truth occupancy with perturbed values
    init = synth.perturbed(gt, seed=seed + 1000, device=dev)
    dens, sh = init.density, init.sh
    out = {"scene": f"{reso[0]}^3 blobs at {occupancy:.0%} occupancy", "steps": steps,
           "batch_rays": batch, "heldout": "10 poses at 200x200", "runs": {}}
    renders = {}
    for name in ("f32", "bf16", "f16"):
        grid = Grid.from_mask(gt.mask, reso, dens, sh, sh_dtype=B.DTYPES[name])
        trainer = Trainer(grid, TrainConfig(), seed=seed)
        sampler = RaySampler(o, d, tgt, batch, seed=seed)
        p0 = psnr(render_rays(grid, ho, hd), htgt)
        t0 = time.perf_counter()
        ms = _timed_steps(trainer, sampler, steps)
        wall = time.perf_counter() - t0
        img = render_rays(grid, ho, hd)
        renders[name] = img
        loss = trainer.loss_sum.item() / max(steps, 1)
        out["runs"][name] = {"psnr_heldout_init": round(p0, 3), "psnr_heldout": round(psnr(img, htgt), 3),
                             "ms_per_step": round(ms, 4), "mean_train_loss": loss,
                             "wall_s": round(wall, 1)}
        log(f"drift {name}: PSNR {p0:.2f} -> {out['runs'][name]['psnr_heldout']:.2f}, "
            f"{ms:.3f} ms/step")
        if on_final is not None:
            on_final(name, grid, (ho, hd))
        del grid, trainer, sampler
        torch.cuda.empty_cache()
    for name in ("bf16", "f16"):
        diff = (renders[name] - renders["f32"]).abs()
        out["runs"][name]["vs_f32"] = {"psnr": round(psnr(renders[name], renders["f32"]), 3),
                                       "max_abs": float(diff.max()), "mean_abs": float(diff.mean()),
                                       "p99_abs": float(torch.quantile(diff.flatten()[::7], 0.99))}
    return out


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("run", choices=["coarse_to_fine", "drift", "forward_facing", "unbounded_360"])
    ap.add_argument("--steps", type=int, default=None)
    ap.add_argument("--prune", choices=["density", "weight"], default="density")
    ap.add_argument("--prune-thresh", type=float, default=None)
    ap.add_argument("--lambda-beta", type=float, default=None)
    args = ap.parse_args(argv)
    torch.cuda.set_device(0)
    log = lambda *a: print(*a, file=sys.stderr, flush=True)  # noqa: E731
    if args.run == "coarse_to_fine":
        s = args.steps or 300
        res = coarse_to_fine(steps_coarse=s, steps_fine=s, prune=args.prune,
                             prune_thresh=args.prune_thresh, log=log)
    elif args.run == "unbounded_360":
        s = args.steps or 300
        res = unbounded_360(steps_coarse=s, steps_fine=s, log=log,
                            lambda_beta=1e-5 if args.lambda_beta is None else args.lambda_beta)
    elif args.run == "forward_facing":
        s = args.steps or 300
        res = forward_facing(steps_coarse=s, steps_fine=s, log=log,
                             prune_sigma=1.0 if args.prune_thresh is None else args.prune_thresh)
    else:
        res = precision_drift(steps=args.steps or 2000, log=log)
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
