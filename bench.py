"""Throughput benchmark of the Plenoxels training step on one MI355X.

Workload (the differentiation/scale configuration): a 512^3 sparse grid at 5%
occupancy (6.71M voxels, FP32 records) built from 32 seeded Gaussian density
blobs, 100 cameras on the radius-2 sphere at 800x800, and 1M-ray batches drawn
uniformly from all their pixels (listed in camera / Morton-pixel order; the
same rays shuffled are timed too); targets are renders of the ground-truth
grid.  The trained grid has the same occupancy with perturbed values.  One
step = fused render + MSE + backward over the batch, TV on a random
contiguous 1% segment of the cells, and sparse RMSProp on the active voxels.

Prints one JSON line: whole-step Mrays/s, the roofline of the dominant kernel
(render_train, algorithmic bytes from the library's work counters over its
HIP-event duration; beside it the bytes rocprofv3's counters measured for
the same call, over the same duration, and their ratio to the algorithmic
bytes), the same step with BF16/FP16 SH storage and with
shuffled rays and with the sparsity and beta priors on, separate
forward/backward with and without stored per-sample state, the
pruning-by-weight pass, the serving latency leg, and the FP64
oracle timed on a bounded sample of the same workload on the host cores.
"""
import argparse
import json
import math
import os
import sys
import time

import numpy as np
import torch

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import synth  # noqa: E402
from paper_2112_05131_amd import binding as B  # noqa: E402
from paper_2112_05131_amd.grid import Grid  # noqa: E402
from paper_2112_05131_amd.train import TrainConfig, Trainer  # noqa: E402

METRIC = "fwd+bwd Mrays/s & HBM GB/s vs plain FP32; p50/p99 view-render latency"
HBM_PEAK_GBS = 8000.0
RESO = (512, 512, 512)
OCC = 0.05
N_BLOBS = 32
SEED = 2
BATCH = 1 << 20
N_CAMS, W, H = 100, 800, 800
# HBM bytes moved by one plx_render_train call of this workload (FP32
# records), from rocprofv3 FETCH_SIZE and WRITE_SIZE passes over
# `bench.py --counters`, each scaled by its reading for a 1 GiB device copy
# (FETCH x2, WRITE x1): 9.811 GB fetched + 8.766 GB written.  Re-measure
# whenever the render kernels change.
RENDER_TRAIN_TRAFFIC_GB_F32 = 18.58
# the same with BF16 SH records (`--dtype bf16`): 4.765 GB + 8.744 GB
RENDER_TRAIN_TRAFFIC_GB_BF16 = 13.51


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def build_workload(sh_dtype, n_batches, coherent=True):
    t0 = time.time()
    gt = synth.blob_scene(RESO, N_BLOBS, OCC, SEED, device="cuda")
    gt_grid = Grid.from_mask(gt.mask, RESO, gt.density, gt.sh)
    gen = torch.Generator(device="cuda")
    gen.manual_seed(SEED + 1000)
    dens = gt.density * (0.5 + torch.rand(gt.n_vox, device="cuda", generator=gen))
    sh = gt.sh + 0.05 * torch.randn(gt.n_vox, 27, device="cuda", generator=gen)
    grid = Grid.from_mask(gt.mask, RESO, dens, sh, sh_dtype=sh_dtype)
    poses = synth.sphere_poses(N_CAMS, seed=SEED)
    batches = []
    for b in range(n_batches):
        o, d, _ = synth.sampled_camera_rays(poses, W, H, BATCH, seed=SEED + 10 * b, device="cuda",
                                            coherent=coherent)
        tgt = torch.empty(BATCH, 3, device="cuda")
        B.plx_render_fwd(gt_grid.desc(), o, d, tgt)
        batches.append((o, d, tgt))
    torch.cuda.synchronize()
    log(f"workload built in {time.time() - t0:.1f}s: M={grid.n_vox}, batches={n_batches}")
    return gt, grid, batches, (dens, sh)


def time_steps(trainer, batches, warmup, steps):
    g = trainer.grid
    c = trainer.cfg
    for i in range(warmup):
        o, d, t = batches[i % len(batches)]
        trainer.step(o, d, t)
    torch.cuda.synchronize()
    evs = []
    t0 = time.perf_counter()
    start = torch.cuda.Event(enable_timing=True)
    end = torch.cuda.Event(enable_timing=True)
    start.record()
    for i in range(steps):
        o, d, t = batches[(warmup + i) % len(batches)]
        e = [torch.cuda.Event(enable_timing=True) for _ in range(4)]
        lr_s, lr_h = trainer.learning_rates()
        e[0].record()
        B.plx_render_train(g.desc(), o, d, t, 1.0 / o.shape[0], trainer.grad, trainer.touched,
                           trainer.loss_sum, None, c.background, trainer.priors())
        e[1].record()
        s0, cnt = trainer.tv_segment()
        B.plx_tv_grad(g.desc(), s0, cnt, c.lambda_tv_sigma, c.lambda_tv_sh, c.tv_eps, trainer.grad,
                      trainer.touched, trainer.tv_loss_sum)
        e[2].record()
        B.plx_rmsprop_step(g.desc(), g.master, trainer.vstate, trainer.grad, trainer.touched, lr_s,
                           lr_h, c.beta, c.eps)
        e[3].record()
        trainer.step_id += 1
        evs.append(e)
    end.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms = start.elapsed_time(end) / steps
    k_ms = np.array([[e[0].elapsed_time(e[1]), e[1].elapsed_time(e[2]), e[2].elapsed_time(e[3])]
                     for e in evs]).mean(axis=0)
    return ms, wall, k_ms


def work_counters(grid, batch):
    o, d, _ = batch
    cm = torch.zeros((grid.n_cells + 31) // 32, dtype=torch.int32, device="cuda")
    vm = torch.zeros((grid.n_vox + 31) // 32, dtype=torch.int32, device="cuda")
    return B.plx_render_stats(grid.desc(), o, d, cm, vm)


def active_count(trainer, batch):
    """Active-set size of one step (untimed; the state is restored)."""
    g, c = trainer.grid, trainer.cfg
    o, d, t = batch
    grad0 = trainer.grad.clone()
    touched0 = trainer.touched.clone()
    B.plx_render_train(g.desc(), o, d, t, 1.0 / o.shape[0], trainer.grad, trainer.touched,
                       trainer.loss_sum, None, c.background)
    s0, cnt = trainer.tv_segment()
    B.plx_tv_grad(g.desc(), s0, cnt, c.lambda_tv_sigma, c.lambda_tv_sh, c.tv_eps, trainer.grad,
                  trainer.touched, trainer.tv_loss_sum)
    a = B.plx_touched_count(trainer.touched, g.n_vox)
    trainer.grad.copy_(grad0)
    trainer.touched.copy_(touched0)
    return a, cnt


def cpu_baseline(gt, grid_vals, batch, budget_s=15.0):
    """The FP64 oracle on a bounded sample of the same workload: fwd + MSE +
    bwd over S rays of the batch, TV on S/R of the step's segment and RMSProp
    on the sample's active voxels, timed on the host."""
    from oracle import oracle as O
    dens, sh = grid_vals
    og = O.make_grid(np.array(RESO, np.int32), gt.mask.cpu().numpy(), dens.cpu().double().numpy(),
                     sh.cpu().double().numpy())
    o, d, t = (x.cpu().numpy() for x in batch)
    ncell = RESO[0] * RESO[1] * RESO[2]

    def run(s):
        t0 = time.perf_counter()
        rgb = O.render_fwd(og, o[:s], d[:s])[0]
        g_rgb, _ = O.mse_grad(rgb, t[:s])
        gd, gs, act = O.render_bwd(og, o[:s], d[:s], g_rgb)
        cnt = max(1, int(math.ceil(0.01 * ncell * s / BATCH)))
        _, td, ts, a2 = O.tv(og, 12345, cnt, 1e-5, 1e-3)
        act = act | a2
        m = og.n_vox
        O.rmsprop(act, og.density, og.sh, np.zeros(m), np.zeros((m, 27)), gd + td, gs + ts,
                  1.0, 0.01)
        return time.perf_counter() - t0

    run(500)  # first touch of the grid arrays
    s = 4000
    ts_ = run(s)
    while ts_ < 0.5 * budget_s and s < BATCH:
        s = int(min(BATCH, s * min(8.0, budget_s / max(ts_, 1e-6))))
        ts_ = run(s)
    cores = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    return {"value": round(s / ts_ / 1e6, 6), "unit": "Mrays/s", "cores": cores, "kind": "oracle",
            "sample": f"{s} rays of one 1M-ray batch (fwd+MSE+bwd), TV on {s}/{BATCH} of the 1% "
                      f"segment, RMSProp on the sample's active voxels; {ts_:.1f} s FP64"}


def state_leg(grid, batch, steps, cap=640):
    """Separate forward + backward of one batch, with the backward recomputing
    every sample (plx_render_fwd/bwd) or replaying the samples stored by the
    forward pass (plx_render_fwd_state/bwd_state, at most `cap` per ray)."""
    o, d, t = batch
    n = o.shape[0]
    rgb = torch.empty(n, 3, device="cuda")
    tau = torch.empty(n, device="cuda")
    g_rgb = torch.empty(n, 3, device="cuda")
    grad = torch.zeros(grid.n_vox, B.REC_SLOTS, device="cuda")
    touched = torch.zeros(grid.n_vox, dtype=torch.uint8, device="cuda")
    state = torch.empty(B.plx_render_state_bytes(n, cap), dtype=torch.uint8, device="cuda")
    reps = max(3, steps // 4)

    def timed(fn):
        fn()
        torch.cuda.synchronize()
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        for _ in range(reps):
            fn()
        b.record()
        torch.cuda.synchronize()
        return a.elapsed_time(b) / reps

    desc = grid.desc()
    fwd = timed(lambda: B.plx_render_fwd(desc, o, d, rgb, tau))
    torch.sub(rgb, t, out=g_rgb).mul_(2.0 / n)
    bwd = timed(lambda: B.plx_render_bwd(desc, o, d, g_rgb, tau, grad, touched))
    fwd_s = timed(lambda: B.plx_render_fwd_state(desc, o, d, rgb, tau, state, cap))
    bwd_s = timed(lambda: B.plx_render_bwd_state(desc, o, d, g_rgb, tau, state, cap, grad, touched))
    counts = state[:4 * n].view(torch.int32)
    over = int((counts > cap).sum())
    del state, grad
    torch.cuda.empty_cache()
    log(f"recompute fwd {fwd:.3f} bwd {bwd:.3f} ms; stored state fwd {fwd_s:.3f} bwd {bwd_s:.3f} ms")
    return {"recompute": {"fwd_ms": round(fwd, 4), "bwd_ms": round(bwd, 4)},
            "stored": {"fwd_ms": round(fwd_s, 4), "bwd_ms": round(bwd_s, 4), "cap": cap,
                       "state_gb": round(B.plx_render_state_bytes(n, cap) / 1e9, 3),
                       "rays_over_cap": over}}


def prune_weight_leg(grid, batches, counts, thresh=0.01):
    """Pruning by weight on the training workload: the per-voxel maximum
    sample weight accumulated over the distinct 1M-ray batches from zeros
    (plx_render_max_weight once per batch, brick order, density only), then
    the dilated threshold count over the whole grid
    (plx_grid_prune_weight_count), timed with HIP events on the stream the
    calls are launched on.  Algorithmic bytes of one weight call: the index
    entries read (4 B each), per voxel read its density (4 B) and one
    read-modify-write of its maximum (8 B), and 24 B of ray per ray."""
    wmax = torch.zeros(grid.n_vox, device="cuda")
    keep = torch.empty(grid.n_cells, dtype=torch.uint8, device="cuda")
    desc = grid.desc()
    o, d, _ = batches[0]
    B.plx_render_max_weight(desc, o, d, wmax)  # warm-up (library and allocator)
    wmax.zero_()
    torch.cuda.synchronize()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record()
    for o, d, _ in batches:
        B.plx_render_max_weight(desc, o, d, wmax)
    b.record()
    torch.cuda.synchronize()
    ms = a.elapsed_time(b) / len(batches)
    a.record()
    kept, pruned = B.plx_grid_prune_weight_count(desc, wmax, thresh, keep)
    b.record()
    torch.cuda.synchronize()
    ms_prune = a.elapsed_time(b)
    n = batches[0][0].shape[0]
    alg = 4 * counts[2] + 12 * counts[3] + 24 * n
    gbs = alg / (ms * 1e-3) / 1e9
    log(f"max weight {ms:.3f} ms per {n}-ray batch ({len(batches)} batches); prune count {ms_prune:.3f} ms "
        f"(kept {kept})")
    del wmax, keep
    torch.cuda.empty_cache()
    return {"max_weight_ms_per_batch": round(ms, 4), "batches": len(batches), "mrays_s": round(n / ms / 1e3, 2),
            "roofline": {"bound": "hbm", "kernel": "max_weight (one plx_render_max_weight call)",
                         "achieved": round(gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                         "frac": round(gbs / HBM_PEAK_GBS, 4), "algorithmic_gb": round(alg / 1e9, 3)},
            "prune_count_ms": round(ms_prune, 3), "threshold": thresh, "kept": kept, "pruned": pruned}


def serving_leg(n_sat=400, n_load=2000):
    """8 resident scenes (4 at 256^3, 4 at 512^3, 5-10% occupancy, FP16 SH),
    requests at 200x200 .. 1920x1080 with random poses on the view sphere:
    saturation throughput (all requests at once), then Poisson arrivals at 50,
    80 and 95% of it.  Returns the serving summary."""
    from paper_2112_05131_amd.serve import Server, random_requests, run_load
    t0 = time.time()
    scenes = []
    for i, seed in enumerate(range(3, 11)):
        reso = (256,) * 3 if i < 4 else (512,) * 3
        occ = 0.05 + 0.05 * (i % 4) / 3.0
        sv = synth.blob_scene(reso, N_BLOBS, occ, seed, device="cuda")
        scenes.append(Grid.from_mask(sv.mask, reso, sv.density, sv.sh, sh_dtype=B.PLX_F16))
        del sv
    torch.cuda.synchronize()
    resident = sum(s.index.numel() * 4 + s.data.numel() * s.data.element_size() +
                   s.occ.numel() * 4 for s in scenes)
    log(f"serving scenes built in {time.time() - t0:.1f}s, resident {resident / 1e9:.2f} GB")
    srv = Server(scenes, hbm_budget=1 << 30, n_streams=4, max_batch=32, keep_outputs=False)
    run_load(srv, random_requests(16, 8, seed=99), None)  # warm-up
    reqs = random_requests(n_sat, 8, seed=100)
    lat, wall = run_load(srv, reqs, None)
    pix = sum(r.n_pixels for r in reqs)
    sat_rps = n_sat / wall
    out = {"scenes": "4x256^3 + 4x512^3, 5-10% occupancy, FP16 SH",
           "resident_gb": round(resident / 1e9, 3),
           "saturation_mrays_s": round(pix / wall / 1e6, 2),
           "saturation_requests_s": round(sat_rps, 1), "loads": []}
    for frac in (0.5, 0.8, 0.95):
        reqs = random_requests(n_load, 8, seed=101 + int(frac * 100))
        lat, wall = run_load(srv, reqs, sat_rps * frac, seed=7)
        pix = sum(r.n_pixels for r in reqs)
        out["loads"].append({"load": frac, "offered_requests_s": round(sat_rps * frac, 1),
                             "p50_ms": round(float(np.percentile(lat, 50)) * 1e3, 3),
                             "p99_ms": round(float(np.percentile(lat, 99)) * 1e3, 3),
                             "mrays_s": round(pix / wall / 1e6, 2), "requests": n_load})
        log(f"serving load {frac}: p50 {out['loads'][-1]['p50_ms']} ms p99 {out['loads'][-1]['p99_ms']} ms")
    del srv, scenes
    torch.cuda.empty_cache()
    return out


def counter_run(sh_dtype, coherent):
    """Dispatch sequence for rocprofv3 --pmc passes: a warm-up step, one
    training step (render_train's kernels, tv_kernel, rmsprop_kernel), then a
    1 GiB device-to-device copy (1 GiB read + 1 GiB written) whose counter
    readings give the scale of FETCH_SIZE / WRITE_SIZE."""
    gt, grid, batches, vals = build_workload(sh_dtype, 1, coherent)
    trainer = Trainer(grid, TrainConfig(), seed=SEED)
    o, d, t = batches[0]
    for _ in range(2):
        trainer.step(o, d, t)
        torch.cuda.synchronize()
    src = torch.ones(1 << 28, device="cuda")
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    dst.copy_(src)
    torch.cuda.synchronize()
    log("counter run done")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--dtype", default="f32", choices=["f32", "bf16", "f16"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-compare", action="store_true", help="skip the BF16/FP16-SH steps")
    ap.add_argument("--no-serving", action="store_true", help="skip the serving latency leg")
    ap.add_argument("--ray-order", default="coherent", choices=["coherent", "random"],
                    help="order of the rays inside each batch (the same rays either way)")
    ap.add_argument("--counters", action="store_true",
                    help="for counter runs under rocprofv3: one warm-up and one timed-shape "
                         "training step on one batch, then a 1 GiB device copy that calibrates "
                         "the byte counters; prints no JSON line")
    ap.add_argument("--serving-only", action="store_true",
                    help="for trace runs under rocprofv3: only the serving leg, printed as its "
                         "own JSON object")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU; --gpus {args.gpus} is not supported "
              "(the library has no multi-GPU path).", file=sys.stderr)
        sys.exit(2)
    torch.cuda.set_device(0)
    sh_dtype = B.DTYPES[args.dtype]
    if args.counters:
        counter_run(sh_dtype, args.ray_order == "coherent")
        return
    if args.serving_only:
        print(json.dumps({"serving": serving_leg()}), flush=True)
        return
    n_batches = min(args.warmup + args.steps, 8)
    gt, grid, batches, vals = build_workload(sh_dtype, n_batches, args.ray_order == "coherent")
    trainer = Trainer(grid, TrainConfig(), seed=SEED)

    counts = work_counters(grid, batches[0])
    n_act, tv_cells = active_count(trainer, batches[0])
    log(f"counters: samples={counts[0]} occupied_samples={counts[1]} U_idx={counts[2]} "
        f"U_occ={counts[3]} active={n_act}")

    ms, wall, k_ms = time_steps(trainer, batches, args.warmup, args.steps)
    mrays = BATCH / (ms * 1e-3) / 1e6
    log(f"step {ms:.3f} ms (wall {wall / args.steps * 1e3:.3f} ms/step); kernels ms: "
        f"render_train {k_ms[0]:.3f} tv {k_ms[1]:.3f} rmsprop {k_ms[2]:.3f}")

    P = 112 if sh_dtype == B.PLX_F32 else 58
    alg_render = 4 * counts[2] + (P + 224) * counts[3] + 36 * BATCH
    achieved = alg_render / (k_ms[0] * 1e-3) / 1e9
    traffic_gb = {B.PLX_F32: RENDER_TRAIN_TRAFFIC_GB_F32, B.PLX_BF16: RENDER_TRAIN_TRAFFIC_GB_BF16}.get(sh_dtype)
    alg_rms = n_act * (672 if sh_dtype == B.PLX_F32 else 726)
    alg_tv = 4 * 4 * tv_cells
    step_gbs = (alg_render + alg_rms + alg_tv) / (ms * 1e-3) / 1e9

    out = {
        "metric": METRIC,
        "value": round(mrays, 3),
        "unit": "Mrays/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": args.dtype,
        "data": "synthetic",
        "config": {
            "workload": "512^3 sparse grid, 5% occupancy (6.71M voxels), SH deg 2, "
                        "1M-ray batches from 100 cameras at 800x800; step = fused "
                        "render+MSE+backward, TV on a 1% contiguous segment, sparse RMSProp",
            "sh_storage": args.dtype,
            "batch_rays": BATCH,
            "ray_order": args.ray_order,
            "grid": list(RESO),
            "n_vox": grid.n_vox,
        },
        "roofline": {
            "bound": "hbm",
            "kernel": "render_train (one plx_render_train call: seg_count, count scans, seg_emit, "
                      "seg_fwd, seg_combine, seg_bwd)",
            "achieved": round(achieved, 1),
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4),
            "traffic": traffic_gb,
            "traffic_unit": "GB per call (measured)",
            "algorithmic_gb": round(alg_render / 1e9, 3),
            # the measured bytes over this run's call time, and their ratio to
            # the algorithmic bytes
            "traffic_gbs": (round(traffic_gb / (k_ms[0] * 1e-3), 1)
                            if traffic_gb else None),
            "traffic_frac": (round(traffic_gb / (k_ms[0] * 1e-3) / HBM_PEAK_GBS, 4)
                             if traffic_gb else None),
            "amplification": (round(traffic_gb * 1e9 / alg_render, 2)
                              if traffic_gb else None),
        },
        "kernels_ms": {"render_train": round(float(k_ms[0]), 4), "tv_grad": round(float(k_ms[1]), 4),
                       "rmsprop_step": round(float(k_ms[2]), 4)},
        "step_hbm_gbs_algorithmic": round(step_gbs, 1),
        "work": {"samples": counts[0], "occupied_samples": counts[1], "index_entries": counts[2],
                 "voxels_read": counts[3], "active_voxels": n_act, "tv_cells": tv_cells},
    }
    if not args.no_compare:
        # the same step with SH stored in FP32, BF16 and FP16 (FP32 optimiser
        # state and accumulation in all three)
        prec = {args.dtype: {"ms_per_step": round(ms, 4), "mrays_s": round(mrays, 3),
                             "render_train_ms": round(float(k_ms[0]), 4)}}
        for name in ("f32", "bf16", "f16"):
            if name in prec:
                continue
            g2 = Grid.from_mask(gt.mask, RESO, vals[0], vals[1], sh_dtype=B.DTYPES[name])
            tr2 = Trainer(g2, TrainConfig(), seed=SEED)
            ms2, _, k2 = time_steps(tr2, batches, 2, max(5, args.steps // 2))
            prec[name] = {"ms_per_step": round(ms2, 4), "mrays_s": round(BATCH / ms2 / 1e3, 3),
                          "render_train_ms": round(float(k2[0]), 4)}
            log(f"{name}: step {ms2:.3f} ms, render_train {k2[0]:.3f} ms")
            del g2, tr2
        for name in prec:
            prec[name]["speedup_vs_f32"] = round(prec["f32"]["ms_per_step"] / prec[name]["ms_per_step"], 4)
        out["precision"] = prec
        if args.ray_order == "coherent":
            # the same rays, shuffled inside each batch
            gen = torch.Generator(device="cuda")
            gen.manual_seed(SEED + 77)
            shuffled = []
            for o, d, t in batches:
                p = torch.randperm(BATCH, device="cuda", generator=gen)
                shuffled.append((o[p].contiguous(), d[p].contiguous(), t[p].contiguous()))
            g3 = Grid.from_mask(gt.mask, RESO, vals[0], vals[1], sh_dtype=sh_dtype)
            tr3 = Trainer(g3, TrainConfig(), seed=SEED)
            ms3, _, k3 = time_steps(tr3, shuffled, 2, max(5, args.steps // 2))
            out["random_order"] = {"ms_per_step": round(ms3, 4), "mrays_s": round(BATCH / ms3 / 1e3, 3),
                                   "render_train_ms": round(float(k3[0]), 4)}
            log(f"random ray order: step {ms3:.3f} ms, render_train {k3[0]:.3f} ms")
            del g3, tr3, shuffled
    if not args.no_compare:
        # the same step with the sparsity and beta priors of Sec. 3.7 on (the
        # paper's 360-degree weights)
        g4 = Grid.from_mask(gt.mask, RESO, vals[0], vals[1], sh_dtype=sh_dtype)
        tr4 = Trainer(g4, TrainConfig(lambda_sparsity=1e-11, lambda_beta=1e-5), seed=SEED)
        ms4, _, k4 = time_steps(tr4, batches, 2, max(5, args.steps // 2))
        out["with_priors"] = {"lambda_sparsity": 1e-11, "lambda_beta": 1e-5, "ms_per_step": round(ms4, 4),
                              "mrays_s": round(BATCH / ms4 / 1e3, 3), "render_train_ms": round(float(k4[0]), 4)}
        log(f"with priors: step {ms4:.3f} ms, render_train {k4[0]:.3f} ms")
        del g4, tr4
        out["backward_state"] = state_leg(grid, batches[0], args.steps)
    out["prune_by_weight"] = prune_weight_leg(grid, batches, counts)
    if not args.no_serving:
        out["serving"] = serving_leg()
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(gt, vals, batches[0])
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
