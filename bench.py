"""Throughput benchmark of the Plenoxels training step on one MI355X.

Workload (the differentiation/scale configuration): a 512^3 sparse grid at 5%
occupancy (6.71M voxels, FP32 records) built from 32 seeded Gaussian density
blobs, and all 64M pixels of 100 cameras on the radius-2 sphere at 800x800
resident on the device with their targets (renders of the ground-truth
grid).  The trained grid has the ground-truth occupancy with perturbed
values.  One step = gather of a 1M-ray batch (a slice of a per-epoch
permutation of all pixels, listed in camera / Morton-pixel order), its
segment lists (count + apply), fused render + MSE + backward, TV on a random
contiguous 1% segment of the cells, and sparse RMSProp on the active voxels;
the gather and segment lists of batch t+1 run on a second stream during step
t (Trainer.run), and the timed region holds every part of every step.

Prints one JSON line: whole-step Mrays/s; the roofline of the dominant kernel
of the fused render call (the longer of seg_fwd, the segment forward, and
seg_scatter, the recorded backward: the algorithmic bytes of the forward or
backward pass from the library's work counters over the kernel's duration
measured with HIP events recorded on its stream), with the per-kernel times
and fractions beside it;
the same step with BF16/FP16 SH storage, with shuffled rays, without the
second stream and with the sparsity and beta priors on; separate
forward/backward with and without stored per-sample state; the
pruning-by-weight pass; the serving latency leg; and the FP64 oracle timed
on a bounded sample of the same workload on all host cores and on one.
"""
import argparse
import gc
import hashlib
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
from paper_2112_05131_amd.runs import _camera_set, render_rays  # noqa: E402
from paper_2112_05131_amd.train import RaySampler, TrainConfig, Trainer  # noqa: E402

METRIC = "fwd+bwd Mrays/s & HBM GB/s vs plain FP32; p50/p99 view-render latency"
HBM_PEAK_GBS = 8000.0
RESO = (512, 512, 512)
OCC = 0.05
N_BLOBS = 32
SEED = 2
BATCH = 1 << 20
N_CAMS, W, H = 100, 800, 800
# HBM bytes per launch of the render kernels measured by rocprofv3 FETCH_SIZE /
# WRITE_SIZE passes (scaled by a plain copy's readings), with the hash of the
# kernel source they were taken on; a changed source makes them stale (null).
COUNTERS = os.path.join(ROOT, "profiles", "render_train_512cubed_1Mrays_counters.json")
# warm-up steps of the comparison legs (each a new trainer: its first steps
# allocate its optimiser state and segment-list buffers)
CMP_WARMUP = 5
RENDER_SRC = os.path.join(ROOT, "paper_2112_05131_amd", "csrc", "render.hip")
# kernels of one plx_render_train call, as rocprofv3 names them
COUNTED_KERNELS = {"seg_fwd": ("seg_fwd_samples_kernel", "seg_fwd_kernel", "seg_fwd_brick_kernel"),
                   "seg_combine": ("seg_combine_kernel",),
                   "seg_scatter": ("seg_scatter_kernel",)}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def source_hash(path=RENDER_SRC) -> str:
    return hashlib.sha256(open(path, "rb").read()).hexdigest()[:16]


def measured_traffic(sh_dtype, kernel):
    """(bytes per launch of `kernel`, source of the figure) from the
    committed counter summary when it was taken on this kernel source, else
    (None, reason)."""
    try:
        c = json.load(open(COUNTERS))
    except (OSError, ValueError):
        return None, "no counter summary"
    key = {B.PLX_F32: "f32", B.PLX_BF16: "bf16", B.PLX_F16: "f16"}[sh_dtype]
    e = c.get(key, {}).get(kernel)
    if not e:
        return None, f"no {key} {kernel} counters"
    if c[key].get("render_hip_sha16") != source_hash():
        return None, "stale: render.hip changed since the counters were taken"
    return e["fetch_bytes"] + e["write_bytes"], c[key].get("command", "")


def counters_summary(dtype, fetch_csv, write_csv):
    """Per-launch HBM bytes of the render kernels from the counter_collection
    CSVs of two rocprofv3 --pmc passes over `bench.py --counters` (FETCH_SIZE,
    then WRITE_SIZE; KiB per dispatch summed over the L2 channels).  The last
    dispatch of each kernel is the measured step's; the run's last dispatch is
    the 1 GiB copy, whose readings scale the counters to bytes."""
    import csv

    def per_dispatch(path, counter):
        rows = {}
        for r in csv.DictReader(open(path)):
            if r["Counter_Name"] != counter:
                continue
            d = int(r["Dispatch_Id"])
            name, val = rows.get(d, (r["Kernel_Name"], 0.0))
            rows[d] = (name, val + float(r["Counter_Value"]))
        return [rows[d] for d in sorted(rows)]

    fetch = per_dispatch(fetch_csv, "FETCH_SIZE")
    write = per_dispatch(write_csv, "WRITE_SIZE")
    copy_kib = 1 << 20  # 1 GiB read and written by the copy
    f_scale, w_scale = copy_kib / fetch[-1][1], copy_kib / write[-1][1]
    out = {"render_hip_sha16": source_hash(),
           "copy": {"kernel": fetch[-1][0][:80], "fetch_kib": fetch[-1][1], "write_kib": write[-1][1],
                    "fetch_scale": round(f_scale, 4), "write_scale": round(w_scale, 4)},
           "command": (f"rocprofv3 --pmc FETCH_SIZE (then WRITE_SIZE) --output-format csv -- python3 bench.py "
                       f"--counters --dtype {dtype}; python bench.py --counters-summary {dtype} "
                       "<fetch counter_collection.csv> <write counter_collection.csv>")}
    for key, names in COUNTED_KERNELS.items():
        fk = [(n, v) for n, v in fetch if any(x + "<" in n or x + "(" in n for x in names)]
        wk = [(n, v) for n, v in write if any(x + "<" in n or x + "(" in n for x in names)]
        if fk and wk:
            out[key] = {"kernel": fk[-1][0][:90], "fetch_kib": fk[-1][1], "write_kib": wk[-1][1],
                        "fetch_bytes": int(fk[-1][1] * 1024 * f_scale), "write_bytes": int(wk[-1][1] * 1024 * w_scale)}
    try:
        allc = json.load(open(COUNTERS))
    except (OSError, ValueError):
        allc = {}
    allc[dtype] = out
    with open(COUNTERS, "w") as f:
        json.dump(allc, f, indent=1)
    print(json.dumps(out, indent=1))


class Workload:
    """Ground truth, the resident ray pool with its targets, and the initial
    values of the trained grid."""

    def __init__(self):
        t0 = time.time()
        self.gt = synth.blob_scene(RESO, N_BLOBS, OCC, SEED, device="cuda")
        gt_grid = Grid.from_mask(self.gt.mask, RESO, self.gt.density, self.gt.sh)
        self.o, self.d = _camera_set(N_CAMS, W, H, SEED, torch.device("cuda"))
        self.t = render_rays(gt_grid, self.o, self.d)
        del gt_grid
        self.init = synth.perturbed(self.gt, seed=SEED + 1000, device="cuda")
        torch.cuda.synchronize()
        log(f"workload built in {time.time() - t0:.1f}s: M={self.gt.n_vox}, pool={self.o.shape[0]} rays")

    def grid(self, sh_dtype):
        return Grid.from_mask(self.init.mask, RESO, self.init.density, self.init.sh, sh_dtype=sh_dtype)

    def sampler(self, coherent=True, seed=SEED):
        return RaySampler(self.o, self.d, self.t, BATCH, seed=seed, coherent=coherent)


def time_steps(trainer, sampler, warmup, steps, overlap=True):
    """W untimed steps, then exactly K steps between two synchronisations;
    returns (ms per step, wall s, mean per-part ms)."""
    # the warm-up takes the timed steps' path, per-part events included (the
    # first timing events of a process are slow to create)
    trainer.run(sampler, warmup, overlap=overlap, events=[])
    # collect the previous legs' garbage (trainers, events) before, not
    # inside, the timed region
    gc.collect()
    torch.cuda.synchronize()
    evs = []
    start = torch.cuda.Event(enable_timing=True)
    end = torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    start.record()
    trainer.run(sampler, steps, overlap=overlap, events=evs)
    end.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms = start.elapsed_time(end) / steps
    parts = [e.durations() for e in evs]
    k_ms = {k: float(np.mean([p[k] for p in parts])) for k in parts[0]}
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


def cpu_model() -> str:
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(wl, batch, budget_s=12.0):
    """The FP64 oracle on a bounded sample of the same workload: fwd + MSE +
    bwd over S rays of the batch, TV on S/R of the step's segment and RMSProp
    on the sample's active voxels, timed on the host with all its threads,
    then with one thread on a smaller sample."""
    from oracle import oracle as O
    init = wl.init
    og = O.make_grid(np.array(RESO, np.int32), init.mask.cpu().numpy(), init.density.cpu().double().numpy(),
                     init.sh.cpu().double().numpy())
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

    def sized(budget):
        s = 2000
        ts_ = run(s)
        while ts_ < 0.5 * budget and s < BATCH:
            s = int(min(BATCH, s * min(8.0, budget / max(ts_, 1e-6))))
            ts_ = run(s)
        return s, ts_

    run(500)  # first touch of the grid arrays
    n0 = O.max_threads()
    s, ts_ = sized(budget_s)
    out = {"value": round(s / ts_ / 1e6, 6), "unit": "Mrays/s", "cores": n0, "kind": "oracle",
           "cpu_model": cpu_model(),
           "sample": f"{s} rays of one 1M-ray batch (fwd+MSE+bwd), TV on {s}/{BATCH} of the 1% "
                     f"segment, RMSProp on the sample's active voxels; {ts_:.1f} s FP64"}
    try:
        O.set_threads(1)
        s1, t1 = sized(budget_s / 2)
    finally:
        O.set_threads(n0)
    out["one_core"] = {"value": round(s1 / t1 / 1e6, 6), "unit": "Mrays/s", "cores": 1,
                       "sample": f"{s1} rays, {t1:.1f} s FP64"}
    log(f"oracle: {out['value']} Mrays/s on {n0} threads, {out['one_core']['value']} on 1 ({out['cpu_model']})")
    return out


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
    bins = B.make_bins(desc, o, d)
    fwd = timed(lambda: B.plx_render_fwd(desc, o, d, rgb, tau, bins=bins))
    torch.sub(rgb, t, out=g_rgb).mul_(2.0 / n)
    bwd = timed(lambda: B.plx_render_bwd(desc, o, d, g_rgb, tau, grad, touched, bins=bins))
    fwd_s = timed(lambda: B.plx_render_fwd_state(desc, o, d, rgb, tau, state, cap))
    bwd_s = timed(lambda: B.plx_render_bwd_state(desc, o, d, g_rgb, tau, state, cap, grad, touched))
    counts = state[:4 * n].view(torch.int32)
    over = int((counts > cap).sum())
    del state, grad, bins
    torch.cuda.empty_cache()
    log(f"recompute fwd {fwd:.3f} bwd {bwd:.3f} ms; stored state fwd {fwd_s:.3f} bwd {bwd_s:.3f} ms")
    return {"recompute": {"fwd_ms": round(fwd, 4), "bwd_ms": round(bwd, 4),
                          "note": "segment lists made once, outside the timed calls"},
            "stored": {"fwd_ms": round(fwd_s, 4), "bwd_ms": round(bwd_s, 4), "cap": cap,
                       "state_gb": round(B.plx_render_state_bytes(n, cap) / 1e9, 3),
                       "rays_over_cap": over}}


def prune_weight_leg(grid, batches, counts, thresh=0.01):
    """Pruning by weight on the training workload: the per-voxel maximum
    sample weight accumulated over the distinct 1M-ray batches from zeros
    (plx_render_max_weight once per batch, brick order, density only), then
    the dilated threshold count over the whole grid
    (plx_grid_prune_weight_count), timed with HIP events on the stream the
    calls are launched on (segment lists made beforehand).  Algorithmic
    bytes of one weight call: the index
    entries read (4 B each), per voxel read its density (4 B) and one
    read-modify-write of its maximum (8 B), and 24 B of ray per ray."""
    wmax = torch.zeros(grid.n_vox, device="cuda")
    keep = torch.empty(grid.n_cells, dtype=torch.uint8, device="cuda")
    desc = grid.desc()
    bins = [B.make_bins(desc, o, d) for o, d, _ in batches]
    o, d, _ = batches[0]
    B.plx_render_max_weight(desc, o, d, wmax, bins=bins[0])  # warm-up
    wmax.zero_()
    torch.cuda.synchronize()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record()
    for (o, d, _), bb in zip(batches, bins):
        B.plx_render_max_weight(desc, o, d, wmax, bins=bb)
    b.record()
    torch.cuda.synchronize()
    ms = a.elapsed_time(b) / len(batches)
    del bins
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
    roof = views_roofline(scenes)
    srv = Server(scenes, hbm_budget=1 << 30, n_streams=4, max_batch=32, keep_outputs=False,
                 max_batch_pixels=1 << 21)
    run_load(srv, random_requests(16, 8, seed=99), None)  # warm-up
    reqs = random_requests(n_sat, 8, seed=100)
    lat, wall = run_load(srv, reqs, None)
    pix = sum(r.n_pixels for r in reqs)
    sat_rps = n_sat / wall
    out = {"scenes": "4x256^3 + 4x512^3, 5-10% occupancy, FP16 SH",
           "resident_gb": round(resident / 1e9, 3),
           "saturation_mrays_s": round(pix / wall / 1e6, 2),
           "saturation_requests_s": round(sat_rps, 1), "views_kernel_roofline": roof, "loads": []}
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


def view_rays(req):
    """Rays of one view by the pinhole definition plx_render_views uses
    (FP64, rounded to FP32), on the device: for the work counters only."""
    dev = torch.device("cuda")
    c2w = torch.tensor(np.asarray(req.c2w, np.float64).reshape(3, 4), dtype=torch.float64, device=dev)
    py, px = torch.meshgrid(torch.arange(req.height, dtype=torch.float64, device=dev),
                            torch.arange(req.width, dtype=torch.float64, device=dev), indexing="ij")
    dc = torch.stack([(px + 0.5 - req.width / 2) / req.focal, -((py + 0.5 - req.height / 2) / req.focal),
                      -torch.ones_like(px)], -1).reshape(-1, 3)
    d = dc @ c2w[:, :3].T
    d = (d / d.norm(dim=1, keepdim=True)).float().contiguous()
    o = c2w[:, 3].float().expand_as(d).contiguous()
    return o, d


def views_roofline(scenes, reps=5):
    """One launch of 8 views at 1920x1080 (one per scene): its duration (HIP
    events on its stream, best of `reps`) against the algorithmic bytes of
    its rays (per view 4 U_idx + P U_occ from the work counters, 12 B of
    colour per pixel)."""
    from paper_2112_05131_amd.serve import random_requests
    reqs = random_requests(len(scenes), len(scenes), seed=77, resolutions=((1920, 1080),))
    views, nbytes, off = [], 0, 0
    P = 112 if scenes[0].sh_dtype == B.PLX_F32 else 58
    for i, r in enumerate(reqs):
        r.scene = i
        v = B.PlxView()
        v.c2w[:] = [float(x) for x in np.asarray(r.c2w, np.float64).reshape(12)]
        v.focal, v.width, v.height, v.scene, v.reserved, v.out_offset = r.focal, r.width, r.height, i, 0, off
        views.append(v)
        off += r.n_pixels
        o, d = view_rays(r)
        g = scenes[i]
        cm = torch.zeros((g.n_cells + 31) // 32, dtype=torch.int32, device="cuda")
        vm = torch.zeros((g.n_vox + 31) // 32, dtype=torch.int32, device="cuda")
        c = B.plx_render_stats(g.desc(), o, d, cm, vm)
        nbytes += 4 * c[2] + P * c[3] + 12 * r.n_pixels
        del o, d, cm, vm
    table = B.SceneTable(scenes)
    out = torch.empty(3 * off, device="cuda")
    q = B.views_queue()
    B.plx_render_views(table, views, out, q)
    best = float("inf")
    for _ in range(reps):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        B.plx_render_views(table, views, out, q)
        b.record()
        b.synchronize()
        best = min(best, a.elapsed_time(b))
    B.plx_render_views_status(q)
    gbs = nbytes / (best * 1e-3) / 1e9
    log(f"views kernel: 8 x 1920x1080 in {best:.3f} ms, {gbs:.1f} GB/s algorithmic")
    return {"launch": "8 views at 1920x1080, one per scene", "ms": round(best, 4),
            "mrays_s": round(off / best / 1e3, 2), "algorithmic_gb": round(nbytes / 1e9, 4),
            "achieved_gbs": round(gbs, 1), "frac": round(gbs / HBM_PEAK_GBS, 4),
            "bytes_model": "per view 4 U_idx + P U_occ (P = 58 B for FP16 SH) + 12 B per pixel"}


def counter_run(sh_dtype, coherent):
    """Dispatch sequence for rocprofv3 --pmc passes: two warm-up steps, one
    training step (its gather, segment lists, seg_fwd, seg_combine, seg_scatter,
    tv and rmsprop kernels), then a 1 GiB device-to-device copy (1 GiB read
    + 1 GiB written) whose counter readings give the scale of FETCH_SIZE /
    WRITE_SIZE."""
    wl = Workload()
    trainer = Trainer(wl.grid(sh_dtype), TrainConfig(), seed=SEED)
    sampler = wl.sampler(coherent)
    for _ in range(3):
        trainer.run(sampler, 1, overlap=False)
        torch.cuda.synchronize()
    src = torch.ones(1 << 28, device="cuda")
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    dst.copy_(src)
    torch.cuda.synchronize()
    log("counter run done")


def c2_leg(steps=200, warmup=200):
    """The coarse-to-fine configuration's step: 5000-ray batches on the 256^3
    grid at 10% occupancy (32 blobs, seed 1; 100 cameras at 800x800 as the
    ray pool, ground-truth renders as targets), with the next batch binned on
    the second stream and without."""
    reso = (256, 256, 256)
    gt = synth.blob_scene(reso, N_BLOBS, 0.10, 1, device="cuda")
    gt_grid = Grid.from_mask(gt.mask, reso, gt.density, gt.sh)
    o, d = _camera_set(N_CAMS, W, H, 1, torch.device("cuda"))
    t = render_rays(gt_grid, o, d)
    del gt_grid
    init = synth.perturbed(gt, seed=1001, device="cuda")
    out = {"grid": list(reso), "n_vox": gt.n_vox, "batch_rays": 5000, "steps": steps}
    for overlap in (True, False):
        g = Grid.from_mask(init.mask, reso, init.density, init.sh)
        tr = Trainer(g, TrainConfig(), seed=1)
        smp = RaySampler(o, d, t, 5000, seed=1)
        ms, wall, k = time_steps(tr, smp, warmup, steps, overlap=overlap)
        key = "overlapped" if overlap else "sequential"
        out[key] = {"ms_per_step": round(ms, 4), "mrays_s": round(5000 / ms / 1e3, 3),
                    "wall_ms_per_step": round(wall / steps * 1e3, 4),
                    "kernels_ms": {kk: round(v, 4) for kk, v in k.items()}}
        log(f"c2 {key}: {ms:.4f} ms per 5000-ray step (wall {wall / steps * 1e3:.4f})")
        del g, tr
    del o, d, t
    torch.cuda.empty_cache()
    return out


def byte_model(counts, n_rays, sh_dtype):
    """Algorithmic bytes of the forward and backward passes over one batch
    from the library's work counters (U_idx distinct index entries read,
    U_occ distinct non-NULL voxels read): forward 4 U_idx + P U_occ + 40 R
    (rays 24 B, colour 12 B, optical depth 4 B per ray), backward with
    recomputation 4 U_idx + P U_occ + 224 U_occ + 28 R (the gradient record
    read and written, rays and dL/dC), P = 112 B (FP32) or 58 B (16-bit) of
    payload per voxel."""
    P = 112 if sh_dtype == B.PLX_F32 else 58
    u_idx, u_occ = counts[2], counts[3]
    fwd = 4 * u_idx + P * u_occ + 40 * n_rays
    bwd = 4 * u_idx + P * u_occ + 224 * u_occ + 28 * n_rays
    fused = 4 * u_idx + (P + 224) * u_occ + 36 * n_rays
    return fwd, bwd, fused


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--dtype", default="f32", choices=["f32", "bf16", "f16"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-compare", action="store_true",
                    help="skip the BF16/FP16-SH, shuffled, sequential and priors steps")
    ap.add_argument("--no-serving", action="store_true", help="skip the serving latency leg")
    ap.add_argument("--no-c2", action="store_true", help="skip the 5000-ray 256^3 step leg")
    ap.add_argument("--ray-order", default="coherent", choices=["coherent", "random"],
                    help="order of the rays inside each batch (the same rays either way)")
    ap.add_argument("--counters", action="store_true",
                    help="for counter runs under rocprofv3: warm-up steps and one training "
                         "step, then a 1 GiB device copy that calibrates the byte counters; "
                         "prints no JSON line")
    ap.add_argument("--counters-summary", nargs=3, metavar=("DTYPE", "FETCH_CSV", "WRITE_CSV"),
                    help="write the per-kernel HBM bytes of two --counters passes (rocprofv3 "
                         "counter_collection.csv files) into the committed counter summary")
    ap.add_argument("--serving-only", action="store_true",
                    help="for trace runs under rocprofv3: only the serving leg, printed as its "
                         "own JSON object")
    args = ap.parse_args()
    if args.counters_summary:
        counters_summary(*args.counters_summary)
        return
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
    coherent = args.ray_order == "coherent"
    wl = Workload()
    grid = wl.grid(sh_dtype)
    trainer = Trainer(grid, TrainConfig(), seed=SEED)
    # the first batch of the timed run's sampler, for the work counters
    batch0 = wl.sampler(coherent).next_batch()
    counts = work_counters(grid, batch0)
    n_act, tv_cells = active_count(trainer, batch0)
    log(f"counters: samples={counts[0]} occupied_samples={counts[1]} U_idx={counts[2]} "
        f"U_occ={counts[3]} active={n_act}")

    ms, wall, k_ms = time_steps(trainer, wl.sampler(coherent), args.warmup, args.steps)
    mrays = BATCH / (ms * 1e-3) / 1e6
    log(f"step {ms:.3f} ms (wall {wall / args.steps * 1e3:.3f} ms/step); kernels ms: "
        + ", ".join(f"{k} {v:.3f}" for k, v in k_ms.items()))

    fwd_b, bwd_b, fused_b = byte_model(counts, BATCH, sh_dtype)
    rec_b = 32 * counts[1]  # sample records: written by seg_fwd, read by seg_scatter
    gbs = lambda b, t_ms: b / (t_ms * 1e-3) / 1e9  # noqa: E731
    # the dominant kernel of the fused call and its algorithmic bytes
    if k_ms["seg_fwd"] >= k_ms["seg_bwd"]:
        dom, dom_ms, dom_b = "seg_fwd", k_ms["seg_fwd"], fwd_b
        dom_desc = "seg_fwd (segment forward of plx_render_train, recording the occupied samples)"
        dom_model = "forward: 4 U_idx + P U_occ + 40 R"
    else:
        dom, dom_ms, dom_b = "seg_scatter", k_ms["seg_bwd"], bwd_b
        dom_desc = "seg_scatter (recorded backward of plx_render_train: recurrence + per-voxel sums)"
        dom_model = "backward with recomputation: 4 U_idx + P U_occ + 224 U_occ + 28 R"
    achieved = gbs(dom_b, dom_ms)
    traffic, traffic_src = measured_traffic(sh_dtype, dom)
    alg_rms = n_act * (672 if sh_dtype == B.PLX_F32 else 726)
    alg_tv = 16 * tv_cells
    step_gbs = gbs(fwd_b + bwd_b + alg_rms + alg_tv, ms)

    def frac(b, t_ms):
        return {"ms": round(t_ms, 4), "algorithmic_gb": round(b / 1e9, 4),
                "achieved_gbs": round(gbs(b, t_ms), 1), "frac": round(gbs(b, t_ms) / HBM_PEAK_GBS, 4)}

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
                        "1M-ray batches from all pixels of 100 cameras at 800x800; step = batch "
                        "gather + segment lists (next batch on a second stream) + fused "
                        "render+MSE+backward + TV on a 1% contiguous segment + sparse RMSProp",
            "sh_storage": args.dtype,
            "batch_rays": BATCH,
            "ray_order": args.ray_order,
            "grid": list(RESO),
            "n_vox": grid.n_vox,
        },
        "roofline": {
            "bound": "hbm",
            "kernel": dom_desc,
            "achieved": round(achieved, 1),
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4),
            "traffic": round(traffic / 1e9, 3) if traffic else None,
            "traffic_unit": "GB per launch (rocprofv3 FETCH_SIZE + WRITE_SIZE, copy-scaled)",
            "traffic_source": traffic_src,
            "algorithmic_gb": round(dom_b / 1e9, 4),
            "bytes_model": dom_model,
        },
        "kernels": {
            "seg_fwd": dict(frac(fwd_b, k_ms["seg_fwd"]), bytes_model="forward: 4 U_idx + P U_occ + 40 R",
                            sample_records_written_gb=round(rec_b / 1e9, 4)),
            "seg_scatter": dict(frac(bwd_b, k_ms["seg_bwd"]),
                                bytes_model="backward with recomputation: 4 U_idx + P U_occ + 224 U_occ + 28 R",
                                sample_records_read_gb=round(rec_b / 1e9, 4)),
            "seg_combine_ms": round(k_ms["seg_combine"], 4),
            "render_train_call": dict(frac(fwd_b + bwd_b, k_ms["render_train"]),
                                      bytes_model="forward + backward with recomputation"),
            "render_train_call_fused_model": dict(frac(fused_b, k_ms["render_train"]),
                                                  bytes_model="4 U_idx + (P + 224) U_occ + 36 R: one "
                                                              "read of each voxel for the whole call"),
            "tv_grad_ms": round(k_ms["tv"], 4),
            "rmsprop_step": frac(alg_rms, k_ms["rmsprop"]),
            "bins_ms_second_stream": round(k_ms.get("bins", 0.0), 4),
        },
        "step_hbm_gbs_algorithmic": round(step_gbs, 1),
        "work": {"samples": counts[0], "occupied_samples": counts[1], "index_entries": counts[2],
                 "voxels_read": counts[3], "active_voxels": n_act, "tv_cells": tv_cells},
    }
    if not args.no_compare:
        # the same step with SH stored in FP32, BF16 and FP16 (FP32 optimiser
        # state and accumulation in all three), the same batches
        prec = {args.dtype: {"ms_per_step": round(ms, 4), "mrays_s": round(mrays, 3),
                             "render_train_ms": round(k_ms["render_train"], 4),
                             "seg_fwd_ms": round(k_ms["seg_fwd"], 4), "seg_scatter_ms": round(k_ms["seg_bwd"], 4)}}
        for name in ("f32", "bf16", "f16"):
            if name in prec:
                continue
            tr2 = Trainer(wl.grid(B.DTYPES[name]), TrainConfig(), seed=SEED)
            ms2, _, k2 = time_steps(tr2, wl.sampler(coherent), CMP_WARMUP, max(5, args.steps))
            prec[name] = {"ms_per_step": round(ms2, 4), "mrays_s": round(BATCH / ms2 / 1e3, 3),
                          "render_train_ms": round(k2["render_train"], 4),
                          "seg_fwd_ms": round(k2["seg_fwd"], 4), "seg_scatter_ms": round(k2["seg_bwd"], 4)}
            log(f"{name}: step {ms2:.3f} ms, render_train {k2['render_train']:.3f} ms")
            del tr2
        for name in prec:
            prec[name]["speedup_vs_f32"] = round(prec["f32"]["ms_per_step"] / prec[name]["ms_per_step"], 4)
        out["precision"] = prec
        if coherent:
            # the same pixels, each batch in the permutation's order
            tr3 = Trainer(wl.grid(sh_dtype), TrainConfig(), seed=SEED)
            ms3, _, k3 = time_steps(tr3, wl.sampler(False), CMP_WARMUP, max(5, args.steps))
            out["random_order"] = {"ms_per_step": round(ms3, 4), "mrays_s": round(BATCH / ms3 / 1e3, 3),
                                   "render_train_ms": round(k3["render_train"], 4)}
            log(f"random ray order: step {ms3:.3f} ms, render_train {k3['render_train']:.3f} ms")
            del tr3
        # the segment lists made on the training stream itself (their count's
        # synchronisation then stalls the device once per step)
        tr5 = Trainer(wl.grid(sh_dtype), TrainConfig(), seed=SEED)
        ms5, _, k5 = time_steps(tr5, wl.sampler(coherent), CMP_WARMUP, max(5, args.steps), overlap=False)
        out["sequential_binning"] = {"ms_per_step": round(ms5, 4), "mrays_s": round(BATCH / ms5 / 1e3, 3)}
        log(f"sequential binning: step {ms5:.3f} ms")
        del tr5
        # the same step with the sparsity and beta priors of Sec. 3.7 on (the
        # paper's 360-degree weights)
        tr4 = Trainer(wl.grid(sh_dtype), TrainConfig(lambda_sparsity=1e-11, lambda_beta=1e-5), seed=SEED)
        ms4, _, k4 = time_steps(tr4, wl.sampler(coherent), CMP_WARMUP, max(5, args.steps))
        out["with_priors"] = {"lambda_sparsity": 1e-11, "lambda_beta": 1e-5, "ms_per_step": round(ms4, 4),
                              "mrays_s": round(BATCH / ms4 / 1e3, 3),
                              "render_train_ms": round(k4["render_train"], 4)}
        log(f"with priors: step {ms4:.3f} ms, render_train {k4['render_train']:.3f} ms")
        del tr4
        out["backward_state"] = state_leg(grid, batch0, args.steps)
    smp = wl.sampler(coherent, seed=SEED + 5)
    out["prune_by_weight"] = prune_weight_leg(grid, [smp.next_batch() for _ in range(4)], counts)
    if not args.no_c2:
        out["c2_step"] = c2_leg()
    if not args.no_serving:
        out["serving"] = serving_leg()
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(wl, batch0)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
