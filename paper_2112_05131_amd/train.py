"""Training driver: one optimisation step = fused render/MSE/backward over a
ray batch, TV on a random contiguous segment of cells, and sparse RMSProp
(Sec. 3.5; hyper-parameters of supplement B.1/B.2).  Host code only chooses
scalars (learning rates, the TV segment) and enqueues library calls."""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np
import torch

from . import binding as B
from .grid import Grid


@dataclass
class TrainConfig:
    # learning-rate schedules (supplement B.1)
    lr_sigma0: float = 30.0
    lr_sigma1: float = 0.05
    lr_sh0: float = 1e-2
    lr_sh1: float = 5e-6
    lr_max_steps: int = 250000
    lr_sigma_delay_steps: int = 15000
    lr_sigma_delay_mult: float = 0.01
    # RMSProp
    beta: float = 0.95
    eps: float = 1e-8
    # TV (synthetic-scene weights, supplement B.2); applied on tv_fraction of
    # the cells per step
    lambda_tv_sigma: float = 1e-5
    lambda_tv_sh: float = 1e-3
    tv_fraction: float = 0.01
    tv_eps: float = 1e-9
    background: tuple = (1.0, 1.0, 1.0)
    # optional priors of Sec. 3.7 (0 = off; 1e-11 and 1e-5 on the paper's
    # 360-degree scenes, supplement B.1)
    lambda_sparsity: float = 0.0
    lambda_beta: float = 0.0
    beta_eps: float = 1e-3
    # MSI background of 360-degree scenes (used when the trainer has one):
    # pure exponential decay of its learning rates (supplement B.1: no delay
    # for the background), and the colour behind its last sphere
    lr_bg_sigma0: float = 3.0
    lr_bg_sigma1: float = 0.05
    lr_bg_color0: float = 1e-2
    lr_bg_color1: float = 5e-6
    bg_background: tuple = (0.0, 0.0, 0.0)
    # TV of the background (wrapping its azimuth), on tv_fraction of its cells
    # (supplement B.1: 1e-3 for both on the 360-degree scenes)
    lambda_tv_bg_sigma: float = 1e-3
    lambda_tv_bg_color: float = 1e-3


class RaySampler:
    """Training batches over a fixed set of rays (all pixels of the training
    cameras) and their target colours.  Each epoch visits every ray once, in
    a seeded random order: batches are consecutive slices of a fresh
    permutation (supplement B.1: 5000-ray batches).  With coherent=True the
    rays of each batch are listed in increasing storage order; the batch holds
    the same rays, but neighbouring rays then run on neighbouring wavefronts
    (store the rays camera by camera, pixels in a spatially coherent order).
    The rays stay resident on the device; a batch is a gather."""

    def __init__(self, rays_o: torch.Tensor, rays_d: torch.Tensor, target: torch.Tensor,
                 batch: int, seed: int = 0, coherent: bool = True):
        if not (rays_o.shape == rays_d.shape == target.shape and rays_o.shape[-1] == 3):
            raise ValueError("rays_o, rays_d and target must all be [N, 3]")
        if batch < 1:
            raise ValueError("batch must be positive")
        self.o, self.d, self.t = rays_o, rays_d, target
        self.n = rays_o.shape[0]
        self.batch = int(batch)
        self.coherent = coherent
        self.gen = torch.Generator(device=rays_o.device)
        self.gen.manual_seed(int(seed))
        self.epoch = -1
        self._perm = None
        self._pos = self.n

    def batch_buffers(self):
        """Device buffers that next_batch(out=...) fills: the batch's rays and
        targets, and the sorted ray ids (values, positions)."""
        dev, b = self.o.device, self.batch
        return (torch.empty(b, 3, dtype=self.o.dtype, device=dev), torch.empty(b, 3, dtype=self.d.dtype, device=dev),
                torch.empty(b, 3, dtype=self.t.dtype, device=dev), torch.empty(b, dtype=torch.int64, device=dev),
                torch.empty(b, dtype=torch.int64, device=dev))

    def next_batch(self, out=None):
        """(rays_o, rays_d, target) of the next batch: new tensors, or the
        first three of `out` (batch_buffers()) filled in place."""
        if self._pos + self.batch > self.n:
            # a new epoch; a short tail of the previous permutation is dropped
            self._perm = torch.randperm(self.n, device=self.o.device, generator=self.gen)
            self._pos = 0
            self.epoch += 1
        ids = self._perm[self._pos:self._pos + self.batch]
        self._pos += self.batch
        if out is None:
            if self.coherent:
                ids = torch.sort(ids).values
            return self.o[ids], self.d[ids], self.t[ids]
        o, d, t, sv, si = out
        if self.coherent:
            torch.sort(ids, out=(sv, si))
            ids = sv
        torch.index_select(self.o, 0, ids, out=o)
        torch.index_select(self.d, 0, ids, out=d)
        torch.index_select(self.t, 0, ids, out=t)
        return o, d, t


# Batches from this size on use the recorded backward (sample buffer and one
# scatter workgroup per brick).  Smaller batches put few segments in each
# brick, so the per-brick set-up of the scatter outweighs what it saves on
# atomics, and the replay's own scatter is faster: at 5000-ray batches on a
# 256^3 grid a step takes 0.62 ms with it and 0.79 ms with the recorded one.
RECORDED_MIN_RAYS = 1 << 16


def recorded_backward(n_rays: int) -> bool:
    return n_rays >= RECORDED_MIN_RAYS


class StepEvents:
    """Device events around the calls of one training step (timing only):
    the binning of its batch (on the stream that made the bins), the four
    events the fused render call records between its kernels (before the
    segment forward, after it, after the per-ray combine, after the segment
    backward), and the ends of TV and of RMSProp."""

    def __init__(self):
        ev = lambda: torch.cuda.Event(enable_timing=True)  # noqa: E731
        self.bins = [ev(), ev()]
        self.render = [ev() for _ in range(4)]
        self.tv = ev()
        self.rmsprop = ev()
        self.binned = False

    def durations(self) -> dict:
        """Milliseconds of each part (after a synchronisation)."""
        r = self.render
        out = {"seg_fwd": r[0].elapsed_time(r[1]), "seg_combine": r[1].elapsed_time(r[2]),
               "seg_bwd": r[2].elapsed_time(r[3]), "render_train": r[0].elapsed_time(r[3]),
               "tv": r[3].elapsed_time(self.tv), "rmsprop": self.tv.elapsed_time(self.rmsprop)}
        if self.binned:
            out["bins"] = self.bins[0].elapsed_time(self.bins[1])
        return out


class Trainer:
    """Holds the optimiser state of one grid (and of an optional MSI
    background grid) and runs training steps."""

    def __init__(self, grid: Grid, cfg: TrainConfig | None = None, seed: int = 0,
                 background: Grid | None = None):
        self.cfg = cfg or TrainConfig()
        self.rng = np.random.default_rng(seed)
        self.step_id = 0
        # the two alternating sets of segment-list buffers of run() and the
        # completion events of the steps that last used them, kept across
        # calls so that a new call neither allocates them again nor refills
        # a set that a step of the previous call may still be reading
        self._run_bufs = [[None, None, None], [None, None, None]]
        self._run_batch = [None, None]  # batch buffers of each set (RaySampler.batch_buffers)
        self._run_done = [None, None]
        self._side = None  # run()'s second stream
        self.set_grid(grid)
        self.set_background(background)

    def set_background(self, bg: Grid | None):
        """Attach an MSI background grid (reso (L, H, W), FP32 records); its
        optimiser state starts from zero."""
        self.bg = bg
        self._bg_bufs = None
        if bg is not None:
            m = bg.n_vox
            self.bg_grad = torch.zeros(m, B.REC_SLOTS, dtype=torch.float32, device=bg.device)
            self.bg_vstate = torch.zeros(m, B.REC_SLOTS, dtype=torch.float32, device=bg.device)
            self.bg_touched = torch.zeros(m, dtype=torch.uint8, device=bg.device)

    def _bg_buffers(self, n):
        if self._bg_bufs is None or self._bg_bufs[0].shape[0] != n:
            dev = self.bg.device
            self._bg_bufs = (torch.empty(n, 3, device=dev), torch.empty(n, 3, device=dev))
        return self._bg_bufs

    def set_grid(self, grid: Grid):
        """Attach a (new) grid; the optimiser state starts from zero."""
        self.grid = grid
        dev = grid.device
        m = grid.n_vox
        self.grad = torch.zeros(m, B.REC_SLOTS, dtype=torch.float32, device=dev)
        self.vstate = torch.zeros(m, B.REC_SLOTS, dtype=torch.float32, device=dev)
        self.touched = torch.zeros(m, dtype=torch.uint8, device=dev)
        self.loss_sum = torch.zeros(1, dtype=torch.float64, device=dev)
        self.tv_loss_sum = torch.zeros(1, dtype=torch.float64, device=dev)
        self.prior_loss_sum = torch.zeros(2, dtype=torch.float64, device=dev)

    def learning_rates(self, step=None):
        c = self.cfg
        t = self.step_id if step is None else step
        lr_s = B.plx_lr_schedule(t, c.lr_sigma0, c.lr_sigma1, c.lr_max_steps,
                                 c.lr_sigma_delay_steps, c.lr_sigma_delay_mult)
        lr_h = B.plx_lr_schedule(t, c.lr_sh0, c.lr_sh1, c.lr_max_steps)
        return lr_s, lr_h

    def priors(self):
        """The sparsity and beta priors of the configuration (None if off);
        their losses accumulate in prior_loss_sum."""
        c = self.cfg
        if c.lambda_sparsity == 0.0 and c.lambda_beta == 0.0:
            return None
        return B.Priors(c.lambda_sparsity, c.lambda_beta, c.beta_eps, self.prior_loss_sum)

    def tv_segment(self):
        n = self.grid.n_cells
        count = max(1, int(math.ceil(self.cfg.tv_fraction * n)))
        start = int(self.rng.integers(0, n))
        return start, count

    def step(self, rays_o, rays_d, target, tv: bool = True, rgb_out=None, bins=None,
             events: StepEvents | None = None):
        """One optimisation step on a ray batch (all device tensors).  bins:
        the batch's segment lists (binding.make_bins), made here when not
        given; events: recorded around the step's calls when given."""
        c, g = self.cfg, self.grid
        lr_s, lr_h = self.learning_rates()
        n = rays_o.shape[0]
        rev = events.render if events is not None else None
        if bins is None:
            bins = B.make_bins(g.desc(), rays_o, rays_d, samples=recorded_backward(n))
        if self.bg is None:
            B.plx_render_train(g.desc(), rays_o, rays_d, target, 1.0 / max(n, 1), self.grad,
                               self.touched, self.loss_sum, rgb_out, c.background, self.priors(),
                               bins=bins, events=rev)
        else:
            # background colours -> fused foreground step (which hands back
            # their gradient) -> background gradient
            cbg, gbg = self._bg_buffers(n)
            B.plx_bg_render_fwd(self.bg.desc(), rays_o, rays_d, cbg, None, c.bg_background)
            B.plx_render_train(g.desc(), rays_o, rays_d, target, 1.0 / max(n, 1), self.grad,
                               self.touched, self.loss_sum, rgb_out, cbg, self.priors(), gbg,
                               bins=bins, events=rev)
            B.plx_bg_render_bwd(self.bg.desc(), rays_o, rays_d, gbg, self.bg_grad, self.bg_touched,
                                c.bg_background)
        if tv and (c.lambda_tv_sigma > 0 or c.lambda_tv_sh > 0):
            start, count = self.tv_segment()
            B.plx_tv_grad(g.desc(), start, count, c.lambda_tv_sigma, c.lambda_tv_sh, c.tv_eps,
                          self.grad, self.touched, self.tv_loss_sum)
        if events is not None:
            events.tv.record()
        B.plx_rmsprop_step(g.desc(), g.master, self.vstate, self.grad, self.touched, lr_s, lr_h,
                           c.beta, c.eps)
        if events is not None:
            events.rmsprop.record()
        if self.bg is not None:
            if tv and (c.lambda_tv_bg_sigma > 0 or c.lambda_tv_bg_color > 0):
                nb = self.bg.n_cells
                count = max(1, int(math.ceil(c.tv_fraction * nb)))
                B.plx_bg_tv_grad(self.bg.desc(), int(self.rng.integers(0, nb)), count, c.lambda_tv_bg_sigma,
                                 c.lambda_tv_bg_color, c.tv_eps, self.bg_grad, self.bg_touched, self.tv_loss_sum)
            t = self.step_id
            lr_bs = B.plx_lr_schedule(t, c.lr_bg_sigma0, c.lr_bg_sigma1, c.lr_max_steps)
            lr_bc = B.plx_lr_schedule(t, c.lr_bg_color0, c.lr_bg_color1, c.lr_max_steps)
            B.plx_rmsprop_step(self.bg.desc(), None, self.bg_vstate, self.bg_grad, self.bg_touched, lr_bs, lr_bc,
                               c.beta, c.eps)
        self.step_id += 1

    def run(self, sampler: RaySampler, n_steps: int, overlap: bool = True, tv: bool = True,
            events: list | None = None):
        """n_steps optimisation steps on consecutive batches of the sampler.

        With overlap, batch t+1 is gathered and binned on a second stream
        while step t runs on the current one: the binning reads only the rays
        and the grid's occupancy, which a step does not change, and its one
        synchronising call (the segment count) then waits for that stream
        alone, so the device never idles on it.  The two sets of batch and
        segment-list buffers alternate (kept by the trainer, so that a step
        allocates nothing once both exist); a set is refilled only after the
        step that used it has finished.  events: a list that gets one
        StepEvents per step."""
        if n_steps <= 0:
            return
        main = torch.cuda.current_stream()
        if overlap and (self._side is None or self._side.device != self.grid.device):
            # one second stream per trainer: a new stream per call costs the
            # runtime a queue set-up at the start of the first calls
            self._side = torch.cuda.Stream(device=self.grid.device)
        side = self._side if overlap else main
        bufs = self._run_bufs
        done = self._run_done

        def prepare(slot):
            se = StepEvents() if events is not None else None
            with torch.cuda.stream(side):
                if done[slot] is not None:
                    side.wait_event(done[slot])
                if se is not None:
                    se.bins[0].record(side)
                bb = self._run_batch[slot]
                if bb is None or bb[0].shape[0] != sampler.batch or bb[0].device != sampler.o.device:
                    bb = self._run_batch[slot] = sampler.batch_buffers()
                o, d, t = sampler.next_batch(out=bb)
                b = B.make_bins(self.grid.desc(), o, d, *bufs[slot], samples=recorded_backward(o.shape[0]))
                bufs[slot] = b.buffers()
                if se is not None:
                    se.bins[1].record(side)
                    se.binned = True
                ev = torch.cuda.Event()
                ev.record(side)
            return o, d, t, b, ev, se

        nxt = prepare(0)
        for i in range(n_steps):
            o, d, t, b, ev, se = nxt
            if side is not main:
                main.wait_event(ev)
                for x in (o, d, t, *b.buffers()):
                    if x is not None:
                        x.record_stream(main)
            self.step(o, d, t, tv=tv, bins=b, events=se)
            if events is not None:
                events.append(se)
            ev_done = torch.cuda.Event()
            ev_done.record(main)
            done[i % 2] = ev_done
            if i + 1 < n_steps:
                nxt = prepare((i + 1) % 2)
