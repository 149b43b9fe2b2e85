"""Helpers of the GPU parity tests: build the GPU grid and the oracle grid
from the same generator output, read GPU results back, and apply the stated
tolerances.  (Plumbing only; neither side's arithmetic lives here.)"""
import sys

import numpy as np
import torch

from oracle import oracle as O
from paper_2112_05131_amd import binding as B
from paper_2112_05131_amd.grid import Grid

RGB_ATOL = 1e-5          # per channel per ray, FP32 path
GRAD_RTOL = 1e-4         # per element, with a floor of GRAD_FLOOR * max |ref| per group
GRAD_FLOOR = 1e-3


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def rounded_sh(sh: torch.Tensor, sh_dtype: int) -> torch.Tensor:
    """SH coefficients as the 16-bit storage holds them (CPU, round to
    nearest even), float64."""
    if sh_dtype == B.PLX_BF16:
        return sh.cpu().to(torch.bfloat16).double()
    if sh_dtype == B.PLX_F16:
        return sh.cpu().to(torch.float16).double()
    return sh.cpu().double()


def make_pair(sv, sh_dtype=B.PLX_F32, lo=(-0.5,) * 3, hi=(0.5,) * 3, step_voxels=0.5):
    """(oracle grid, GPU grid) from one synth.SceneValues."""
    og = O.make_grid(np.array(sv.reso, np.int32), sv.mask.cpu().numpy(),
                     sv.density.cpu().double().numpy(),
                     rounded_sh(sv.sh, sh_dtype).numpy(), lo, hi, step_voxels)
    gg = Grid.from_mask(sv.mask.cuda(), sv.reso, sv.density.cuda(), sv.sh.cuda(), sh_dtype=sh_dtype,
                        lo=lo, hi=hi, step_voxels=step_voxels)
    return og, gg


def bits_to_bool(words: torch.Tensor, n: int) -> np.ndarray:
    w = words.cpu().numpy().astype(np.int32).view(np.uint8)
    return np.unpackbits(w, bitorder="little")[:n].astype(bool)


def gpu_render(gg, o, d, bg=(1.0, 1.0, 1.0)):
    n = o.shape[0]
    rgb = torch.empty(n, 3, dtype=torch.float32, device="cuda")
    tau = torch.empty(n, dtype=torch.float32, device="cuda")
    B.plx_render_fwd(gg.desc(), o.cuda().contiguous(), d.cuda().contiguous(), rgb, tau, bg)
    torch.cuda.synchronize()
    return rgb.cpu().double().numpy(), tau.cpu().double().numpy()


def split_records(rec: torch.Tensor):
    """(density [M], sh [M,27]) float64 numpy from FP32 records."""
    r = rec.detach().cpu().double().numpy()
    return r[:, B.SLOT_SIGMA].copy(), r[:, :B.NSH].copy()


def assert_grads_close(gpu_rec, ref_d, ref_s, what=""):
    gd, gs = split_records(gpu_rec)
    stats = {}
    for name, a, b in (("sigma", gd, ref_d), ("sh", gs, ref_s)):
        mx = float(np.abs(b).max()) if b.size else 0.0
        tol = GRAD_RTOL * (np.abs(b) + GRAD_FLOOR * mx)
        err = np.abs(a - b)
        bad = err > tol
        rel = float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))
        stats[name] = (mx, float(err.max()) if err.size else 0.0, rel)
        assert not bad.any(), (
            f"{what} {name}: {int(bad.sum())} of {bad.size} elements outside tolerance; "
            f"worst err {float(err.max()):.3e} at ref {float(b.reshape(-1)[np.argmax((err - tol).reshape(-1))]):.3e}, "
            f"max|ref| {mx:.3e}")
    return stats


def assert_touched_equal(gpu_words, ref_touched, what=""):
    n = ref_touched.shape[0]
    got = bits_to_bool(gpu_words, n)
    ref = ref_touched.astype(bool)
    assert got.sum() == ref.sum(), f"{what}: touched count {got.sum()} vs {ref.sum()}"
    assert np.array_equal(got, ref), f"{what}: touched sets differ"
    # no bits beyond n
    w = gpu_words.cpu().numpy().astype(np.int32).view(np.uint8)
    assert not np.unpackbits(w, bitorder="little")[n:].any()
