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
GRAD_RTOL = 1e-4         # per element, relative part
GRAD_FLOOR = 1e-3        # floor (times max |ref| of the group) where no mass is given
# A float32 evaluation of a gradient sum differs from the exact one by a small
# multiple of the unit roundoff (6e-8) times the sum of the absolute terms
# (orc_render_bwd_mass); each term carries a few roundings of exp/products and
# of the running sums, so the per-term factor is bounded by 4e-6.
GRAD_MASS = 4e-6
# A float32 pre-activation (trilinear sum and SH dot product, about 20
# roundings) is within 20 * 6e-8 < 1e-5 of the exact one relative to the sum
# of its absolute terms; within that band a ReLU gate may close on either side.
GATE_REL = 1e-5
# Below FLT_MIN = 2^-126 float32 has no relative precision (subnormals carry
# fewer bits, and may be flushed): no float32 result is closer than that.
FLT_MIN = 1.1754943508222875e-38


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


def occupancy_cells(occ_words: torch.Tensor, reso) -> np.ndarray:
    """The cell bitmap of an occupancy structure as a bool array [Nx, Ny, Nz]
    over lower corners (brick-major layout: 512 bits per 8^3 brick, cell
    (i,j,k) at bit (i%8)*64 + (j%8)*8 + k%8 of brick (i/8, j/8, k/8))."""
    nx, ny, nz = reso
    bx, by, bz = [-(-(r - 1) // 8) for r in reso]
    bits = bits_to_bool(occ_words, bx * by * bz * 512).reshape(bx, by, bz, 8, 8, 8)
    full = bits.transpose(0, 3, 1, 4, 2, 5).reshape(bx * 8, by * 8, bz * 8)
    out = np.zeros(reso, bool)
    out[:nx - 1, :ny - 1, :nz - 1] = full[:nx - 1, :ny - 1, :nz - 1]
    return out


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


def grad_mass(og, o, d, g_rgb, bg=(1.0, 1.0, 1.0), chain_rays=None):
    """Tolerance inputs from the oracle: the absolute-term mass of the
    gradient for dL/dC = g_rgb, plus (for fused training, where dL/dC is
    formed on the device from its own colours) the RGB tolerance carried
    through dL/dC = 2(C - target)/R: the mass for |dL/dC| = 2 RGB_ATOL / R."""
    plain_d, plain_s = O.render_bwd_mass(og, o, d, np.abs(g_rgb), bg)
    # terms behind gates that float32 may decide either way count in full
    amb_d, amb_s = O.render_bwd_mass(og, o, d, np.abs(g_rgb), bg, gate_rel=GATE_REL)
    md = GRAD_MASS * plain_d + (amb_d - plain_d)
    ms = GRAD_MASS * plain_s + (amb_s - plain_s)
    if chain_rays:
        cd, cs = O.render_bwd_mass(og, o, d, np.full((o.shape[0], 3), 2.0 * RGB_ATOL / chain_rays),
                                   bg, gate_rel=GATE_REL)
        md, ms = md + cd, ms + cs
    return md, ms


def assert_grads_close(gpu_rec, ref_d, ref_s, what="", mass=None):
    """|gpu - ref| <= GRAD_RTOL |ref| + extra per element, where extra is the
    conditioning term from grad_mass when given, else GRAD_RTOL * GRAD_FLOOR *
    max|ref| of the group.  Returns the worst err/tol and relative L2 error."""
    gd, gs = split_records(gpu_rec)
    stats = {}
    for gi, (name, a, b) in enumerate((("sigma", gd, ref_d), ("sh", gs, ref_s))):
        mx = float(np.abs(b).max()) if b.size else 0.0
        extra = mass[gi] if mass is not None else GRAD_RTOL * GRAD_FLOOR * mx
        tol = GRAD_RTOL * np.abs(b) + extra + FLT_MIN
        err = np.abs(a - b)
        bad = err > tol
        rel = float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))
        worst = float((err / np.maximum(tol, 1e-300)).max()) if err.size else 0.0
        # the plain relative criterion with a floor of 1e-3 of the group's
        # largest value, reported beside the mass criterion above (which is
        # the one asserted): where they disagree, a sum cancels
        o10 = GRAD_RTOL * (np.abs(b) + GRAD_FLOOR * mx) + FLT_MIN
        o10_worst = float((err / o10).max()) if err.size else 0.0
        stats[name] = dict(max_ref=mx, max_err=float(err.max()) if err.size else 0.0,
                           rel_l2=rel, worst_ratio=worst, floor_rel_worst=o10_worst,
                           floor_rel_over=int((err > o10).sum()))
        assert not bad.any(), (
            f"{what} {name}: {int(bad.sum())} of {bad.size} elements outside tolerance; "
            f"worst err {float(err.max()):.3e} at ref {float(b.reshape(-1)[np.argmax((err - tol).reshape(-1))]):.3e}, "
            f"max|ref| {mx:.3e}, worst err/tol {worst:.2f}")
    say(f"  {what}: " + ", ".join(f"{k} rel_l2={v['rel_l2']:.2e} worst_err/tol={v['worst_ratio']:.3f} "
                                  f"(floor-relative: worst {v['floor_rel_worst']:.3f}, "
                                  f"{v['floor_rel_over']} over)"
                                  for k, v in stats.items()))
    return stats


def assert_touched_equal(gpu_bytes, ref_touched, what=""):
    """The touched map (one byte per voxel) equals the oracle's active set."""
    n = ref_touched.shape[0]
    b = gpu_bytes.cpu().numpy()
    assert b.shape[0] == n, f"{what}: touched map has {b.shape[0]} bytes for {n} voxels"
    assert np.isin(b, (0, 1)).all(), f"{what}: touched bytes other than 0/1"
    got = b.astype(bool)
    ref = ref_touched.astype(bool)
    assert got.sum() == ref.sum(), f"{what}: touched count {got.sum()} vs {ref.sum()}"
    assert np.array_equal(got, ref), f"{what}: touched sets differ"
