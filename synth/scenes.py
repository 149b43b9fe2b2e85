"""Seeded synthetic inputs shared by the oracle tests, the GPU parity tests
and the benchmark.

This module only *draws inputs*: occupancy masks, per-voxel parameter values,
camera poses and rays.  It contains none of the rendering, gradient, TV,
optimiser or grid arithmetic of the method, so that neither side of a parity
test can borrow the other's maths through it.

Scenes stand in for the paper's NeRF-synthetic data (not available here):
isotropic Gaussian density blobs in the unit cube [-0.5, 0.5]^3 with peak
density sigma_max, per-blob colour coefficients, and cameras on a sphere of
radius 2 looking at the origin with a 45 degree pinhole and pixel-centred rays.
Forward-facing captures (the LLFF scenes) are stood in for by cameras spread
over a small square of the plane z = 0, looking along -z with small tilts;
their scene values fill a grid over the NDC cube.

Everything is computed in float64 with torch (CPU or GPU) and rounded to
float32 once; a test generates its inputs once and feeds the same arrays to
both sides.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np
import torch

NSH = 27


@dataclass
class SceneValues:
    """An occupancy mask and the values of its occupied voxels in increasing
    storage order (z fastest)."""

    reso: tuple
    mask: torch.Tensor  # uint8 [Nx*Ny*Nz]
    density: torch.Tensor  # float32 [M]
    sh: torch.Tensor  # float32 [M, 27] channel-major
    n_vox: int


def _gen(seed: int) -> torch.Generator:
    g = torch.Generator(device="cpu")
    g.manual_seed(int(seed))
    return g


def blob_params(n_blobs: int, seed: int):
    """Blob centres U([-0.25,0.25]^3), std U(0.03,0.08), DC colour
    coefficients U(0.35, 3.2) per channel, higher-order coefficients
    U(-0.05, 0.05)."""
    g = _gen(seed)
    mu = (torch.rand(n_blobs, 3, generator=g, dtype=torch.float64) - 0.5) * 0.5
    std = 0.03 + 0.05 * torch.rand(n_blobs, generator=g, dtype=torch.float64)
    sh = (torch.rand(n_blobs, 3, 9, generator=g, dtype=torch.float64) - 0.5) * 0.1
    dc = 0.35 + 2.85 * torch.rand(n_blobs, 3, generator=g, dtype=torch.float64)
    sh[:, :, 0] = dc
    return mu, std, sh.reshape(n_blobs, NSH)


def _centres(n: int, device) -> torch.Tensor:
    # voxel centres of n voxels spanning [-0.5, 0.5]
    return (torch.arange(n, device=device, dtype=torch.float64) + 0.5) / n - 0.5


def blob_scene(reso, n_blobs: int, occupancy: float, seed: int, sigma_max: float = 50.0,
               device="cpu") -> SceneValues:
    """Density sigma(x) = sigma_max * max_b exp(-|x - mu_b|^2 / (2 s_b^2)) at
    voxel centres; exactly round(occupancy * N) voxels are occupied (largest
    densities, ties to the smaller storage id).  Colour coefficients are the
    responsibility-weighted blend of the blob coefficients."""
    nx, ny, nz = (int(r) for r in reso)
    ncell = nx * ny * nz
    mu, std, bsh = blob_params(n_blobs, seed)
    mu, std, bsh = mu.to(device), std.to(device), bsh.to(device)
    cx, cy, cz = _centres(nx, device), _centres(ny, device), _centres(nz, device)
    dens = torch.zeros(nx, ny, nz, dtype=torch.float64, device=device)
    for b in range(n_blobs):
        inv = 1.0 / (2.0 * std[b] ** 2)
        ex = torch.exp(-((cx - mu[b, 0]) ** 2) * inv)
        ey = torch.exp(-((cy - mu[b, 1]) ** 2) * inv)
        ez = torch.exp(-((cz - mu[b, 2]) ** 2) * inv)
        val = ex[:, None, None] * ey[None, :, None] * ez[None, None, :]
        torch.maximum(dens, val, out=dens)
    dens = dens.reshape(-1) * sigma_max
    m = int(round(occupancy * ncell))
    m = max(1, min(ncell, m))
    order = torch.sort(dens, descending=True, stable=True).indices[:m]
    ids = torch.sort(order).values  # storage order
    mask = torch.zeros(ncell, dtype=torch.uint8, device=device)
    mask[ids] = 1
    density = dens[ids]
    # responsibilities of the occupied voxels
    ii = ids // (ny * nz)
    jj = (ids // nz) % ny
    kk = ids % nz
    pos = torch.stack([cx[ii], cy[jj], cz[kk]], dim=1)
    sh = torch.zeros(m, NSH, dtype=torch.float64, device=device)
    wsum = torch.zeros(m, dtype=torch.float64, device=device)
    for b in range(n_blobs):
        r2 = ((pos - mu[b]) ** 2).sum(dim=1)
        w = torch.exp(-r2 / (2.0 * std[b] ** 2)) + 1e-30
        sh += w[:, None] * bsh[b][None, :]
        wsum += w
    sh /= wsum[:, None]
    return SceneValues((nx, ny, nz), mask, density.float(), sh.float(), m)


def dense_random(reso, seed: int, sigma_lo=0.5, sigma_hi=40.0, dc_lo=1.0, dc_hi=3.0,
                 ho_scale=0.1, occupancy: float = 1.0, device="cpu") -> SceneValues:
    """Random values, optionally on a random occupancy mask: sigma U(lo, hi),
    DC U(dc_lo, dc_hi), higher orders U(-ho, ho).  With the defaults every
    sample colour is positive and every density is positive, which keeps
    finite-difference checks away from the ReLU kinks."""
    nx, ny, nz = (int(r) for r in reso)
    ncell = nx * ny * nz
    g = _gen(seed)
    if occupancy >= 1.0:
        mask = torch.ones(ncell, dtype=torch.uint8)
    else:
        mask = (torch.rand(ncell, generator=g, dtype=torch.float64) < occupancy).to(torch.uint8)
    m = int(mask.sum())
    dens = sigma_lo + (sigma_hi - sigma_lo) * torch.rand(m, generator=g, dtype=torch.float64)
    sh = (torch.rand(m, 3, 9, generator=g, dtype=torch.float64) * 2.0 - 1.0) * ho_scale
    sh[:, :, 0] = dc_lo + (dc_hi - dc_lo) * torch.rand(m, 3, generator=g, dtype=torch.float64)
    return SceneValues((nx, ny, nz), mask.to(device), dens.float().to(device),
                       sh.reshape(m, NSH).float().to(device), m)


def perturbed(sv: SceneValues, seed: int, device=None) -> SceneValues:
    """The same occupancy with every density scaled by U(0.5, 1.5) and every
    colour coefficient shifted by N(0, 0.05): a grid part-way through
    training towards sv."""
    g = _gen(seed)
    m = sv.n_vox
    scale = 0.5 + torch.rand(m, generator=g, dtype=torch.float64)
    noise = 0.05 * torch.randn(m, NSH, generator=g, dtype=torch.float64)
    dev = sv.density.device if device is None else device
    density = (sv.density.double().cpu() * scale).float().to(dev)
    sh = (sv.sh.double().cpu() + noise).float().to(dev)
    return SceneValues(sv.reso, sv.mask.to(dev), density, sh, m)


def uniform_values(reso, mask: torch.Tensor, sigma0: float, dc: float) -> SceneValues:
    """Constant init on a given mask: density sigma0, DC coefficient dc in
    every channel, higher orders 0."""
    m = int(mask.sum())
    density = torch.full((m,), float(sigma0), dtype=torch.float32, device=mask.device)
    sh = torch.zeros(m, NSH, dtype=torch.float32, device=mask.device)
    sh[:, 0] = dc
    sh[:, 9] = dc
    sh[:, 18] = dc
    return SceneValues(tuple(int(r) for r in reso), mask, density, sh, m)


def sphere_poses(n: int, seed: int, radius: float = 2.0) -> torch.Tensor:
    """n camera-to-world matrices [n,3,4] (float64): centres uniform on the
    sphere, looking at the origin, up = +z (or +y when nearly parallel)."""
    g = _gen(seed)
    v = torch.randn(n, 3, generator=g, dtype=torch.float64)
    c = radius * v / v.norm(dim=1, keepdim=True)
    fwd = -c / c.norm(dim=1, keepdim=True)
    poses = torch.zeros(n, 3, 4, dtype=torch.float64)
    for i in range(n):
        up = torch.tensor([0.0, 0.0, 1.0], dtype=torch.float64)
        if abs(float(fwd[i] @ up)) > 0.99:
            up = torch.tensor([0.0, 1.0, 0.0], dtype=torch.float64)
        right = torch.linalg.cross(fwd[i], up)
        right = right / right.norm()
        true_up = torch.linalg.cross(right, fwd[i])
        # camera axes: x = right, y = up, z = -forward
        poses[i, :, 0] = right
        poses[i, :, 1] = true_up
        poses[i, :, 2] = -fwd[i]
        poses[i, :, 3] = c[i]
    return poses


def sky_background(reso, seed: int, shell=(0.4, 0.5), sigma: float = 12.0):
    """Values of an MSI background grid of reso (L, H, W) for the 360-degree
    scenes: every voxel stored; density `sigma` in the layers between the
    fractions shell[0] and shell[1] of L (0 elsewhere); degree-0 colour
    coefficients smooth in the voxel-centre angles (theta = pi (y + 1/2)/H,
    phi = 2 pi (x + 1/2)/W) with seeded frequencies and phases.  Returns
    (mask uint8 [L*H*W], density float32 [M], coef float32 [M, 3])."""
    L, H, W = (int(r) for r in reso)
    g = _gen(seed)
    f1 = torch.randint(1, 4, (3,), generator=g).double()
    f2 = torch.randint(1, 3, (3,), generator=g).double()
    ph = torch.rand(3, 2, generator=g, dtype=torch.float64) * 2.0 * np.pi
    l = torch.arange(L, dtype=torch.float64)[:, None, None]
    th = (np.pi * (torch.arange(H, dtype=torch.float64) + 0.5) / H)[None, :, None]
    phi = (2.0 * np.pi * (torch.arange(W, dtype=torch.float64) + 0.5) / W)[None, None, :]
    dens = torch.where((l >= shell[0] * L) & (l < shell[1] * L), sigma, 0.0).expand(L, H, W)
    coef = torch.stack([1.8 + 0.9 * torch.sin(f1[c] * phi + ph[c, 0]) * torch.sin(th) +
                        0.5 * torch.cos(f2[c] * th + ph[c, 1]) + 0.0 * l for c in range(3)], dim=-1)
    coef = coef.expand(L, H, W, 3)
    mask = torch.ones(L * H * W, dtype=torch.uint8)
    return mask, dens.reshape(-1).float().contiguous(), coef.reshape(-1, 3).float().contiguous()


def forward_facing_poses(n: int, seed: int, spread: float = 0.1, tilt_deg: float = 3.0) -> torch.Tensor:
    """n camera-to-world matrices [n,3,4] (float64) of a forward-facing
    capture: centres uniform in the square [-spread, spread]^2 of the plane
    z = 0, each looking along -z turned by up to tilt_deg about the x and y
    axes (the frame of the reference camera, which sits at the origin)."""
    g = _gen(seed)
    c = (torch.rand(n, 2, generator=g, dtype=torch.float64) * 2.0 - 1.0) * spread
    ang = (torch.rand(n, 2, generator=g, dtype=torch.float64) * 2.0 - 1.0) * np.deg2rad(tilt_deg)
    poses = torch.zeros(n, 3, 4, dtype=torch.float64)
    for i in range(n):
        a, b = float(ang[i, 0]), float(ang[i, 1])
        rx = torch.tensor([[1.0, 0.0, 0.0], [0.0, np.cos(a), -np.sin(a)], [0.0, np.sin(a), np.cos(a)]],
                          dtype=torch.float64)
        ry = torch.tensor([[np.cos(b), 0.0, np.sin(b)], [0.0, 1.0, 0.0], [-np.sin(b), 0.0, np.cos(b)]],
                          dtype=torch.float64)
        poses[i, :, :3] = ry @ rx
        poses[i, 0, 3] = c[i, 0]
        poses[i, 1, 3] = c[i, 1]
    return poses


def camera_rays(pose: torch.Tensor, width: int, height: int, fov_deg: float = 45.0,
                device="cpu"):
    """Pixel-centred pinhole rays of one camera, row-major.  Returns
    (rays_o, rays_d) float32 [H*W, 3]; directions normalised in float64."""
    pose = pose.to(device=device, dtype=torch.float64)
    f = 0.5 * width / np.tan(0.5 * np.deg2rad(fov_deg))
    j, i = torch.meshgrid(torch.arange(height, device=device, dtype=torch.float64),
                          torch.arange(width, device=device, dtype=torch.float64),
                          indexing="ij")
    dx = (i + 0.5 - 0.5 * width) / f
    dy = -(j + 0.5 - 0.5 * height) / f
    dz = -torch.ones_like(dx)
    dcam = torch.stack([dx, dy, dz], dim=-1).reshape(-1, 3)
    d = dcam @ pose[:, :3].T
    d = d / d.norm(dim=1, keepdim=True)
    o = pose[:, 3].expand_as(d)
    return o.float().contiguous(), d.float().contiguous()


def all_camera_rays(poses: torch.Tensor, width: int, height: int, fov_deg=45.0, device="cpu"):
    os_, ds_ = [], []
    for p in poses:
        o, d = camera_rays(p, width, height, fov_deg, device=device)
        os_.append(o)
        ds_.append(d)
    return torch.cat(os_), torch.cat(ds_)


def morton2(x: torch.Tensor, y: torch.Tensor) -> torch.Tensor:
    """Interleaves the bits of two non-negative int64 tensors (< 2^16)."""
    def spread(v):
        v = v & 0xFFFF
        v = (v | (v << 8)) & 0x00FF00FF
        v = (v | (v << 4)) & 0x0F0F0F0F
        v = (v | (v << 2)) & 0x33333333
        v = (v | (v << 1)) & 0x55555555
        return v
    return spread(x) | (spread(y) << 1)


def focal_length(width: int, fov_deg: float = 45.0) -> float:
    """Focal length in pixels of the pinhole cameras above (horizontal FOV)."""
    return float(0.5 * width / np.tan(0.5 * np.deg2rad(fov_deg)))


def sampled_camera_rays(poses: torch.Tensor, width: int, height: int, n: int, seed: int,
                        fov_deg: float = 45.0, device="cpu", coherent: bool = False):
    """n rays drawn uniformly (with replacement) from all pixels of all
    cameras, as a training batch is.  With coherent=True the same rays are
    returned ordered by camera and by Morton order of the pixel (a data-loader
    choice that changes no ray, only the order they are listed in).  Returns
    (rays_o, rays_d, pixel_ids) where pixel_ids index the row-major
    concatenation of the images."""
    g = _gen(seed)
    npix = width * height
    ids = torch.randint(0, poses.shape[0] * npix, (n,), generator=g, dtype=torch.int64)
    ids = ids.to(device)
    if coherent:
        cam_, pix_ = ids // npix, ids % npix
        key = cam_ * (1 << 32) + morton2(pix_ % width, pix_ // width)
        ids = ids[torch.argsort(key)]
    cam = ids // npix
    pix = ids % npix
    j = (pix // width).double()
    i = (pix % width).double()
    f = 0.5 * width / np.tan(0.5 * np.deg2rad(fov_deg))
    dcam = torch.stack([(i + 0.5 - 0.5 * width) / f, -(j + 0.5 - 0.5 * height) / f,
                        -torch.ones_like(i)], dim=-1)
    P = poses.to(device=device, dtype=torch.float64)[cam]  # [n,3,4]
    d = torch.einsum("nij,nj->ni", P[:, :, :3], dcam)
    d = d / d.norm(dim=1, keepdim=True)
    o = P[:, :, 3]
    return o.float().contiguous(), d.float().contiguous(), ids


def random_rays(n: int, seed: int, radius: float = 2.0, target_half: float = 0.45):
    """n rays from the radius-`radius` sphere towards uniform points of the box
    [-target_half, target_half]^3 (float32, unit directions)."""
    g = _gen(seed)
    v = torch.randn(n, 3, generator=g, dtype=torch.float64)
    o = radius * v / v.norm(dim=1, keepdim=True)
    tgt = (torch.rand(n, 3, generator=g, dtype=torch.float64) * 2.0 - 1.0) * target_half
    d = tgt - o
    d = d / d.norm(dim=1, keepdim=True)
    return o.float().contiguous(), d.float().contiguous()


def targets_uniform(n: int, seed: int) -> torch.Tensor:
    """Random target colours U(0,1)^3, float32 [n,3]."""
    return torch.rand(n, 3, generator=_gen(seed), dtype=torch.float64).float()
