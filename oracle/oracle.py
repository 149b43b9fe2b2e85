"""Python front end of the FP64 CPU oracle (plenoxel_oracle.c).

TEST INFRASTRUCTURE ONLY: imported by the test suite, the smoke check and the
CPU-baseline leg of the benchmark, never by the HIP library or its binding.
It builds the C oracle with gcc (``-ffp-contract=off`` keeps the FP32 sample
recipe unfused) and wraps it with ctypes over NumPy arrays.

Array conventions (all host, C-contiguous):
  index    int32  [Nx*Ny*Nz]   -1 = NULL, z fastest
  density  float64 [M]
  sh       float64 [M, 27]     channel-major: R0..R8, G0..G8, B0..B8
  rays_o   float32 [R, 3], rays_d float32 [R, 3] (unit directions)
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "plenoxel_oracle.c")
_BUILD = os.path.join(_HERE, "_build")
_LIB_PATH = os.path.join(_BUILD, "liboracle.so")

_lib = None


def build(force: bool = False) -> str:
    """Compile the oracle shared library (gcc, FP64, OpenMP)."""
    os.makedirs(_BUILD, exist_ok=True)
    if force or not os.path.exists(_LIB_PATH) or (
        os.path.getmtime(_LIB_PATH) < os.path.getmtime(_SRC)
    ):
        tmp = _LIB_PATH + ".tmp%d" % os.getpid()
        cmd = [
            "gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-fopenmp",
            "-ffp-contract=off", "-fno-fast-math", "-Wall", "-Wextra",
            "-Wno-unused-parameter", _SRC, "-o", tmp, "-lm",
        ]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


_P = ctypes.c_void_p


def _ptr(a: np.ndarray | None):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def lib():
    global _lib
    if _lib is None:
        build()
        L = ctypes.CDLL(_LIB_PATH)
        i64, f32, f64, i32 = ctypes.c_int64, ctypes.c_float, ctypes.c_double, ctypes.c_int
        L.orc_grid_geometry.argtypes = [_P, _P, _P, f64, _P, _P, _P]
        L.orc_grid_geometry.restype = None
        L.orc_sh_basis.argtypes = [_P, _P]
        L.orc_sh_basis.restype = None
        L.orc_render_fwd.argtypes = [_P, _P, _P, f32, _P, _P, _P, _P, _P, i64, _P, i64,
                                     _P, _P, _P, _P]
        L.orc_render_fwd.restype = None
        L.orc_trace_ray.argtypes = [_P, _P, _P, f32, _P, _P, _P, _P, _P, i32, _P,
                                    _P, _P, _P, _P]
        L.orc_trace_ray.restype = i32
        L.orc_camera_rays.argtypes = [_P, f64, ctypes.c_int32, ctypes.c_int32, _P, _P]
        L.orc_camera_rays.restype = None
        L.orc_rays_to_ndc.argtypes = [_P, _P, i64, ctypes.c_int32, ctypes.c_int32, f64, f64, _P, _P]
        L.orc_rays_to_ndc.restype = None
        L.orc_bg_render_fwd.argtypes = [_P, _P, _P, _P, _P, _P, i64, _P, _P, _P]
        L.orc_bg_render_fwd.restype = None
        L.orc_bg_render_bwd.argtypes = [_P, _P, _P, _P, _P, _P, i64, _P, _P, f64, _P, _P, _P]
        L.orc_bg_render_bwd.restype = None
        L.orc_ray_extent.argtypes = [_P, _P, _P, f32, _P, _P, _P, _P, _P]
        L.orc_ray_extent.restype = i32
        L.orc_render_bwd.argtypes = [_P, _P, _P, f32, _P, _P, _P, _P, _P, i64, _P, i64,
                                     _P, _P, _P, _P]
        L.orc_render_bwd.restype = None
        L.orc_render_bwd_mass.argtypes = [_P, _P, _P, f32, _P, _P, _P, _P, _P, i64, _P, i64,
                                          _P, f64, _P, _P]
        L.orc_render_bwd_mass.restype = None
        L.orc_tv.argtypes = [_P, _P, _P, _P, i64, i64, f64, f64, f64, _P, _P, _P]
        L.orc_tv.restype = f64
        L.orc_bg_tv.argtypes = [_P, _P, _P, _P, i64, i64, f64, f64, f64, _P, _P, _P]
        L.orc_bg_tv.restype = f64
        L.orc_rmsprop.argtypes = [i64, _P, _P, _P, _P, _P, _P, _P, f64, f64, f64, f64]
        L.orc_rmsprop.restype = None
        L.orc_grid_create.argtypes = [_P, _P, _P]
        L.orc_grid_create.restype = i64
        L.orc_max_weight.argtypes = [_P, _P, _P, f32, _P, _P, _P, _P, _P, i64, _P]
        L.orc_max_weight.restype = None
        L.orc_regularisers.argtypes = [_P, _P, _P, f32, _P, _P, _P, _P, _P, i64, f64, f64, f64,
                                       f64, _P, _P, _P]
        L.orc_regularisers.restype = None
        L.orc_prune_mask.argtypes = [_P, _P, _P, f64, _P, _P]
        L.orc_prune_mask.restype = i64
        L.orc_upsample_count.argtypes = [_P, _P, _P]
        L.orc_upsample_count.restype = i64
        L.orc_upsample.argtypes = [_P, _P, _P, _P, _P, _P, _P, _P]
        L.orc_upsample.restype = i64
        L.orc_lr_schedule.argtypes = [f64, f64, f64, f64, f64, f64]
        L.orc_lr_schedule.restype = f64
        L.orc_set_threads.argtypes = [i32]
        L.orc_set_threads.restype = None
        L.orc_max_threads.argtypes = []
        L.orc_max_threads.restype = i32
        _lib = L
    return _lib


def _c(a, dtype):
    return np.ascontiguousarray(a, dtype=dtype)


@dataclass
class Grid:
    """Oracle grid: geometry + index + FP64 table."""

    reso: np.ndarray  # int32[3]
    scale: np.ndarray  # float32[3]
    offset: np.ndarray  # float32[3]
    step: np.float32
    index: np.ndarray  # int32[N]
    density: np.ndarray  # float64[M]
    sh: np.ndarray  # float64[M,27]

    @property
    def n_vox(self) -> int:
        return int(self.density.shape[0])


def grid_geometry(reso, lo=(-0.5, -0.5, -0.5), hi=(0.5, 0.5, 0.5), step_voxels=0.5):
    """Grid frame (scale, offset, step) of an axis-aligned box, FP32."""
    r = _c(reso, np.int32)
    scale = np.zeros(3, np.float32)
    offset = np.zeros(3, np.float32)
    step = np.zeros(1, np.float32)
    lib().orc_grid_geometry(_ptr(r), _ptr(_c(lo, np.float64)), _ptr(_c(hi, np.float64)),
                            float(step_voxels), _ptr(scale), _ptr(offset), _ptr(step))
    return scale, offset, np.float32(step[0])


def grid_create(reso, mask) -> tuple[np.ndarray, int]:
    r = _c(reso, np.int32)
    m = _c(mask, np.uint8).reshape(-1)
    index = np.empty(m.shape[0], np.int32)
    n = lib().orc_grid_create(_ptr(r), _ptr(m), _ptr(index))
    return index, int(n)


def make_grid(reso, mask, density, sh, lo=(-0.5,) * 3, hi=(0.5,) * 3, step_voxels=0.5) -> Grid:
    index, m = grid_create(reso, mask)
    density = _c(density, np.float64).reshape(-1)
    sh = _c(sh, np.float64).reshape(-1, 27)
    assert density.shape[0] == m and sh.shape[0] == m
    scale, offset, step = grid_geometry(reso, lo, hi, step_voxels)
    return Grid(_c(reso, np.int32), scale, offset, step, index, density, sh)


def sh_basis(d) -> np.ndarray:
    d = _c(d, np.float64).reshape(-1, 3)
    out = np.empty((d.shape[0], 9), np.float64)
    for i in range(d.shape[0]):
        lib().orc_sh_basis(_ptr(d[i]), _ptr(out[i]))
    return out


def _grid_args(g: Grid):
    return (_ptr(g.reso), _ptr(g.scale), _ptr(g.offset), float(g.step), _ptr(g.index),
            _ptr(g.density), _ptr(g.sh))


def _bg(bg, n):
    """Background colours: one (3,) colour for every ray, or (n, 3) per ray."""
    b = _c(bg, np.float64)
    if b.size == 3 and b.ndim == 1:
        return b, 0
    b = b.reshape(-1, 3)
    assert b.shape[0] == n
    return b, 3


def render_fwd(g: Grid, rays_o, rays_d, bg=(1.0, 1.0, 1.0)):
    """Returns rgb[R,3], tau[R] (optical depth), t_final[R], n_samples[R].
    bg: one colour or one per ray ([R,3])."""
    o = _c(rays_o, np.float32).reshape(-1, 3)
    d = _c(rays_d, np.float32).reshape(-1, 3)
    n = o.shape[0]
    rgb = np.empty((n, 3), np.float64)
    tau = np.empty(n, np.float64)
    tf = np.empty(n, np.float64)
    ns = np.empty(n, np.int32)
    b, bs = _bg(bg, n)
    lib().orc_render_fwd(*_grid_args(g), _ptr(o), _ptr(d), n, _ptr(b), bs,
                         _ptr(rgb), _ptr(tau), _ptr(tf), _ptr(ns))
    return rgb, tau, tf, ns


def render_bwd(g: Grid, rays_o, rays_d, grad_rgb, bg=(1.0, 1.0, 1.0)):
    """Returns grad_density[M], grad_sh[M,27], touched[M] (uint8)."""
    o = _c(rays_o, np.float32).reshape(-1, 3)
    d = _c(rays_d, np.float32).reshape(-1, 3)
    gr = _c(grad_rgb, np.float64).reshape(-1, 3)
    gd = np.zeros(g.n_vox, np.float64)
    gs = np.zeros((g.n_vox, 27), np.float64)
    touched = np.zeros(g.n_vox, np.uint8)
    b, bs = _bg(bg, o.shape[0])
    lib().orc_render_bwd(*_grid_args(g), _ptr(o), _ptr(d), o.shape[0],
                         _ptr(b), bs, _ptr(gr), _ptr(gd), _ptr(gs),
                         _ptr(touched))
    return gd, gs, touched


def render_bwd_mass(g: Grid, rays_o, rays_d, gabs_rgb, bg=(1.0, 1.0, 1.0), gate_rel=0.0):
    """Per-element sums of the absolute gradient terms for |dL/dC| =
    gabs_rgb (see orc_render_bwd_mass): (mass_density[M], mass_sh[M,27]).
    Terms behind a ReLU gate within gate_rel of its kink count as open."""
    o = _c(rays_o, np.float32).reshape(-1, 3)
    d = _c(rays_d, np.float32).reshape(-1, 3)
    ga = np.abs(_c(gabs_rgb, np.float64).reshape(-1, 3))
    md = np.zeros(g.n_vox, np.float64)
    ms = np.zeros((g.n_vox, 27), np.float64)
    b, bs = _bg(bg, o.shape[0])
    lib().orc_render_bwd_mass(*_grid_args(g), _ptr(o), _ptr(d), o.shape[0],
                              _ptr(b), bs, _ptr(ga), float(gate_rel), _ptr(md),
                              _ptr(ms))
    return md, ms


def mse_grad(rgb, target):
    """dL/dC of L = 1/R sum_r ||C_r - target_r||^2 (Sec. 3.5 reconstruction
    loss), and L itself."""
    rgb = np.asarray(rgb, np.float64)
    target = np.asarray(target, np.float64)
    n = rgb.shape[0]
    diff = rgb - target
    return 2.0 * diff / n, float((diff * diff).sum() / n)


def trace_ray(g: Grid, o, d, cap=None):
    """Per-sample trace: dict of t, delta, sigma_pre, rgb_pre[n,3], cell[n,3]."""
    o = _c(o, np.float32).reshape(3)
    d = _c(d, np.float32).reshape(3)
    if cap is None:
        cap = int(np.ceil(np.sqrt(float((g.reso.astype(np.float64) ** 2).sum())) /
                          (float(g.step) * float(np.min(g.scale))))) + 8
    t = np.empty(cap, np.float64)
    delta = np.empty(cap, np.float64)
    sp = np.empty(cap, np.float64)
    rp = np.empty((cap, 3), np.float64)
    cell = np.empty((cap, 3), np.int32)
    n = lib().orc_trace_ray(*_grid_args(g), _ptr(o), _ptr(d), cap, _ptr(t), _ptr(delta),
                            _ptr(sp), _ptr(rp), _ptr(cell))
    assert n <= cap, "trace capacity too small"
    return dict(t=t[:n], delta=delta[:n], sigma_pre=sp[:n], rgb_pre=rp[:n], cell=cell[:n])


def camera_rays(c2w, focal, width, height):
    """Pixel-centred pinhole rays of one view (orc_camera_rays):
    (rays_o, rays_d) float32 [H*W, 3]."""
    m = _c(c2w, np.float64).reshape(12)
    o = np.empty((width * height, 3), np.float32)
    d = np.empty((width * height, 3), np.float32)
    lib().orc_camera_rays(_ptr(m), float(focal), int(width), int(height), _ptr(o), _ptr(d))
    return o, d


def rays_to_ndc(rays_o, rays_d, width, height, focal, near=1.0):
    """NDC rays of forward-facing scenes (orc_rays_to_ndc): float32 [R, 3]
    origins and unit directions."""
    o = _c(rays_o, np.float32).reshape(-1, 3)
    d = _c(rays_d, np.float32).reshape(-1, 3)
    oo = np.empty_like(o)
    dd = np.empty_like(d)
    lib().orc_rays_to_ndc(_ptr(o), _ptr(d), o.shape[0], int(width), int(height), float(focal), float(near),
                          _ptr(oo), _ptr(dd))
    return oo, dd


def bg_grid(reso, mask, density, rgb_coef):
    """MSI background grid of reso (L, H, W) from a mask and per-voxel
    density [M] and degree-0 colour coefficients [M, 3] (sh slots 24-26)."""
    index, m = grid_create(reso, mask)
    dens = _c(density, np.float64).reshape(-1)
    k = _c(rgb_coef, np.float64).reshape(-1, 3)
    assert dens.shape[0] == m and k.shape[0] == m
    sh = np.zeros((m, 27), np.float64)
    sh[:, 24:27] = k
    scale = np.ones(3, np.float32)
    offset = np.zeros(3, np.float32)
    return Grid(_c(reso, np.int32), scale, offset, np.float32(0.5), index, dens, sh)


def bg_render_fwd(g: Grid, rays_o, rays_d, bg=(1.0, 1.0, 1.0)):
    """Background colour of each ray and the transmittance left after it:
    (rgb[R,3], t[R])."""
    o = _c(rays_o, np.float32).reshape(-1, 3)
    d = _c(rays_d, np.float32).reshape(-1, 3)
    rgb = np.empty((o.shape[0], 3), np.float64)
    t = np.empty(o.shape[0], np.float64)
    lib().orc_bg_render_fwd(_ptr(g.reso), _ptr(g.index), _ptr(g.density), _ptr(g.sh), _ptr(o), _ptr(d),
                            o.shape[0], _ptr(_c(bg, np.float64)), _ptr(rgb), _ptr(t))
    return rgb, t


def bg_render_bwd(g: Grid, rays_o, rays_d, grad_rgb, bg=(1.0, 1.0, 1.0)):
    """Gradient of the background colours for dL/dC_bg = grad_rgb:
    (grad_density[M], grad_sh[M,27], touched[M])."""
    o = _c(rays_o, np.float32).reshape(-1, 3)
    d = _c(rays_d, np.float32).reshape(-1, 3)
    gr = _c(grad_rgb, np.float64).reshape(-1, 3)
    gd = np.zeros(g.n_vox, np.float64)
    gs = np.zeros((g.n_vox, 27), np.float64)
    touched = np.zeros(g.n_vox, np.uint8)
    lib().orc_bg_render_bwd(_ptr(g.reso), _ptr(g.index), _ptr(g.density), _ptr(g.sh), _ptr(o), _ptr(d),
                            o.shape[0], _ptr(_c(bg, np.float64)), _ptr(gr), -1.0, _ptr(gd), _ptr(gs),
                            _ptr(touched))
    return gd, gs, touched


def bg_render_bwd_mass(g: Grid, rays_o, rays_d, gabs_rgb, bg=(1.0, 1.0, 1.0), gate_rel=0.0):
    """Absolute-term sums of the background gradient for |dL/dC_bg| =
    gabs_rgb (see orc_bg_render_bwd): (mass_density[M], mass_sh[M,27])."""
    o = _c(rays_o, np.float32).reshape(-1, 3)
    d = _c(rays_d, np.float32).reshape(-1, 3)
    ga = np.abs(_c(gabs_rgb, np.float64).reshape(-1, 3))
    md = np.zeros(g.n_vox, np.float64)
    ms = np.zeros((g.n_vox, 27), np.float64)
    touched = np.zeros(g.n_vox, np.uint8)
    lib().orc_bg_render_bwd(_ptr(g.reso), _ptr(g.index), _ptr(g.density), _ptr(g.sh), _ptr(o), _ptr(d),
                            o.shape[0], _ptr(_c(bg, np.float64)), _ptr(ga), max(0.0, float(gate_rel)), _ptr(md),
                            _ptr(ms), _ptr(touched))
    return md, ms


def ray_extent(g: Grid, o, d):
    o = _c(o, np.float32).reshape(3)
    d = _c(d, np.float32).reshape(3)
    tn = ctypes.c_float()
    tf = ctypes.c_float()
    ns = ctypes.c_int32()
    hit = lib().orc_ray_extent(_ptr(g.reso), _ptr(g.scale), _ptr(g.offset), float(g.step),
                               _ptr(o), _ptr(d), ctypes.byref(tn), ctypes.byref(tf),
                               ctypes.byref(ns))
    return bool(hit), np.float32(tn.value), np.float32(tf.value), int(ns.value)


def tv(g: Grid, start, count, lambda_sigma, lambda_sh, eps=1e-9):
    """Returns loss, grad_density[M], grad_sh[M,27], touched[M].  eps > 0
    (the square root's derivative is unbounded at 0)."""
    if not eps > 0.0:
        raise ValueError("TV eps must be positive")
    gd = np.zeros(g.n_vox, np.float64)
    gs = np.zeros((g.n_vox, 27), np.float64)
    touched = np.zeros(g.n_vox, np.uint8)
    loss = lib().orc_tv(_ptr(g.reso), _ptr(g.index), _ptr(g.density), _ptr(g.sh),
                        int(start), int(count), float(lambda_sigma), float(lambda_sh),
                        float(eps), _ptr(gd), _ptr(gs), _ptr(touched))
    return float(loss), gd, gs, touched


def bg_tv(g: Grid, start, count, lambda_sigma, lambda_color, eps=1e-9):
    """TV of an MSI background grid (azimuth wraps, colour slots 24-26):
    loss, grad_density[M], grad_sh[M,27], touched[M]; eps > 0 as for tv."""
    if not eps > 0.0:
        raise ValueError("TV eps must be positive")
    gd = np.zeros(g.n_vox, np.float64)
    gs = np.zeros((g.n_vox, 27), np.float64)
    touched = np.zeros(g.n_vox, np.uint8)
    loss = lib().orc_bg_tv(_ptr(g.reso), _ptr(g.index), _ptr(g.density), _ptr(g.sh),
                           int(start), int(count), float(lambda_sigma), float(lambda_color),
                           float(eps), _ptr(gd), _ptr(gs), _ptr(touched))
    return float(loss), gd, gs, touched


def rmsprop(active, density, sh, v_density, v_sh, grad_density, grad_sh,
            lr_sigma, lr_sh, beta=0.95, eps=1e-8):
    """In-place RMSProp on the active voxels (all arrays float64, modified)."""
    act = _c(active, np.uint8)
    for a in (density, sh, v_density, v_sh, grad_density, grad_sh):
        assert a.dtype == np.float64 and a.flags["C_CONTIGUOUS"]
    lib().orc_rmsprop(act.shape[0], _ptr(act), _ptr(density), _ptr(sh), _ptr(v_density),
                      _ptr(v_sh), _ptr(grad_density), _ptr(grad_sh), float(lr_sigma),
                      float(lr_sh), float(beta), float(eps))


def regularisers(g: Grid, rays_o, rays_d, lambda_s, lambda_b, eps=1e-3, gate_rel=0.0):
    """Cauchy sparsity and beta transmittance priors (Sec. 3.7) over the
    rays: returns (loss_s, loss_b, grad_density[M], mass_density[M])."""
    o = _c(rays_o, np.float32).reshape(-1, 3)
    d = _c(rays_d, np.float32).reshape(-1, 3)
    loss = np.zeros(2, np.float64)
    gd = np.zeros(g.n_vox, np.float64)
    md = np.zeros(g.n_vox, np.float64)
    lib().orc_regularisers(_ptr(g.reso), _ptr(g.scale), _ptr(g.offset), float(g.step), _ptr(g.index),
                           _ptr(g.density), _ptr(g.sh), _ptr(o), _ptr(d), o.shape[0], float(lambda_s),
                           float(lambda_b), float(eps), float(gate_rel), _ptr(loss), _ptr(gd), _ptr(md))
    return float(loss[0]), float(loss[1]), gd, md


def max_weight(g: Grid, rays_o, rays_d, wmax=None):
    """Per-voxel maximum sample weight over the rays (float64[M]); raises
    `wmax` in place when given (accumulation over batches)."""
    o = _c(rays_o, np.float32).reshape(-1, 3)
    d = _c(rays_d, np.float32).reshape(-1, 3)
    if wmax is None:
        wmax = np.zeros(g.n_vox, np.float64)
    assert wmax.dtype == np.float64 and wmax.flags["C_CONTIGUOUS"] and wmax.shape == (g.n_vox,)
    lib().orc_max_weight(_ptr(g.reso), _ptr(g.scale), _ptr(g.offset), float(g.step), _ptr(g.index),
                         _ptr(g.density), _ptr(g.sh), _ptr(o), _ptr(d), o.shape[0], _ptr(wmax))
    return wmax


def prune_mask(g: Grid, thresh, values=None):
    """Keep mask of pruning with dilation: a voxel is occupied when
    values[id] >= thresh (values = the stored density unless given, e.g. the
    maximum sample weight for pruning by weight)."""
    vals = g.density if values is None else _c(values, np.float64)
    assert vals.shape == (g.n_vox,)
    keep = np.empty(g.index.shape[0], np.uint8)
    npr = ctypes.c_int64()
    kept = lib().orc_prune_mask(_ptr(g.reso), _ptr(g.index), _ptr(vals), float(thresh),
                                _ptr(keep), ctypes.byref(npr))
    return keep, int(kept), int(npr.value)


def prune(g: Grid, thresh, values=None) -> tuple[Grid, int, int]:
    """Prunes and compacts (table order preserved)."""
    keep, kept, npruned = prune_mask(g, thresh, values)
    old_ids = g.index[keep.astype(bool)]
    index, m = grid_create(g.reso, keep)
    assert m == kept
    out = Grid(g.reso.copy(), g.scale.copy(), g.offset.copy(), g.step, index,
               g.density[old_ids].copy(), g.sh[old_ids].copy())
    return out, kept, npruned


def upsample(g: Grid, new_reso, lo=(-0.5,) * 3, hi=(0.5,) * 3, step_voxels=0.5) -> Grid:
    nr = _c(new_reso, np.int32)
    m = lib().orc_upsample_count(_ptr(g.reso), _ptr(g.index), _ptr(nr))
    index = np.empty(int(np.prod(nr.astype(np.int64))), np.int32)
    dens = np.empty(m, np.float64)
    sh = np.empty((m, 27), np.float64)
    m2 = lib().orc_upsample(_ptr(g.reso), _ptr(g.index), _ptr(g.density), _ptr(g.sh),
                            _ptr(nr), _ptr(index), _ptr(dens), _ptr(sh))
    assert m2 == m
    scale, offset, step = grid_geometry(nr, lo, hi, step_voxels)
    return Grid(nr, scale, offset, step, index, dens, sh)


def lr_schedule(step, lr0, lr1, max_steps, delay_steps=0.0, delay_mult=1.0) -> float:
    return float(lib().orc_lr_schedule(float(step), float(lr0), float(lr1), float(max_steps),
                                       float(delay_steps), float(delay_mult)))


def set_threads(n: int):
    """Host threads of the oracle's parallel loops (results do not depend on
    it: sums are formed in a fixed order)."""
    lib().orc_set_threads(int(n))


def max_threads() -> int:
    return int(lib().orc_max_threads())
