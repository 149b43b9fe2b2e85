"""Grid container: owns the device tensors of one Plenoxel grid (index grid,
voxel records, cell occupancy bitmap and, for 16-bit SH storage, the FP32
master records) and drives the library's grid calls."""
from __future__ import annotations

import torch

from . import binding as B


def _alloc_records(n: int, sh_dtype: int, device) -> torch.Tensor:
    """[n, 32] float32 (128-byte records) or [n, 32] int16 (64-byte records)."""
    n = max(int(n), 0)
    if sh_dtype == B.PLX_F32:
        return torch.zeros(n, B.REC_SLOTS, dtype=torch.float32, device=device)
    return torch.zeros(n, B.REC_SLOTS, dtype=torch.int16, device=device)


class Grid:
    """A sparse voxel grid in the box [lo, hi] with resolution reso.

    index  int32  [Nx*Ny*Nz]   -1 = NULL, else table id (storage order)
    data   records [M, 32]     float32 (PLX_F32) or int16 (16-bit SH)
    master float32 [M, 32]     FP32 records behind 16-bit data (else None)
    occ    int32  [bytes/4]    occupancy structure: cell bitmap + brick
                               distances (rebuilt on change)
    """

    def __init__(self, reso, index, data, sh_dtype=B.PLX_F32, master=None,
                 lo=(-0.5,) * 3, hi=(0.5,) * 3, step_voxels=0.5, build_occ=True):
        self.reso = tuple(int(r) for r in reso)
        self.lo, self.hi, self.step_voxels = tuple(lo), tuple(hi), float(step_voxels)
        self.scale, self.offset, self.step = B.plx_grid_geometry(self.reso, lo, hi, step_voxels)
        self.index = index
        self.data = data
        self.sh_dtype = int(sh_dtype)
        self.master = master
        self.occ = torch.zeros(B.plx_occ_bytes(self.reso) // 4, dtype=torch.int32, device=index.device)
        if build_occ:
            self.rebuild_occupancy()

    # ---------------------------------------------------------------- info
    @property
    def n_vox(self) -> int:
        return int(self.data.shape[0])

    @property
    def n_cells(self) -> int:
        return self.reso[0] * self.reso[1] * self.reso[2]

    @property
    def device(self):
        return self.index.device

    def desc(self, data=None, sh_dtype=None) -> B.PlxGrid:
        """C descriptor (optionally over other records, e.g. the master)."""
        data = self.data if data is None else data
        g = B.PlxGrid()
        for a in range(3):
            g.reso[a] = self.reso[a]
            g.scale[a] = self.scale[a]
            g.offset[a] = self.offset[a]
        g.step = self.step
        g.sh_dtype = self.sh_dtype if sh_dtype is None else sh_dtype
        g.n_vox = int(data.shape[0])
        g.index = self.index.data_ptr()
        g.data = data.data_ptr() if data.numel() else None
        g.occ = self.occ.data_ptr()
        return g

    def param_records(self) -> torch.Tensor:
        """The FP32 records that training updates."""
        return self.data if self.sh_dtype == B.PLX_F32 else self.master

    # ---------------------------------------------------------------- build
    @classmethod
    def from_mask(cls, mask: torch.Tensor, reso, density=None, sh=None, sigma0=0.1, dc=0.5 / 0.28209479,
                  sh_dtype=B.PLX_F32, lo=(-0.5,) * 3, hi=(0.5,) * 3, step_voxels=0.5) -> "Grid":
        """Index grid from a uint8 mask (device), records from density [M] /
        sh [M, 27] (device float32) or from the constant init (sigma0, DC)."""
        dev = mask.device
        reso = tuple(int(r) for r in reso)
        m = B.plx_mask_count(mask)
        index = torch.empty(reso[0] * reso[1] * reso[2], dtype=torch.int32, device=dev)
        B.plx_grid_create(mask, reso, index)
        rec32 = _alloc_records(m, B.PLX_F32, dev)
        if density is not None:
            density = density.to(device=dev, dtype=torch.float32).contiguous()
        if sh is not None:
            sh = sh.to(device=dev, dtype=torch.float32).contiguous()
        B.plx_records_pack(B.PLX_F32, m, density, sh, sigma0, dc, rec32)
        if sh_dtype == B.PLX_F32:
            return cls(reso, index, rec32, B.PLX_F32, None, lo, hi, step_voxels)
        rec16 = _alloc_records(m, sh_dtype, dev)
        B.plx_records_convert(B.PLX_F32, rec32, sh_dtype, rec16, m)
        return cls(reso, index, rec16, sh_dtype, rec32, lo, hi, step_voxels)

    def rebuild_occupancy(self):
        B.plx_grid_build_occupancy(self.desc(), self.occ)

    def sync_from_master(self):
        """Re-rounds the 16-bit records from the FP32 master."""
        if self.master is not None:
            B.plx_records_convert(B.PLX_F32, self.master, self.sh_dtype, self.data, self.n_vox)

    def to_dtype(self, sh_dtype: int) -> "Grid":
        """Copy with another SH storage type (FP32 master kept for 16-bit)."""
        src = self.param_records()
        if sh_dtype == B.PLX_F32:
            return Grid(self.reso, self.index.clone(), src.clone(), B.PLX_F32, None, self.lo,
                        self.hi, self.step_voxels)
        rec16 = _alloc_records(self.n_vox, sh_dtype, self.device)
        B.plx_records_convert(B.PLX_F32, src, sh_dtype, rec16, self.n_vox)
        return Grid(self.reso, self.index.clone(), rec16, sh_dtype, src.clone(), self.lo, self.hi,
                    self.step_voxels)

    def unpack(self, master: bool = False):
        """(density [M], sh [M, 27]) float32 of the stored records (or of
        the FP32 master)."""
        recs = self.master if (master and self.master is not None) else self.data
        dt = B.PLX_F32 if (master and self.master is not None) else self.sh_dtype
        d = torch.empty(self.n_vox, dtype=torch.float32, device=self.device)
        s = torch.empty(self.n_vox, B.NSH, dtype=torch.float32, device=self.device)
        B.plx_records_unpack(dt, self.n_vox, recs, d, s)
        return d, s

    # ---------------------------------------------------------------- coarse to fine
    def prune(self, sigma_thresh: float):
        """Density-threshold prune with dilation; returns (new grid, kept,
        pruned)."""
        keep = torch.empty(self.n_cells, dtype=torch.uint8, device=self.device)
        src = self.param_records()
        src_dt = B.PLX_F32 if self.master is not None else self.sh_dtype
        kept, pruned = B.plx_grid_prune_count(self.desc(src, src_dt), sigma_thresh, keep)
        return self._compact(keep, kept), kept, pruned

    def max_weight(self, rays_o, rays_d, batch: int = 1 << 20, wmax=None) -> torch.Tensor:
        """Per-voxel maximum sample weight over all the rays (float32 [M]),
        taken in batches of `batch` rays: the statistic of pruning by
        weight.  Raises `wmax` in place when given."""
        if wmax is None:
            wmax = torch.zeros(self.n_vox, dtype=torch.float32, device=self.device)
        g = self.desc()
        for s in range(0, rays_o.shape[0], batch):
            B.plx_render_max_weight(g, rays_o[s:s + batch], rays_d[s:s + batch], wmax)
        return wmax

    def prune_by_weight(self, wmax: torch.Tensor, w_thresh: float):
        """Weight-threshold prune with dilation (wmax from max_weight);
        returns (new grid, kept, pruned)."""
        keep = torch.empty(self.n_cells, dtype=torch.uint8, device=self.device)
        kept, pruned = B.plx_grid_prune_weight_count(self.desc(), wmax, w_thresh, keep)
        return self._compact(keep, kept), kept, pruned

    def _compact(self, keep: torch.Tensor, kept: int) -> "Grid":
        src = self.param_records()
        src_dt = B.PLX_F32 if self.master is not None else self.sh_dtype
        index = torch.empty(self.n_cells, dtype=torch.int32, device=self.device)
        new_src = _alloc_records(kept, src_dt, self.device)
        out = B.PlxGrid()
        out.reso[:] = self.reso
        out.sh_dtype = src_dt
        out.n_vox = kept
        out.index = index.data_ptr()
        out.data = new_src.data_ptr() if kept else None
        B.plx_grid_prune_apply(self.desc(src, src_dt), keep, out)
        if self.master is None:
            g = Grid(self.reso, index, new_src, self.sh_dtype, None, self.lo, self.hi,
                     self.step_voxels)
        else:
            rec16 = _alloc_records(kept, self.sh_dtype, self.device)
            B.plx_records_convert(B.PLX_F32, new_src, self.sh_dtype, rec16, kept)
            g = Grid(self.reso, index, rec16, self.sh_dtype, new_src, self.lo, self.hi,
                     self.step_voxels)
        return g

    def upsample(self, new_reso, step_voxels: float | None = None) -> "Grid":
        """Trilinear resampling to new_reso (values from the FP32 records);
        the sample step stays step_voxels finest-axis voxels (this grid's
        unless given)."""
        new_reso = tuple(int(r) for r in new_reso)
        sv = self.step_voxels if step_voxels is None else float(step_voxels)
        src = self.param_records()
        src_dt = B.PLX_F32 if self.master is not None else self.sh_dtype
        n = B.plx_grid_upsample_count(self.desc(src, src_dt), new_reso)
        ncell = new_reso[0] * new_reso[1] * new_reso[2]
        index = torch.empty(ncell, dtype=torch.int32, device=self.device)
        new_src = _alloc_records(n, src_dt, self.device)
        out = B.PlxGrid()
        out.reso[:] = new_reso
        out.sh_dtype = src_dt
        out.n_vox = n
        out.index = index.data_ptr()
        out.data = new_src.data_ptr() if n else None
        B.plx_grid_upsample_apply(self.desc(src, src_dt), out)
        if self.master is None:
            return Grid(new_reso, index, new_src, self.sh_dtype, None, self.lo, self.hi, sv)
        rec16 = _alloc_records(n, self.sh_dtype, self.device)
        B.plx_records_convert(B.PLX_F32, new_src, self.sh_dtype, rec16, n)
        return Grid(new_reso, index, rec16, self.sh_dtype, new_src, self.lo, self.hi, sv)
