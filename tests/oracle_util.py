"""Small helpers for the oracle tests: turn synthetic scene values into oracle
grids.  (Test plumbing only; no method arithmetic.)"""
import numpy as np

from oracle import oracle as O


def oracle_grid(sv, lo=(-0.5,) * 3, hi=(0.5,) * 3, step_voxels=0.5):
    """Oracle grid from synth.SceneValues (values upcast exactly to float64)."""
    return O.make_grid(np.array(sv.reso, np.int32), sv.mask.cpu().numpy(),
                       sv.density.cpu().double().numpy(), sv.sh.cpu().double().numpy(),
                       lo, hi, step_voxels)


def dense_grid(reso, density, sh, lo=(-0.5,) * 3, hi=(0.5,) * 3, step_voxels=0.5):
    n = int(np.prod(reso))
    return O.make_grid(np.array(reso, np.int32), np.ones(n, np.uint8),
                       np.asarray(density, np.float64).reshape(-1),
                       np.asarray(sh, np.float64).reshape(n, 27), lo, hi, step_voxels)


def lattice_coords(reso):
    nx, ny, nz = reso
    i, j, k = np.meshgrid(np.arange(nx), np.arange(ny), np.arange(nz), indexing="ij")
    return i.reshape(-1), j.reshape(-1), k.reshape(-1)
