import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_collection_modifyitems(config, items):
    import torch

    if torch.cuda.is_available():
        return
    skip = pytest.mark.skip(reason="no GPU visible (torch.cuda.is_available() is False)")
    for item in items:
        if "gpu" in item.keywords:
            item.add_marker(skip)


@pytest.fixture(scope="session")
def c3_scene():
    """512^3 at 5% occupancy (about 6.7M voxels), 100 cameras at 800x800,
    a 1M-ray batch (seed 2): (scene values, GPU grid, oracle grid, o, d)."""
    import numpy as np

    import synth
    from oracle import oracle as O
    from paper_2112_05131_amd.grid import Grid
    from tests.gpu_util import say

    say("building c3 scene")
    sv = synth.blob_scene((512, 512, 512), n_blobs=32, occupancy=0.05, seed=2, device="cuda")
    poses = synth.sphere_poses(100, seed=2)
    o, d, _ = synth.sampled_camera_rays(poses, 800, 800, 1 << 20, seed=2, device="cuda")
    gg = Grid.from_mask(sv.mask, sv.reso, sv.density, sv.sh)
    og = O.make_grid(np.array(sv.reso, np.int32), sv.mask.cpu().numpy(),
                     sv.density.cpu().double().numpy(), sv.sh.cpu().double().numpy())
    return sv, gg, og, o, d
