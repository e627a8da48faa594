import os
import sys

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (runs the HIP library)")


def _gpu_available() -> bool:
    try:
        import torch
        return torch.cuda.is_available()
    except Exception:
        return False


def pytest_collection_modifyitems(config, items):
    if _gpu_available():
        return
    skip = pytest.mark.skip(reason="no GPU in this environment")
    for it in items:
        if "gpu" in it.keywords:
            it.add_marker(skip)


@pytest.fixture(scope="session")
def small_workload():
    """The small workload (200x200 at 0.04 m, 20k-point clouds, one camera),
    generated once per session.  Frame count kept at 10 as specified."""
    from paper_2309_16818_amd import synth
    ter, frames = synth.small_frames(seed=0, n_frames=10)
    return ter, frames


@pytest.fixture(scope="session")
def small_workload_3():
    from paper_2309_16818_amd import synth
    ter, frames = synth.small_frames(seed=7, n_frames=3, n_points=5000, cam_hw=(120, 160))
    return ter, frames
