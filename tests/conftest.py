import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: long-running CPU test")


@pytest.fixture(scope="session")
def room_scene():
    import synth
    return synth.scene_for_config("room", seed=0)


@pytest.fixture(scope="session")
def lnr():
    """The HIP library binding; GPU tests fail loudly if it is not built."""
    import paper_2502_11618_amd as L
    return L


@pytest.fixture(scope="session")
def ctx(lnr):
    import torch
    assert torch.cuda.is_available(), "GPU tests need a visible GPU"
    return lnr.lnr_context_create(0)


@pytest.fixture(scope="session")
def room_grid(room_scene):
    from oracle import grid as G
    return G.partition(room_scene.xyz, room_scene.rgb, 0.5)


@pytest.fixture(scope="session")
def room_cloud(lnr, ctx, room_scene):
    return lnr.lnr_cloud_load(ctx, room_scene.xyz, room_scene.rgb, 0.5)


@pytest.fixture(scope="session")
def room_cams(room_scene):
    import synth
    return synth.room_cameras(room_scene, 16, seed=0, width=256, height=256, fov_deg=70.0)
