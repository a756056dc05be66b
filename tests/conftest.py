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
def tiny_case():
    import synth
    import oracle
    sc = synth.make_tiny(0)
    cam = synth.tiny_camera()
    prm = oracle.RenderParams()
    proj = oracle.project(sc.means, sc.scales, sc.quats, sc.opacity, cam, prm)
    gids, offs, _ = oracle.bin_sort(proj["rect"], proj["depth"], 4, 4)
    return dict(scene=sc, cam=cam, params=prm, proj=proj, gids=gids, offs=offs)
