import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU")
    config.addinivalue_line("markers", "slow: long-running CPU test")


@pytest.fixture(scope="session")
def tiny():
    import synth
    return synth.tiny_box()


@pytest.fixture(scope="session")
def tiny_oracle(tiny):
    from oracle import bake as ob
    return ob.OracleScene(tiny)


@pytest.fixture(scope="session")
def tiny_points(tiny_oracle):
    """The oracle's shading points of the tiny box, rounded to float32."""
    from oracle import bake as ob
    prim = ob.primary(tiny_oracle)
    pts, tri = ob.points_f32(prim)
    return pts, tri, prim
