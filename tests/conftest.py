import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: long-running CPU check")


@pytest.fixture(autouse=True)
def _restore_launch_settings(request):
    """The library's launch shapes and steps per launch are process-wide:
    every GPU test gets them back as it found them, so that which kernel a
    test exercises does not depend on the tests run before it."""
    if request.node.get_closest_marker("gpu") is None:
        yield
        return
    import paper_2204_03380_amd as rtm
    snap = rtm.tuning_snapshot()
    try:
        yield
    finally:
        rtm.tuning_restore(snap)


@pytest.fixture
def progress(capsys):
    """Prints a line past pytest's output capture, at once: long tests mark
    the end of each step with it, so that a long run is visibly alive."""
    def say(msg):
        with capsys.disabled():
            print(f"  [{msg}]", flush=True)
    return say
