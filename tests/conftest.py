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
def orc():
    import oracle

    oracle.lib()
    return oracle


def pytest_collection_finish(session):
    # the full-size parity tests compare with oracle runs of one to three
    # minutes each: start them in host threads as soon as those tests are
    # selected, so they overlap the other GPU tests
    if any(item.nodeid.startswith("tests/test_gpu_fullsize.py") and item.get_closest_marker("gpu")
           for item in session.items):
        try:
            import torch

            if not torch.cuda.is_available():
                return
        except Exception:
            return
        import fullsize_jobs

        fullsize_jobs.start()
