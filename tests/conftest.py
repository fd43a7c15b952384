import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (HIP device) to run")
    config.addinivalue_line("markers", "slow: long-running check")
    config.addinivalue_line("markers", "batch_inputs(*cfgs): uses the pairs of the batched "
                                       "workloads cfgs (drawn before any GPU call)")


def pytest_collection_finish(session):
    """Draw the pairs of the batched workloads that the selected tests use while
    the process has not touched the GPU yet (the host pool forks)."""
    cfgs = set()
    for item in session.items:
        for m in item.iter_markers("batch_inputs"):
            cfgs.update(m.args)
    if cfgs:
        from paper_1509_08197_amd import scenes
        scenes.prefetch(sorted(cfgs))


@pytest.fixture(scope="session")
def orc():
    from oracle import oracle
    oracle.build()
    return oracle
