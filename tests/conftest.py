import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs a GPU (MI355X) and the built HIP library")


@pytest.fixture(scope="session")
def hfcr_ctx():
    import torch
    import paper_1409_2081_amd as hf
    if not torch.cuda.is_available():
        pytest.fail("gpu test run without a visible GPU")
    ctx = hf.Context(0)
    yield ctx
    ctx.close()


def pytest_runtest_logstart(nodeid, location):
    # name every GPU case on its own line before it runs, so that a run that
    # ends abruptly still shows which case was on the device
    if "gpu" in nodeid:
        sys.__stderr__.write(f"[start] {nodeid}\n")
        sys.__stderr__.flush()
