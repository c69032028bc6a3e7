import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: CPU test that takes more than a few seconds")


@pytest.fixture(scope="session")
def gpu():
    """(torch, dmlmc module, Context) on cuda:0; the HIP library must be built."""
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2211_15383_amd import dmlmc

    ctx = dmlmc.Context(0)
    yield torch, dmlmc, ctx
    torch.cuda.synchronize()
