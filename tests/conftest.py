import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the HIP library")
    config.addinivalue_line("markers", "slow: longer CPU test")


@pytest.fixture(scope="session")
def orc():
    from oracle import oracle
    if not os.path.exists(oracle.LIB):
        oracle.build()
    return oracle


@pytest.fixture(scope="session")
def gpu():
    """(torch, pd, Context) on cuda:0.  Fails loudly without a GPU or library."""
    import torch
    assert torch.cuda.is_available(), "GPU tests need a ROCm GPU"
    from paper_1806_06917_amd import pd
    ctx = pd.Context(0)
    yield torch, pd, ctx
    torch.cuda.synchronize()
    ctx.close()


def say(*args):
    """Progress line naming the case, flushed before each GPU step."""
    print("[case]", *args, flush=True)
