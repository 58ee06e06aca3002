import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU")
    config.addinivalue_line("markers", "slow: long CPU-only oracle pin")


@pytest.fixture(autouse=True, scope="session")
def _torch_threads():
    # The oracle issues many small tensor ops; one thread per process avoids
    # OpenMP spin overhead dominating them.
    import torch
    torch.set_num_threads(int(os.environ.get("ORACLE_THREADS", "1")))
    yield
