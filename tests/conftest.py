import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: long-running GPU parity case")


@pytest.fixture(scope="session", autouse=True)
def _oracle_built():
    import oracle
    if not os.path.exists(os.path.join(ROOT, "oracle", "liboracle.so")):
        oracle.build()
    yield


def pytest_runtest_logstart(nodeid, location):
    # Name the case on stderr before it runs, so a run that ends abruptly
    # still shows which GPU case was executing.
    sys.stderr.write(f"\n[start] {nodeid}\n")
    sys.stderr.flush()


@pytest.fixture(scope="session")
def gpu():
    """Skip unless a GPU and the built HIP library are present; the library
    must load (no fallback exists)."""
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1903_05575_amd as q
    q.lib()
    return torch.device("cuda:0")
