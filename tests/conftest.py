import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: takes more than a few seconds on the CPU")


def golden(name):
    """Parse a tests/golden fixture into a list of (key, [values]) records."""
    path = os.path.join(ROOT, "tests", "golden", name)
    recs = []
    with open(path) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            k, v = line.split(":", 1)
            recs.append((k.strip(), [int(t) for t in v.split()]))
    return recs


@pytest.fixture(scope="session")
def gpu_lib():
    """The built HIP library on a machine with a GPU; skip elsewhere."""
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1609_01010_amd as pm

    pm.lib()  # raises loudly if the library is missing
    return pm
