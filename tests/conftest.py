import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)
HERE = os.path.dirname(os.path.abspath(__file__))
if HERE not in sys.path:
    sys.path.insert(0, HERE)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (runs through the HIP library)")


@pytest.fixture(scope="session")
def oracle_mod():
    import oracle
    if not os.path.exists(os.path.join(ROOT, "oracle", "librei_oracle.so")):
        oracle.build()
    return oracle


@pytest.fixture(scope="session")
def golden():
    import json
    with open(os.path.join(HERE, "golden", "paper_examples.json"), encoding="utf-8") as f:
        return json.load(f)


@pytest.fixture(scope="session")
def rei():
    """The GPU library; GPU tests fail loudly if it is not built or no GPU is visible."""
    import paper_2305_18575_amd as rei_mod
    rei_mod.load_library()
    import torch
    assert torch.cuda.is_available(), "GPU test run without a visible GPU"
    return rei_mod
