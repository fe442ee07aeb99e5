import json
import os
import sys
from pathlib import Path

import numpy as np
import pytest

ROOT = Path(__file__).resolve().parent.parent
if str(ROOT) not in sys.path:
    sys.path.insert(0, str(ROOT))

PARAMS_PATH = ROOT / "paper_2505_23618_amd" / "params" / "adjust_params.json"


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: long-running CPU test")


@pytest.fixture(scope="session")
def params():
    with open(PARAMS_PATH) as f:
        return {e["name"]: e for e in json.load(f)["entries"]}


@pytest.fixture(scope="session")
def rng():
    return np.random.Generator(np.random.PCG64(12345))
