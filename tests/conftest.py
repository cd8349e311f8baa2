import os
import sys

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (runs through the HIP C-ABI library)")
    config.addinivalue_line("markers", "slow: longer CPU test")


@pytest.fixture(scope="session")
def tiny_pair():
    from synth import make_workload_pair, params_for
    return make_workload_pair("tiny-64x48"), params_for("tiny-64x48")


@pytest.fixture(scope="session")
def tiny_oracle(tiny_pair):
    from oracle import Oracle
    pair, prm = tiny_pair
    return Oracle(prm, pair.left, pair.right)




@pytest.fixture
def rng():
    return np.random.default_rng(1234)
