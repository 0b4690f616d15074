import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU")
    config.addinivalue_line("markers", "slow: long CPU test")


@pytest.fixture(scope="session")
def orc():
    """The CPU oracle module (built on first use)."""
    from oracle import oracle as O
    O.lib()
    return O


def oracle_einasto_extremal_spin(lam_e: float) -> float:
    """The extremal spin of the Einasto seed from the oracle (0 without one)."""
    from oracle import oracle as O
    from paper_2605_05635_amd import workloads as W
    r = O.extremal_spin(W.image(metric="einasto", spin=0.0, halo=(lam_e, 0.0)))
    return r[0] if r else 0.0


@pytest.fixture(scope="session")
def batch64():
    """The 64-image batch workload, drawn with the oracle's extremal spin."""
    from paper_2605_05635_amd import workloads as W
    return W.batch_64(oracle_einasto_extremal_spin)
