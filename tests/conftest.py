import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: statistical or exhaustive checks taking tens of seconds")


@pytest.fixture(scope="session")
def orc():
    """The CPU oracle, built if its shared object is missing."""
    import oracle
    oracle.oracle._load()
    return oracle


def seed_block(config_id: int, p_index: int, n: int, start: int = 0):
    """Seeds (config_id << 40) | (p_index << 32) | i, the workload seed recipe."""
    from paper_2506_03266_amd.workloads import seeds
    return seeds(config_id, p_index, n, start)
