import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: long-running CPU test")


@pytest.fixture(scope="session")
def orc():
    import oracle
    oracle.build()
    return oracle


def pytest_terminal_summary(terminalreporter, exitstatus, config):
    # the measured parity figures of every GPU check (R20 per conserved
    # variable, difference over sigma, fraction of the bar used)
    try:
        import parity
    except ImportError:
        return
    lines = parity.summary_lines()
    if lines:
        terminalreporter.section("parity against the oracle")
        for ln in lines:
            terminalreporter.write_line(ln)
