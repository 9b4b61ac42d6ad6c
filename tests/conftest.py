import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (runs the HIP path)")
    config.addinivalue_line("markers", "slow: longer CPU test")


@pytest.fixture(scope="session")
def orc():
    import oracle
    oracle.lib()
    return oracle


@pytest.fixture(scope="session")
def gt():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2608_25830_amd import gtmp
    return gtmp


def pytest_terminal_summary(terminalreporter):
    """Figures the parity tests record (excused edges, compared indices...),
    printed after the run so that they appear in a quiet run's output."""
    from tests import parity
    if parity.NOTES:
        terminalreporter.section("parity figures")
        for line in parity.NOTES:
            terminalreporter.write_line(line)
