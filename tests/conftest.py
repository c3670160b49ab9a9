import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (HIP device) and the built HIP library")


def pytest_collection_modifyitems(config, items):
    # GPU tests are selected with -m gpu; without a device they fail loudly
    # instead of silently passing on a fallback.
    pass


@pytest.fixture(scope="session")
def oracle_lib():
    import oracle

    oracle.build()
    return oracle


def pytest_terminal_summary(terminalreporter, exitstatus, config):
    # divergence totals of the edge-list parity comparisons run in this session
    import parity

    s = parity.summary()
    if s["comparisons"]:
        terminalreporter.write_line(
            "edge parity: {comparisons} comparisons, {edges_compared} edges compared, {divergences} divergences "
            "({near_tie_rows} near-tie rows in the oracle's traces)".format(**s))
