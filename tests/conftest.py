import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: statistical test that runs for tens of seconds on the CPU")


@pytest.fixture(scope="session")
def oracle_lib():
    import oracle
    oracle.build(force=False)
    return oracle.load()


def pytest_terminal_summary(terminalreporter, exitstatus, config):
    """Largest differences against the oracle seen by the parity tests of
    this session, and the ties they accepted."""
    try:
        import parity_bars
    except ImportError:
        return
    if not parity_bars.OBSERVED and not parity_bars.TIES["count"]:
        return
    tr = terminalreporter
    tr.section("parity against the oracle: largest observed differences")
    for k in sorted(parity_bars.OBSERVED):
        tr.write_line(f"{k:60s} {parity_bars.OBSERVED[k]:.3e}")
    tr.write_line(f"tolerated ties (oracle margin < {parity_bars.TIE:g}): {parity_bars.TIES['count']}")
    for w in parity_bars.TIES["where"]:
        tr.write_line("  " + w)
