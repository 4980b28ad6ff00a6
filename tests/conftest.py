import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (HIP device) and the built libburn.so")
    config.addinivalue_line("markers", "slow: longer CPU test")


@pytest.fixture(scope="session")
def oracle():
    from oracle import oracle as O
    if not os.path.exists(O.LIB):
        O.build()
    return O


def pytest_terminal_summary(terminalreporter, exitstatus, config):
    """One line per parity check of the run (cells, share of cells with the
    oracle's decisions, largest error in tolerance units among those cells
    and overall, error of the divergent cells against a tight reference), so
    that the figures stay in the tail of a quiet run's output."""
    from tests.parity import RECORD
    if not RECORD:
        return
    tr = terminalreporter
    tr.write_line("parity: test | cells | counters equal | max ewt (same counters) | max ewt "
                  "| divergent vs tight")
    for e in RECORD:
        name = e["test"].split("::")[-1][:48]
        tight = "-" if e["tight_err"] is None else f"{e['tight_err']:.2f}"
        tr.write_line(f"parity: {name} | {e['cells']} | {e['counters_equal']:.4f} | "
                      f"{e['max_ewt_same']:.2e} | {e['max_ewt']:.2e} | {tight}")
