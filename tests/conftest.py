import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

_REPORTS = []


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")


@pytest.fixture(scope="session")
def fp64_log():
    """Collects binary64 cross-check reports (not gates); printed at the end of
    the session, also under -q."""
    return _REPORTS


def pytest_terminal_summary(terminalreporter):
    if _REPORTS:
        terminalreporter.section("binary64 cross-check (report, not a gate)")
        for line in _REPORTS:
            terminalreporter.write_line(line)
