import os
import sys
from pathlib import Path

import pytest

ROOT = Path(__file__).resolve().parent.parent
if str(ROOT) not in sys.path:
    sys.path.insert(0, str(ROOT))
HERE = Path(__file__).resolve().parent
if str(HERE) not in sys.path:
    sys.path.insert(0, str(HERE))


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: long CPU-side oracle runs")


@pytest.fixture(scope="session")
def orc():
    import oracle
    oracle.lib()
    return oracle


@pytest.fixture(autouse=True)
def _parity_record_test_id(request):
    """Tags the parity records (parity_checks.record) with the running test."""
    import parity_checks
    parity_checks.CURRENT_TEST["id"] = request.node.nodeid
    yield
    parity_checks.CURRENT_TEST["id"] = None


def pytest_sessionfinish(session, exitstatus):
    import parity_checks
    path = parity_checks.write_records(ROOT)
    if path is not None:
        print(f"\nparity records: {len(parity_checks.RECORDS)} appended to {path}", flush=True)
