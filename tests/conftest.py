import json
import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

_ERRORS = []


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (runs through the HIP library)")
    config.addinivalue_line("markers", "slow: full-size parity case (seconds to a minute)")


@pytest.fixture
def errlog(request):
    """errlog(label, value, tol) records a measured error next to the
    tolerance it is held to and returns the value; the records of a session
    go to the JSON file named by TBS_ERRLOG (if set)."""
    def record(label, value, tol):
        _ERRORS.append({"test": request.node.nodeid, "label": label, "value": float(value), "tol": float(tol)})
        return float(value)
    return record


def pytest_sessionfinish(session, exitstatus):
    path = os.environ.get("TBS_ERRLOG")
    if path and _ERRORS:
        with open(path, "w") as fh:
            json.dump(_ERRORS, fh, indent=0)
