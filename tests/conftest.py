import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (HIP device) and the built library")
    config.addinivalue_line("markers", "slow: long CPU-only physics pin")


@pytest.fixture(scope="session")
def oracle_lib():
    from oracle import oracle
    oracle.build(force=not os.path.exists(oracle.LIB_PATH))
    return oracle


# Measured parity maxima, written at the end of the session to the file named
# by FDLBM_PARITY_RECORD (JSON: test id -> field -> max error), so that the
# figures behind the tolerances are kept, not only the pass/fail outcome.
PARITY_RECORD = {}


@pytest.fixture
def parity_record(request):
    def rec(errs, tol=None):
        entry = PARITY_RECORD.setdefault(request.node.nodeid, {})
        for k, v in errs.items():
            entry[k] = float(v)
        if tol is not None:
            entry.setdefault("_tol", float(tol))
    return rec


def pytest_sessionfinish(session, exitstatus):
    path = os.environ.get("FDLBM_PARITY_RECORD")
    if path and PARITY_RECORD:
        import json
        os.makedirs(os.path.dirname(os.path.abspath(path)), exist_ok=True)
        with open(path, "w") as fh:
            json.dump(PARITY_RECORD, fh, indent=1, sort_keys=True)
