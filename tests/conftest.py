import json
import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (runs through the HIP library)")
    config.addinivalue_line("markers", "slow: CPU test that takes more than a few seconds")
    config.addinivalue_line("markers", "oracle_job(*names): needs the named background oracle runs "
                                       "(tests/oracle_jobs.py), started once collection is done")


def pytest_collection_finish(session):
    """Start the oracle runs that the selected tests need, in the background."""
    names = set()
    for item in session.items:
        for m in item.iter_markers("oracle_job"):
            names.update(m.args)
    if names:
        from tests import oracle_jobs

        oracle_jobs.start(names)


@pytest.fixture(scope="session")
def oracle_mod():
    import oracle

    oracle._load()
    return oracle


def load_golden(name):
    """A fixture file under tests/golden/ (values the paper prints, each file
    with its citation)."""
    with open(os.path.join(ROOT, "tests", "golden", name)) as f:
        return json.load(f)
