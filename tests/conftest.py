import json
import os
import sys

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs a real MI355X (runs through the C ABI on HIP)")
    config.addinivalue_line("markers", "slow: larger CPU oracle runs")


@pytest.fixture(autouse=True)
def leaf_start(monkeypatch):
    """Plans start the sweep at the leaves (Section 2.2, step 2) unless a test
    asks for another start level; the start-level tests set it themselves."""
    monkeypatch.setenv("BFSFT_START_LEVEL", "0")


@pytest.fixture(scope="session")
def oracle_mod():
    import oracle
    oracle.build(force=False)
    return oracle


def rel_l2(a, b):
    a = np.asarray(a)
    b = np.asarray(b)
    den = np.linalg.norm(b)
    return float(np.linalg.norm(a - b) / (den if den > 0 else 1.0))


def within_measured(err, measured, name, factor=3.0):
    """Assert err <= factor x the deviation measured on the GPU for this case
    (reduced-precision paths against the oracle); with BFSFT_ERR_LOG set,
    also append the case and its error to that file (for refreshing the
    measured values)."""
    path = os.environ.get("BFSFT_ERR_LOG")
    if path:
        with open(path, "a") as fh:
            fh.write(json.dumps({"case": name, "err": err, "measured": measured}) + "\n")
    assert err <= factor * measured, f"{name}: {err:.3e} > {factor} x measured {measured:.3e}"
