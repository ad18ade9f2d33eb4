import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)
# the oracle's mutation test runs the pins against a modified copy of the
# oracle package placed in this directory
_ORACLE_ROOT = os.environ.get("FEDFEM_ORACLE_ROOT")
if _ORACLE_ROOT:
    sys.path.insert(0, _ORACLE_ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: long-running (full-size) case")
