import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (runs through the HIP C-ABI)")


@pytest.fixture(scope="session")
def oracle_mod():
    import oracle
    oracle.build(force=False)
    return oracle


@pytest.fixture(scope="session")
def synth_mod():
    import synth
    synth.build(force=False)
    return synth


def pytest_sessionfinish(session, exitstatus):
    # per-feature maxima of every GPU parity comparison of the session
    try:
        import gpu_util
    except ImportError:
        return
    path = gpu_util.write_record(ROOT)
    if path:
        print(f"\nper-feature parity errors: {path}")
