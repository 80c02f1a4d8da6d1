import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU")
    config.addinivalue_line("markers", "slow: long-running CPU test")


@pytest.fixture(scope="session")
def oracle_lib():
    from oracle import build
    if not os.path.exists(build.LIB):
        build.build()
    return build.LIB


# Tests whose measurements are listed last (closest to the end of the output):
# parity at the configurations' full sizes and stated step counts.
KEY_TESTS = ("test_long_horizon_gpu.py", "test_full_size", "test_drude_dipole_32")


def pytest_terminal_summary(terminalreporter):
    """List the errors the GPU tests measured (their say() lines), one per
    line under the test that measured them; the full-size and long-horizon
    parity tests last."""
    mod = sys.modules.get("tests.gpu_util")
    rows = getattr(mod, "MEASURED", None) if mod else None
    if not rows:
        return
    terminalreporter.section("measured errors (GPU vs oracle)")
    key = [r for r in rows if any(k in r[0] for k in KEY_TESTS)]
    last = None
    for test, msg in [r for r in rows if r not in key] + key:
        if test != last:
            terminalreporter.write_line(test or "(outside a test)")
            last = test
        terminalreporter.write_line("    " + msg)
