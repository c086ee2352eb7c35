import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")


@pytest.fixture(scope="session", autouse=True)
def _oracle_built():
    from oracle import build
    if not os.path.exists(build.LIB) or os.path.getmtime(build.LIB) < os.path.getmtime(build.SRC):
        build.build()


def pytest_terminal_summary(terminalreporter, exitstatus, config):
    """Flagged-pixel fractions of every image comparison against the oracle
    (pixels whose decisions sit within the oracle's threshold windows)."""
    try:
        from tests.gpu_helpers import IMAGE_RECORDS
    except Exception:
        return
    if not IMAGE_RECORDS:
        return
    tr = terminalreporter
    tr.write_sep("-", "image parity: flagged pixels per comparison")
    worst = 0.0
    for test, label, npx, nflag, err, err_flag in IMAGE_RECORDS:
        frac = nflag / max(npx, 1)
        worst = max(worst, frac)
        tr.write_line(f"{frac:9.2e} flagged ({nflag:6d} of {npx:8d}), max err {err:.2e} clean / {err_flag:.2e} "
                      f"flagged  {test} {label}")
    tr.write_line(f"largest flagged fraction: {worst:.3e}")
