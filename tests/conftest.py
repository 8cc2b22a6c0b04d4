import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: CPU test that takes more than a few seconds")


@pytest.fixture(scope="session")
def orc():
    from oracle import oracle
    oracle.build()
    return oracle


def pytest_terminal_summary(terminalreporter):
    """Mismatch rates of the screened (tiled) comparisons against the oracle."""
    mod = sys.modules.get("tests.gpu_util")
    rows = getattr(mod, "MISMATCHES", None) if mod else None
    if not rows:
        return
    bad = sum(r[1] for r in rows)
    tot = sum(r[2] for r in rows)
    terminalreporter.write_line(f"screened comparisons: {len(rows)}, rows differing from the oracle "
                                f"{bad}/{tot} ({bad / max(tot, 1):.4%}); worst:")
    for tag, b, t in sorted(rows, key=lambda r: -r[1] / max(r[2], 1))[:8]:
        terminalreporter.write_line(f"  {tag}: {b}/{t}")
