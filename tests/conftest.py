"""Shared pytest configuration: the ``gpu`` marker and repo-root import path."""
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (runs the HIP library)")
    config.addinivalue_line("markers", "slow: long-running CPU oracle test")


def pytest_terminal_summary(terminalreporter):
    try:
        from harness import OBSERVED
    except ImportError:
        return
    if not OBSERVED:
        return
    tr = terminalreporter
    tr.section("observed parity error maxima (value / bound)")
    for (test, q), (v, b) in sorted(OBSERVED.items()):
        tr.write_line(f"{test:90s} {q:7s} {v:9.2e} / {b:7.1e}  ({v / b:.1e} of the bound)")
