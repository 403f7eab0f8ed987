"""Test configuration: markers and import paths.

Markers:
  gpu  -- needs a HIP device (an MI355X); the CPU suite runs ``-m "not gpu"``.
  slow -- longer CPU checks (still part of the default CPU run).
"""
import os
import sys

_ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if _ROOT not in sys.path:
    sys.path.insert(0, _ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs a HIP device (MI355X)")
    config.addinivalue_line("markers", "slow: longer CPU check")
