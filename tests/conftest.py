import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)
HERE = os.path.dirname(os.path.abspath(__file__))
if HERE not in sys.path:
    sys.path.insert(0, HERE)
# The emulated device code (tests/hipemu) runs the workgroups of every launch on two host
# threads at once unless told otherwise: workgroups then really race on global memory, and the
# emulated suites finish sooner.
os.environ.setdefault("HIPEMU_THREADS", "2")


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: long-running test (about a minute or more)")
