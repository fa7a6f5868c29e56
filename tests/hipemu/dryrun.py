"""Run bench.py or __graft_entry__.smoke() end to end on the CPU -- TEST INFRASTRUCTURE ONLY.

    python tests/hipemu/dryrun.py bench <bench.py arguments>
    python tests/hipemu/dryrun.py smoke
    python tests/hipemu/dryrun.py pytest <pytest arguments>

The process installs the numpy stand-in for torch (faketorch.py) and binds the package's
ctypes module to the emulated library before anything imports them, so the benchmark's and the
smoke check's own Python code runs unchanged.  Its figures are the emulator's, not a GPU's.
"""
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
TESTS = os.path.dirname(HERE)
ROOT = os.path.dirname(TESTS)
for p in (ROOT, TESTS):
    if p not in sys.path:
        sys.path.insert(0, p)

import hipemu  # noqa: E402
from hipemu import faketorch  # noqa: E402

sys.modules["torch"] = faketorch
sys.modules["paper_1807_10727_amd._cc"] = hipemu.binding()


def main():
    what = sys.argv[1]
    if what == "bench":
        import bench
        sys.argv = ["bench.py"] + sys.argv[2:]
        bench.main()
    elif what == "smoke":
        import __graft_entry__
        __graft_entry__.smoke()
    elif what == "pytest":
        # GPU tests' own logic against the emulated library (toy sizes only: they are slow here)
        import pytest
        raise SystemExit(pytest.main(sys.argv[2:]))
    else:
        raise SystemExit("usage: dryrun.py bench|smoke [arguments]")


if __name__ == "__main__":
    main()
