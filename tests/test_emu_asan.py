"""The emulated device code under bounds checking (CPU only).

tests/hipemu builds the library's kernels and engine for the host; with HIPEMU_ASAN=1 that
build runs under AddressSanitizer, and every buffer the engine carves from a workspace is
followed by a guard gap of LC_WS_GUARD bytes that no access may touch.  An access outside any
allocation, or past the declared size of a workspace buffer into its neighbour (which on the
GPU would go unnoticed or fault), then stops the child process with a report.  The whole
emulated parity suite (every round-0 form, input layout, label rule, MergeToLarge, explicit
orderings, recorded rounds, checkpoints, batch and server) and the smoke check run this way.
"""
import os
import subprocess
import sys

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)

hipemu = pytest.importorskip("hipemu")


def asan_env():
    try:
        return hipemu.asan_env()
    except (RuntimeError, OSError, subprocess.CalledProcessError) as e:
        pytest.skip("no AddressSanitizer runtime: %s" % e)


def run(args, timeout):
    proc = subprocess.run([sys.executable] + args, cwd=ROOT, env=asan_env(), stdout=subprocess.PIPE,
                          stderr=subprocess.STDOUT, text=True, timeout=timeout)
    assert "AddressSanitizer" not in proc.stdout, proc.stdout[-6000:]
    assert proc.returncode == 0, proc.stdout[-4000:]
    return proc.stdout


def test_guard_gaps_are_in_place():
    """The bounds-checking build really is one: its workspace plan is larger than the plain
    build's by the guard gaps, and the child process runs with the sanitizer loaded."""
    code = ("import hipemu, ctypes\n"
            "cc = hipemu.binding()\n"
            "assert 'asan' in cc.LIB_PATH, cc.LIB_PATH\n"
            "ctx = cc.cc_create(1000, 5000, cc.CC_EDGES_SOA_I32, 0x1000, 0x2000)\n"
            "print('WS', cc.cc_workspace_size(ctx))\n"
            "cc.cc_destroy(ctx)\n"
            "asan = ctypes.CDLL(None)\n"
            "print('ASAN', hasattr(asan, '__asan_poison_memory_region'))\n")
    out = run(["-c", "import sys; sys.path.insert(0, %r); exec(%r)" % (HERE, code)], 300)
    ws = int(out.split("WS ")[1].split()[0])
    assert "ASAN True" in out
    plain = hipemu.binding()
    ctx = plain.cc_create(1000, 5000, plain.CC_EDGES_SOA_I32, 0x1000, 0x2000)
    try:
        assert ws > plain.cc_workspace_size(ctx) + 10 * 256
    finally:
        plain.cc_destroy(ctx)


@pytest.mark.slow
def test_emulated_parity_suite_under_bounds_checking():
    """The whole emulated parity suite, in four worker processes (the first test of this file
    has built the library, so the workers do not race to build it)."""
    try:
        import xdist  # noqa: F401
        workers = ["-n", "4"]
    except ImportError:
        workers = []
    out = run(["-m", "pytest", "-q", "-x", "-p", "no:cacheprovider"] + workers +
              [os.path.join(HERE, "test_emu_parity.py")], 1200)
    assert " passed" in out and "failed" not in out and "skipped" not in out


def test_smoke_under_bounds_checking():
    out = run([os.path.join(HERE, "hipemu", "dryrun.py"), "smoke"], 300)
    assert "smoke ok" in out
