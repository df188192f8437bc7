"""The library's host code under AddressSanitizer and UndefinedBehaviorSanitizer.

Builds a copy of the library whose host compilation carries the sanitizers
(device code as usual, not instrumented) into a temporary directory, links
the C program ``tests/host_sanitize/abi_check.c`` against it and runs it:
every workspace query on valid and invalid inputs, every compute entry point
on arguments it must reject before any device work, the status strings and
the phase profiler.  No GPU is needed; the sanitizers abort the program on
the first out-of-bounds access, use after free, leak or undefined behaviour.
"""

import os
import subprocess

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_abi_host_paths_under_sanitizers(tmp_path):
    from paper_1207_6365_amd import build

    exe = build.build_host_sanitized(str(tmp_path), os.path.join(ROOT, "tests", "host_sanitize", "abi_check.c"))
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0:halt_on_error=1",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    r = subprocess.run([exe], capture_output=True, text=True, timeout=300, env=env)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "abi host checks passed" in r.stdout
