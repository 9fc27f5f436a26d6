"""The oracle under host sanitizers: AddressSanitizer with
UndefinedBehaviorSanitizer, and ThreadSanitizer for the threaded trace
(private Gamma per thread, shared source counter under a mutex).  The test program
(oracle/sanitize_main.c) runs every oracle entry point on small inputs and
checks each trace's photon budget; any sanitizer report fails the run."""
import os
import subprocess

import pytest

from oracle import build


@pytest.mark.parametrize("kind", ["address", "thread"])
def test_oracle_clean_under_sanitizer(tmp_path, kind):
    exe = str(tmp_path / f"oracle_{kind}")
    try:
        build.build_sanitized(kind, exe)
    except subprocess.CalledProcessError as e:  # no sanitizer runtime for this compiler
        pytest.skip(f"gcc cannot build with -fsanitize for {kind}: {e.stderr[-300:]}")
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:halt_on_error=1",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1",
               TSAN_OPTIONS="halt_on_error=1")
    p = subprocess.run([exe], capture_output=True, text=True, timeout=300, env=env)
    assert p.returncode == 0 and "ok" in p.stdout, p.stderr[-3000:]
