"""The serving runtime's concurrency stress (tests/serve_stress.cpp) in its
host-sanitized build (tests/bin/serve_stress_asan, made by the package build):
AddressSanitizer watches the ticket lifecycle, the server thread, admission
and harvest for heap misuse while four threads submit and poll, a fifth polls
unknown tickets and the main thread runs blocking solves on the same context.
The kernels are built as usual; only host code is instrumented.  The driver
checks every served and blocking result against a residual computed on the
host, destroys the context with requests still pending, and must exit 0 with
no sanitizer report.  (ThreadSanitizer is not usable here: under it the HIP
runtime finds no device.)"""
import os
import subprocess
import sys

import pytest

pytestmark = pytest.mark.gpu

BIN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "bin")


def test_address_sanitized_serve_stress():
    exe = os.path.join(BIN, "serve_stress_asan")
    assert os.path.exists(exe), "build the package first (it builds %s)" % exe
    env = dict(os.environ)
    env["ASAN_OPTIONS"] = "detect_leaks=0:halt_on_error=1:abort_on_error=0"
    print("serve stress under AddressSanitizer", file=sys.stderr, flush=True)
    r = subprocess.run([exe], capture_output=True, text=True, timeout=300, env=env)
    print(r.stdout[-2000:], r.stderr[-4000:], file=sys.stderr, flush=True)
    assert "Sanitizer" not in r.stderr
    assert r.returncode == 0
    assert "ok" in r.stdout
