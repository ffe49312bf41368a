"""Host-side AddressSanitizer / UndefinedBehaviorSanitizer run of the library's host code.

`__graft_entry__.build()` compiles a copy of libcola whose host code is instrumented (device code
as usual) and the C driver tests/native/abi_sanitize.cpp, which calls every entry point through the
C ABI on small operators and checks the FP64 product against a host product written from the
definition.  A heap overflow, use after free, double free or undefined behaviour anywhere in the
host code of those calls stops the driver with a sanitizer report and a non-zero status.  Leak
checking is off: the HIP runtime keeps allocations until exit by design.
"""
import os
import subprocess

import pytest

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
DRIVER = os.path.join(ROOT, "tests", "native", "_asan", "abi_sanitize")


def test_every_entry_point_under_host_sanitizers():
    if not os.path.exists(DRIVER):
        pytest.fail(f"{DRIVER} is missing: __graft_entry__.build() builds it")
    env = dict(os.environ)
    env["ASAN_OPTIONS"] = ("detect_leaks=0:halt_on_error=1:verify_asan_link_order=0:protect_shadow_gap=0")
    env["UBSAN_OPTIONS"] = "print_stacktrace=1:halt_on_error=1"
    print("running", DRIVER, flush=True)
    r = subprocess.run([DRIVER], env=env, capture_output=True, text=True, timeout=300)
    out = r.stdout + r.stderr
    print(r.stdout.strip().splitlines()[-1] if r.stdout.strip() else "(no output)", flush=True)
    assert r.returncode == 0, out[-6000:]
    assert "all checks passed" in r.stdout, out[-6000:]
    assert "runtime error" not in out and "AddressSanitizer" not in out, out[-6000:]
