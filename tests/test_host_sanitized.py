"""The host side of the library under AddressSanitizer and
UndefinedBehaviorSanitizer (no GPU): the argument battery of
tests/host_battery.py against a build whose hand-written host code is
instrumented, in a child process with the sanitizer runtime preloaded.  Any
out-of-bounds access, use after free or undefined operation in the checks,
the plan and table code or the filter's sphere tables aborts the child."""
import os
import subprocess
import sys

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)


def _checked_library():
    sys.path.insert(0, ROOT)
    from paper_1412_3228_amd import build as plain
    from paper_1412_3228_amd import build_checked as checked

    if not os.path.exists(plain.LIB):
        pytest.skip("libhm.so not built")
    try:
        return checked.build_checked(), checked.runtime_path()
    except RuntimeError as e:  # plain objects or the sanitizer runtime missing
        pytest.skip(str(e))


def _dynamic_undefined(lib):
    r = subprocess.run(["nm", "-D", "--undefined-only", lib], capture_output=True, text=True)
    if r.returncode != 0:
        pytest.skip("nm unavailable")
    return r.stdout


def test_host_checks_clean_under_sanitizers():
    lib, runtime = _checked_library()
    # the host objects carry the instrumentation (its hooks resolve from the runtime)
    und = _dynamic_undefined(lib)
    assert "__asan_report_load" in und and "__ubsan_handle_" in und
    env = dict(os.environ)
    env.update(LD_PRELOAD=runtime, ASAN_OPTIONS="detect_leaks=0:halt_on_error=1",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")
    r = subprocess.run([sys.executable, os.path.join(HERE, "host_battery.py"), lib], capture_output=True, text=True,
                       env=env, timeout=600)
    out = r.stdout + r.stderr
    assert "Sanitizer" not in out, out[-4000:]
    assert r.returncode == 0, out[-4000:]
    assert "0 failures" in out
