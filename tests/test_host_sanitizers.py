"""Host sanitizer tier: the C++ runtime (argument validation, planning, the
serving loop's host side) built with AddressSanitizer and
UndefinedBehaviorSanitizer (libgmrf_san.so, host code only), and the
host-side C-ABI tests run against it in a child process with the sanitizer
runtime preloaded.  The child must pass with no sanitizer report."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_host_runtime_under_address_and_undefined_behavior_sanitizers(built_library, tmp_path):
    sys.path.insert(0, ROOT)
    from paper_1606_00980_amd import build
    lib = build.build_sanitized(verbose=False, out=str(tmp_path / "libgmrf_san.so"))
    syms = subprocess.run(["nm", "-D", lib], capture_output=True, text=True).stdout
    assert "__asan_" in syms and "__ubsan_handle_" in syms, "the host code is not instrumented"
    env = dict(os.environ)
    env.update({
        "GMRF_LIB": lib,
        "LD_PRELOAD": build.sanitizer_runtime(),
        # Python itself is not instrumented: its allocations are not checked
        # for leaks; any other report ends the child with an error.
        "ASAN_OPTIONS": "detect_leaks=0:abort_on_error=1:halt_on_error=1",
        "UBSAN_OPTIONS": "halt_on_error=1:print_stacktrace=1",
    })
    res = subprocess.run([sys.executable, "-m", "pytest", "-q", "-p", "no:cacheprovider",
                          os.path.join(ROOT, "tests", "test_capi.py"),
                          os.path.join(ROOT, "tests", "test_host_validation.py")],
                         cwd=ROOT, env=env, capture_output=True, text=True, timeout=600)
    out = res.stdout + res.stderr
    assert res.returncode == 0, out[-4000:]
    assert "AddressSanitizer" not in out and "runtime error:" not in out, out[-4000:]
    assert " passed" in out
