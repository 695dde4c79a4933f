"""The host ABI tests once more, against a build of the C ABI layer
(mlp_api.cpp) with AddressSanitizer: every argument check, status string
and error message path runs under the sanitizer, which aborts the run on an
out-of-bounds access, a use after free or a double free in host code.  No
GPU is used (the ABI tests make no compute call)."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_abi_tests_pass_under_host_address_sanitizer():
    from paper_1908_07847_amd import build
    lib = build.build_asan()
    env = dict(os.environ, MLP_LIBRARY=lib, LD_PRELOAD=build.asan_runtime(),
               ASAN_OPTIONS="detect_leaks=0:abort_on_error=1")
    r = subprocess.run([sys.executable, "-m", "pytest", "-q", "-x", "-p", "no:cacheprovider", "-m", "not gpu",
                        os.path.join(ROOT, "tests", "test_abi.py")], cwd=ROOT, env=env, capture_output=True,
                       text=True, timeout=600)
    assert r.returncode == 0, r.stdout[-3000:] + r.stderr[-3000:]
    assert "passed" in r.stdout
    # the sanitized copy was the one loaded
    probe = subprocess.run([sys.executable, "-c", "from paper_1908_07847_amd import _lib; print(_lib.LIB_PATH)"],
                           cwd=ROOT, env=env, capture_output=True, text=True, timeout=300)
    assert probe.stdout.strip() == lib, probe.stdout + probe.stderr
