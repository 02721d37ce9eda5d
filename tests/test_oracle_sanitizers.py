"""The oracle under host sanitizers: `oracle/sanitize_check.cpp` runs every
oracle entry point (Algorithm 1 from the root, ParMCE under every rank with
one and two threads, brute force, the incremental and decremental steps) on
small random graphs and cross-checks their answers, built once with
AddressSanitizer + UndefinedBehaviorSanitizer and once with ThreadSanitizer
(the threaded ParMCE and state creation).  CPU only."""

import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = [os.path.join(ROOT, "oracle", "mce_oracle.cpp"), os.path.join(ROOT, "oracle", "sanitize_check.cpp")]
ENV = {"ASAN_OPTIONS": "detect_leaks=1:abort_on_error=1", "UBSAN_OPTIONS": "halt_on_error=1:print_stacktrace=1",
       "TSAN_OPTIONS": "halt_on_error=1"}


@pytest.mark.parametrize("sanitizers,args", [("address,undefined", []), ("thread", ["quick"])],
                         ids=["asan-ubsan", "tsan"])
def test_oracle_under_sanitizers(sanitizers, args):
    if shutil.which("g++") is None:
        pytest.skip("no g++")
    out = os.path.join(ROOT, "oracle", "_build", "sanitize_check_" + sanitizers.split(",")[0])
    os.makedirs(os.path.dirname(out), exist_ok=True)
    flags = ["-fsanitize=" + sanitizers] + ([] if sanitizers == "thread" else ["-fno-omit-frame-pointer"])
    subprocess.check_call(["g++", "-std=c++17", "-O1", "-g", *flags, "-pthread", *SRC, "-o", out])
    r = subprocess.run([out, *args], env=dict(os.environ, **ENV), capture_output=True, text=True, timeout=600)
    assert r.returncode == 0, (r.stdout + r.stderr)[-4000:]
    assert "sanitize_check ok" in r.stdout
