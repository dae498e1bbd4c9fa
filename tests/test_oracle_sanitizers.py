"""The CPU oracle under the compiler's sanitizers (CPU only): AddressSanitizer
with UndefinedBehaviorSanitizer, and ThreadSanitizer over its pthread pool.
A small C driver (oracle_sanitize_driver.c) runs closed-form cases with caps,
enumeration, several thread counts and a time limit; it must exit 0 with no
sanitizer report."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
ORACLE = os.path.join(ROOT, "oracle", "oracle.c")
DRIVER = os.path.join(ROOT, "tests", "oracle_sanitize_driver.c")


@pytest.mark.parametrize("flags", [["-fsanitize=address,undefined", "-fno-sanitize-recover=undefined"],
                                   ["-fsanitize=thread"]], ids=["asan-ubsan", "tsan"])
def test_oracle_is_clean_under_sanitizers(tmp_path, flags):
    if shutil.which("gcc") is None:
        pytest.skip("gcc not available")
    exe = str(tmp_path / "driver")
    build = subprocess.run(["gcc", "-O1", "-g", "-std=c11", "-fno-omit-frame-pointer", *flags, "-pthread",
                            "-o", exe, ORACLE, DRIVER], capture_output=True, text=True)
    assert build.returncode == 0, build.stderr
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0", TSAN_OPTIONS="halt_on_error=1")
    run = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=300)
    report = run.stderr
    assert run.returncode == 0, report[-4000:]
    for marker in ("ERROR: AddressSanitizer", "runtime error:", "WARNING: ThreadSanitizer", "ERROR: LeakSanitizer"):
        assert marker not in report, report[-4000:]
    assert "sanitizer driver ok" in run.stdout
