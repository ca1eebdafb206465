"""The oracle built with AddressSanitizer and UndefinedBehaviorSanitizer (gcc,
host only): a driver calls every oracle function on small lattices, boundary
sizes included; any invalid access or undefined arithmetic aborts the run."""
import os
import subprocess
import tempfile

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_oracle_under_asan_and_ubsan():
    with tempfile.TemporaryDirectory() as td:
        exe = os.path.join(td, "oracle_sanitized")
        subprocess.check_call(["gcc", "-std=c11", "-O1", "-g", "-fno-omit-frame-pointer",
                               "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
                               "-I", os.path.join(ROOT, "oracle"), "-o", exe,
                               os.path.join(ROOT, "oracle", "oracle.c"),
                               os.path.join(ROOT, "tests", "oracle_sanitize_main.c"), "-lm"])
        # (the environment is passed on unchanged apart from the sanitizer options;
        # verify_asan_link_order=0 lets the run proceed when another library is preloaded)
        env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0:verify_asan_link_order=0",
                   UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
        r = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=300)
    assert r.returncode == 0, r.stdout[-3000:] + r.stderr[-3000:]
    assert "sanitized oracle run complete" in r.stdout
