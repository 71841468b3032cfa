"""The CPU oracle built with AddressSanitizer and UndefinedBehaviorSanitizer
(gcc, serial) and run over every entry point on small and degenerate grids
(tests/oracle_sanitize_driver.c): no access outside the documented array
sizes and no undefined operation."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_oracle_is_clean_under_asan_and_ubsan(tmp_path):
    if shutil.which("gcc") is None:
        pytest.skip("gcc is not available")
    exe = str(tmp_path / "oracle_sanitized")
    cmd = ["gcc", "-std=c11", "-O1", "-g", "-ffp-contract=off", "-fno-omit-frame-pointer",
           "-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-Wall", "-Wno-unknown-pragmas",
           "-I", os.path.join(ROOT, "oracle"), "-o", exe,
           os.path.join(ROOT, "tests", "oracle_sanitize_driver.c"), os.path.join(ROOT, "oracle", "mpdata_ref.c"),
           "-lm"]
    subprocess.run(cmd, check=True)
    # the ASan runtime is linked into the executable; other preloaded
    # libraries of the environment may come before it
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:verify_asan_link_order=0",
               UBSAN_OPTIONS="print_stacktrace=1")
    r = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=600)
    assert r.returncode == 0, r.stderr[-4000:]
    assert "all calls clean" in r.stdout
