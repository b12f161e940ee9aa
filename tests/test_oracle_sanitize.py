"""The oracle's C code under AddressSanitizer and UndefinedBehaviorSanitizer
(CPU): tests/native/oracle_sanitize.c drives every entry point on random
small graphs; a memory error, a leak or undefined behaviour aborts it."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)


@pytest.mark.skipif(shutil.which("gcc") is None, reason="needs gcc")
def test_oracle_clean_under_asan_and_ubsan(tmp_path):
    exe = str(tmp_path / "oracle_sanitize")
    subprocess.check_call(["gcc", "-O1", "-g", "-std=c11", "-pthread",
                           "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
                           "-fno-omit-frame-pointer",
                           os.path.join(ROOT, "oracle", "oracle.c"),
                           os.path.join(HERE, "native", "oracle_sanitize.c"), "-o", exe])
    # verify_asan_link_order=0: the environment may preload a library of its
    # own ahead of the sanitizer runtime
    env = dict(os.environ,
               ASAN_OPTIONS="detect_leaks=1:abort_on_error=1:verify_asan_link_order=0",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    r = subprocess.run([exe], env=env, capture_output=True, text=True, timeout=300)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "300 graphs clean" in r.stdout
