"""The oracle's C code under AddressSanitizer and UndefinedBehaviorSanitizer (host only).

`oracle_sanitize_driver.c` calls every C routine of the oracle on a 6x4x4x6 lattice and
checks two identities of the results; built with clang's sanitizers (abort on the first
report, leak check on), it must run clean. clang, because gcc 11's AddressSanitizer does
not check the complex-typed loads and stores that the oracle's link and spinor arithmetic
is made of (an overrun planted there goes unreported), while clang's does.
"""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)


CLANG = next((c for c in ("/opt/rocm/llvm/bin/clang", shutil.which("clang") or "")
              if c and os.path.exists(c)), None)


@pytest.mark.skipif(CLANG is None, reason="needs clang")
def test_oracle_c_under_sanitizers(tmp_path):
    exe = str(tmp_path / "oracle_sanitized")
    build = subprocess.run(
        [CLANG, "-std=gnu99", "-O1", "-g", "-fno-omit-frame-pointer", "-fopenmp",
         "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
         os.path.join(HERE, "oracle_sanitize_driver.c"), os.path.join(ROOT, "oracle", "oracle.c"),
         "-o", exe, "-lm"],
        capture_output=True, text=True)
    if build.returncode != 0 and "sanitize" in build.stderr and "cannot find" in build.stderr:
        pytest.skip("sanitizer runtimes not installed")
    assert build.returncode == 0, build.stderr
    # the OpenMP runtime keeps one allocation of its own to the end: not the oracle's
    supp = tmp_path / "lsan.supp"
    supp.write_text("leak:libomp.so\n")
    env = dict(os.environ, OMP_NUM_THREADS="2", ASAN_OPTIONS="detect_leaks=1:abort_on_error=0",
               LSAN_OPTIONS="suppressions=%s" % supp, UBSAN_OPTIONS="print_stacktrace=1")
    run = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=300)
    if run.returncode != 0 and "does not come first in initial library list" in run.stderr:
        pytest.skip("the sanitizer runtime cannot load first in this environment")
    assert run.returncode == 0, run.stdout + run.stderr
    assert run.stdout.startswith("ok"), run.stdout
