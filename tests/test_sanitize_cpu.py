"""AddressSanitizer + UndefinedBehaviorSanitizer build of the host C and C++
sources (the oracle and the input generators), driven by
tests/sanitize/san_driver.cpp on small graphs of every family.  Errors are
not recoverable: any report aborts the driver, and the test fails."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SAN = ["-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer", "-g", "-O1"]


@pytest.mark.skipif(shutil.which("gcc") is None or shutil.which("g++") is None, reason="needs gcc and g++")
def test_oracle_and_generators_under_asan_ubsan(tmp_path):
    out = str(tmp_path)
    oracle_o = os.path.join(out, "oracle.o")
    gen_o = os.path.join(out, "graphgen.o")
    drv_o = os.path.join(out, "san_driver.o")
    exe = os.path.join(out, "san_driver")
    subprocess.run(["gcc", *SAN, "-std=c99", "-ffp-contract=off", "-c", os.path.join(ROOT, "oracle", "oracle.c"),
                    "-o", oracle_o], check=True)
    subprocess.run(["g++", *SAN, "-std=c++17", "-fopenmp", "-c", os.path.join(ROOT, "graphgen", "graphgen.cpp"),
                    "-o", gen_o], check=True)
    subprocess.run(["g++", *SAN, "-std=c++17", "-c", os.path.join(ROOT, "tests", "sanitize", "san_driver.cpp"),
                    "-o", drv_o], check=True)
    subprocess.run(["g++", *SAN, "-fopenmp", oracle_o, gen_o, drv_o, "-o", exe, "-lm"], check=True)
    # verify_asan_link_order=0: the run also works where the environment
    # preloads another library ahead of the sanitizer runtime
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=1:verify_asan_link_order=0",
               UBSAN_OPTIONS="print_stacktrace=1", OMP_NUM_THREADS="2")
    r = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=600)
    assert r.returncode == 0, r.stdout[-2000:] + r.stderr[-4000:]
    assert "sanitized run ok" in r.stdout
