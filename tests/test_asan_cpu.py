"""The C oracle and the library's host-only tuning-cache code built with the
host compiler's AddressSanitizer and UndefinedBehaviorSanitizer and run on
small inputs (CPU only; the GPU kernels are not part of this build)."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.mark.skipif(shutil.which("gcc") is None or shutil.which("g++") is None, reason="no host compiler")
def test_oracle_and_tune_cache_under_asan(tmp_path):
    san = ["-fsanitize=address,undefined", "-fno-omit-frame-pointer", "-g", "-O1"]
    objs = []
    for src, cc, std in ((os.path.join(ROOT, "oracle", "mrdft_oracle.c"), "gcc", "-std=c11"),
                         (os.path.join(ROOT, "tests", "asan", "asan_driver.c"), "gcc", "-std=c11"),
                         (os.path.join(ROOT, "paper_1507_02525_amd", "csrc", "mrdft_tune_cache.cpp"), "g++",
                          "-std=c++17")):
        obj = str(tmp_path / (os.path.basename(src) + ".o"))
        subprocess.run([cc, *san, std, "-D_DEFAULT_SOURCE", "-I" + os.path.join(ROOT, "include"), "-c", src, "-o", obj],
                       check=True, capture_output=True)
        objs.append(obj)
    exe = str(tmp_path / "asan_driver")
    subprocess.run(["g++", *san, *objs, "-o", exe, "-lm"], check=True, capture_output=True)
    # verify_asan_link_order=0: the sanitizer runtime need not be the first
    # library of the process (the environment may preload others)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=1:verify_asan_link_order=0",
               UBSAN_OPTIONS="halt_on_error=1")
    r = subprocess.run([exe, str(tmp_path)], capture_output=True, text=True, env=env, timeout=600)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "asan driver clean" in r.stdout
    assert "ERROR: AddressSanitizer" not in r.stderr and "runtime error" not in r.stderr, r.stderr
