"""The library's host-side client code (key generation, encryption,
decryption, program-function tables) built with g++ under AddressSanitizer
and UndefinedBehaviorSanitizer and driven through both parameter sets and
its error paths.  CPU only: the GPU code is not part of this compilation."""
import os
import shutil
import subprocess
import tempfile

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(ROOT, "paper_2309_09025_amd", "csrc")


@pytest.mark.skipif(shutil.which("g++") is None, reason="needs g++")
def test_host_code_is_clean_under_asan_and_ubsan():
    with tempfile.TemporaryDirectory(prefix="fs_asan_") as tmp:
        exe = os.path.join(tmp, "host_sanitize")
        cmd = ["g++", "-std=c++17", "-O1", "-g", "-fno-omit-frame-pointer",
               "-fsanitize=address,undefined", "-fno-sanitize-recover=undefined",
               "-I", os.path.join(ROOT, "include"), "-I", CSRC,
               os.path.join(HERE, "host_sanitize_main.cpp"), os.path.join(CSRC, "host_keys.cpp"),
               "-o", exe, "-lpthread"]
        subprocess.run(cmd, check=True, capture_output=True, text=True)
        # the environment may preload a library ahead of the ASan runtime;
        # ASan's own option accepts that instead of refusing to start
        env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:verify_asan_link_order=0",
                   UBSAN_OPTIONS="print_stacktrace=1")
        r = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=600)
        assert r.returncode == 0, r.stdout + r.stderr
        assert "host sanitizer run: ok" in r.stdout
        assert "runtime error" not in r.stderr and "ERROR: AddressSanitizer" not in r.stderr
