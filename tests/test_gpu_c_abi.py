"""The library from plain C: a C99 program that includes only
include/fhesnn.h and the HIP runtime runs keygen, encryption, key upload,
fs_pbs_lif on device buffers and decryption, and checks the error path
(tests/c_abi_roundtrip.c).  It runs as a child process."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

pytestmark = pytest.mark.gpu


def test_c_client_round_trip():
    from paper_2309_09025_amd import build as B
    if not os.path.exists(B.C_CLIENT):
        B.build_c_client()
    r = subprocess.run([B.C_CLIENT], capture_output=True, text=True, timeout=240)
    print(r.stdout, r.stderr)
    assert r.returncode == 0, r.stderr
    assert "c-abi: ok" in r.stdout

